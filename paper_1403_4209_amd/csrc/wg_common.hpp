// Internal declarations shared by the libwgrid translation units (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wgrid.h"

namespace wg {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxS = WG_MAX_SUPPORT;
constexpr int kSlots = 7;          // most cell classes per lane in the gridder (120 VGPRs; 8 measure alike with 5 spilled)
constexpr int kSlotsNarrow = 6;    // the same with BF16/FP16 tables (measured faster there)
constexpr int kDegridSlots = 7;    // the same for the degridder (FP32 tables: 3.06 ms, 3.14 with 5)
constexpr int kDegridSlotsNarrow = 6;  // with BF16/FP16 tables (2.51 ms, 2.57 with 5)
constexpr int kSlotsPol2 = 5;      // gridder with two polarisations (any table type)
constexpr int kSlotsPol4 = 3;      // gridder with four polarisations (2 to 5 measured alike)
constexpr int kDegridSlotsPol2 = 5;  // degridder with two polarisations (4.33 vs 4.61 ms with 4)
constexpr int kDegridSlotsPol4 = 3;  // with four (9.55 vs 11.65 ms with 2, 20.8 with 1)

// ---------------------------------------------------------------------------------------
// Plan layout (int32 words). Items are local chunks (first run, one past last run) of
// consecutive runs of one segment that share a support; they are grouped by support, the
// largest support first.
//   [kPlanCount + S]   items with support S              (S = 1..63, odd)
//   [kPlanOff + S]     first item slot of support S       (kPlanOff + 64 = total)
//   [kPlanCur + S]     append cursor of support S
//   [kPlanQueueDegrid] degridder work-list counter and exit count (2 words), zero between launches
//   [kPlanQueueGrid]   the same for the gridder's counter walk (large grids)
//   [kPlanGrids]       number of grids the runs address (channels, w-planes or 1)
//   [kPlanHdr ...]     items: 2 * capacity words
//   then               runs per segment, scanned in place: n_seg + 1 words
//   then               scan tile totals: n_tiles + 1 words
// ---------------------------------------------------------------------------------------
constexpr int kPlanCount = 0;
constexpr int kPlanOff = 64;
constexpr int kPlanCur = 129;
constexpr int kPlanQueueDegrid = 200;
constexpr int kPlanQueueGrid = 208;
constexpr int kPlanGrids = 240;  // read by every batch: kept off the work counter's cache line
constexpr int kPlanHdr = 256;
constexpr int kScanTile = 4096;

inline int64_t plan_items_at() { return kPlanHdr; }
inline int64_t plan_segcnt_at(int64_t capacity) { return kPlanHdr + 2 * capacity; }
inline int64_t plan_tiles_at(int64_t capacity, int64_t n_seg) { return plan_segcnt_at(capacity) + n_seg + 1; }
inline int64_t n_scan_tiles(int64_t n_seg) { return (n_seg + kScanTile - 1) / kScanTile; }

// Decomposition of a support-S local chunk into waves: the S*S cell classes (y mod S,
// x mod S) are numbered c = p*S + q and spread evenly over nchunk_of(S, slots) waves, at most
// `slots` classes per lane.
__host__ __device__ inline int nchunk_of(int S, int slots) { return (S * S + kWave * slots - 1) / (kWave * slots); }

// Status helpers
#define WG_HIP_CHECK(expr)                                   \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return WG_EHIP;                \
    } while (0)

// Polarisation slot whose value (weight, flag) a record puts into slot q: with four products
// a flipped record (psi < 0) exchanges the cross hands (V_pq(-u) = conj V_qp(u)). The
// exchange is its own inverse, so the adjoint reads slot pol_source(p) for value p.
template <int NP>
__device__ inline int pol_source(int q, int psi) {
    return (NP == 4 && psi < 0 && (q == 1 || q == 2)) ? 3 - q : q;
}

// Polarisations per record (n_pol 0 is read as 1).
inline int npol_of(const wg_geom *g) { return g->n_pol > 1 ? g->n_pol : 1; }

inline int launch_status() { return hipGetLastError() == hipSuccess ? WG_OK : WG_EHIP; }

// Geometry checks shared by every entry point.
int check_geom(const wg_geom *g);
int check_table(const wg_geom *g, const wg_ktable *kt);

// Wave-level helpers --------------------------------------------------------------------
__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & (kWave - 1);
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <typename T>
__device__ inline T wave_sum(T v) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Float mod for small positive divisors: x mod S for 0 <= x < 2^22 and S <= 63.
__device__ inline int mod_small(int x, int S, float rS) {
    int q = (int)((float)x * rS);
    int r = x - q * S;
    r += (r < 0) ? S : 0;
    r -= (r >= S) ? S : 0;
    return r;
}

}  // namespace wg
