// Internal declarations shared by the libwgrid translation units (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wgrid.h"

namespace wg {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxS = WG_MAX_SUPPORT;
// Class pairs per lane (each pair is two cell classes fetched with one load; the last pair
// of a footprint row has one class): the largest count any kernel instantiation uses, and
// the counts per kernel, table type and polarisation count.
constexpr int kPairSlots = 5;
constexpr int kGridPairs = 3;          // gridder, FP32 tables, one polarisation (4 spill at 128 VGPRs)
constexpr int kGridPairsNarrow = 3;    // the same with BF16/FP16 tables (4 spill)
constexpr int kGridPairsPol2 = 2;      // gridder with two polarisations (any table type; 3 spill)
constexpr int kGridPairsPol4 = 1;      // gridder with four polarisations (2 spill)
constexpr int kDegridPairs = 3;        // degridder, FP32 tables, one polarisation (7.8 ms on the
                                       // 4096^2 workload, 8.0 with 4 and 8.1 with 5)
constexpr int kDegridPairsNarrow = 5;  // the same with BF16/FP16 tables (6.7 ms, 6.8 with 4, 7.0 with 3)
constexpr int kDegridPairsPol2 = 3;    // degridder with two polarisations (4 measure alike)
constexpr int kDegridPairsPol4 = 3;    // degridder with four polarisations (5.5 ms on 2048^2, 5.65 with 2)

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

// Decomposition of a support-S local chunk into waves: the cell classes (y mod S, x mod S)
// of footprint row p are paired as (q, q + 1) for q = 0, 2, ..., S - 1 (the last pair has no
// second class), S (S + 1) / 2 pairs in all, numbered row by row and spread evenly over
// nchunk_pairs(S, slots) waves, at most `slots` pairs per lane.
__host__ __device__ inline int npairs(int S) { return S * (S + 1) / 2; }
__host__ __device__ inline int nchunk_pairs(int S, int slots) { return (npairs(S) + kWave * slots - 1) / (kWave * slots); }

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
