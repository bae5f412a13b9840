// Internal declarations shared by the libwgrid translation units (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wgrid.h"

namespace wg {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxS = WG_MAX_SUPPORT;
constexpr int kNumS = (kMaxS + 1) / 2;  // odd supports 1..kMaxS; support S has index S >> 1
__host__ __device__ inline int sidx(int S) { return S >> 1; }
// Cell classes are owned in groups of neighbouring columns of one footprint row, as many as
// one 16-byte table load holds: pairs with FP32 tables, quads with 16-bit tables (the last
// group of a row may be short). Table rows carry group - 1 repeated columns on each side.
__host__ __device__ constexpr int group_of(int dtype) { return dtype == WG_KF32 ? 2 : 4; }
__host__ __device__ constexpr int pad_of(int dtype) { return group_of(dtype) - 1; }
constexpr int kPadMax = 3;  // the widest padding (16-bit tables)

// Groups per lane: the largest count any kernel instantiation uses, and the counts per
// kernel, table type and polarisation count (measured; the notes give what one more group
// per lane did: with Kahan sums it spills at the 128-VGPR cap, with plain sums it fits at
// the VGPRs given and was no faster, or does not fit).
constexpr int kGroupSlots = 5;
constexpr int kGridGroups = 3;          // gridder, FP32 pairs, one polarisation (4: 126 VGPRs plain)
constexpr int kGridGroupsNarrow = 2;    // gridder, 16-bit quads, one polarisation (3: 139 VGPRs plain)
constexpr int kGridGroupsPol2 = 2;      // gridder, FP32 pairs, two polarisations (3: 125 VGPRs plain)
constexpr int kGridGroupsPol4 = 1;      // gridder, FP32 pairs, four polarisations (2: 126 VGPRs plain)
constexpr int kGridGroupsNarrowPol = 1; // gridder, 16-bit tables: quads with two (2: 133 VGPRs plain), pairs with four polarisations
constexpr int kDegridGroups = 5;        // degridder, FP32 pairs, one polarisation (3: 4 % slower, 6: alike)
constexpr int kDegridGroupsNarrow = 3;  // degridder, 16-bit quads, one polarisation (4: 3 % slower, 5: 20 %)
constexpr int kDegridGroupsPol = 4;     // degridder, FP32 pairs, two or four polarisations (3: 6 % slower)
constexpr int kDegridGroupsNarrowPol = 2;  // degridder, 16-bit tables: quads with two, pairs with four

// ---------------------------------------------------------------------------------------
// Plan layout (int32 words). Items are local chunks (first run, one past last run) of
// consecutive runs of one segment that share a support; they are grouped by support, the
// largest support first.
//   [kPlanCount + S/2] items with support S              (S = 1..kMaxS, odd)
//   [kPlanOff + S/2]   first item slot of support S       (kPlanOff + kNumS = total)
//   [kPlanCur + S/2]   append cursor of support S
//   [kPlanQueueDegrid] degridder work-list counter and exit count (2 words), zero between launches
//   [kPlanQueueGrid]   the same for the gridder's counter walk (large grids)
//   [kPlanGrids]       number of grids the runs address (channels, w-planes or 1)
//   [kPlanHdr ...]     items: 2 * capacity words
//   then               runs per segment, scanned in place: n_seg + 1 words
//   then               scan tile totals: n_tiles + 1 words
// ---------------------------------------------------------------------------------------
constexpr int kPlanCount = 0;
constexpr int kPlanOff = kNumS;
constexpr int kPlanCur = 2 * kNumS + 1;
constexpr int kPlanQueueDegrid = 800;  // each counter on its own 128-byte line
constexpr int kPlanQueueGrid = 832;
constexpr int kPlanGrids = 864;  // read by every batch: kept off the work counters' cache lines
constexpr int kPlanHdr = 896;
static_assert(kPlanCur + kNumS <= kPlanQueueDegrid, "plan header words do not overlap");
constexpr int kScanTile = 4096;

inline int64_t plan_items_at() { return kPlanHdr; }
inline int64_t plan_segcnt_at(int64_t capacity) { return kPlanHdr + 2 * capacity; }
inline int64_t plan_tiles_at(int64_t capacity, int64_t n_seg) { return plan_segcnt_at(capacity) + n_seg + 1; }
inline int64_t n_scan_tiles(int64_t n_seg) { return (n_seg + kScanTile - 1) / kScanTile; }

// Decomposition of a support-S local chunk into waves: the cell classes (y mod S, x mod S)
// of footprint row p are grouped as (q, ..., q + G - 1) for q = 0, G, 2G, ... (the last group
// of a row holds what is left of it), ceil(S / G) groups per row and S ceil(S / G) in all,
// numbered row by row and dealt in order to nchunk_groups(S, G, slots) waves, 64 x `slots`
// groups to each but the last.
__host__ __device__ inline int groups_per_row(int S, int G) { return (S + G - 1) / G; }
__host__ __device__ inline int ngroups(int S, int G) { return S * groups_per_row(S, G); }
__host__ __device__ inline int nchunk_groups(int S, int G, int slots) {
    return (ngroups(S, G) + kWave * slots - 1) / (kWave * slots);
}

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

// Float mod for small positive divisors: x mod S for 0 <= x < 2^22 and 1 <= S <= 2^10.
__device__ inline int mod_small(int x, int S, float rS) {
    int q = (int)((float)x * rS);
    int r = x - q * S;
    r += (r < 0) ? S : 0;
    r -= (r >= S) ? S : 0;
    return r;
}

}  // namespace wg
