// Gridding phase (eq. gridding) and its adjoint on gfx950.
//
// Work unit = one local chunk (consecutive runs of one baseline/channel trajectory with a
// common support S) x one share of its cell classes. A class (p, q) stands for the grid
// cells with y = p mod S and x = q mod S; every footprint position holds exactly one cell of
// each class. Lane l owns a few classes: as the footprint slides along the trajectory the
// lane keeps updating the same cell, accumulating gamma*K in FP32 registers with Kahan
// compensation (or, on request, plain FP32 sums as in the thesis's single-precision gridder),
// and commits with FP32 atomic adds only when the cell leaves the footprint -- the ownership
// idea of Romein's gridder, applied per wavefront.
//
// Classes are owned in groups of neighbouring columns of one footprint row, as many as one
// 16-byte load holds: pairs (q, q + 1) with FP32 tables, quads (q, ..., q + 3) with 16-bit
// tables. Their samples sit next to each other in a table row (padded with G - 1 repeated
// columns on each side, so that a group that wraps from column S - 1 to column 0 is
// adjacent too, read forwards or, for a mirrored matrix, backwards) and one load fetches
// them all. A vector load instruction costs about the same whatever its width, and the
// instruction rate of the vector memory path is what bounds these kernels.
#include <type_traits>

#include "wg_common.hpp"

#pragma clang fp contract(off)

namespace wg {
namespace {

struct GArgs {
    int n, beta, n_w, nc, nt;
    int npol;  // polarisations per record, run and cell (1, 2 or 4)
    int64_t n_rec, data_cap;
    const int32_t *start, *len, *x, *y;
    const int16_t *plane;
    const int8_t *ou, *ov;
    const float2 *gamma;
    const int32_t *plan, *items;
    const int16_t *grid_id;  // the grid of each run (its channel or its w-plane), else NULL
    int64_t cells;           // cells of one polarisation's grid (n*n); polarisation p of a
                             // cell is cells*p values further on
    int32_t *queue;  // work-list counter and exit count of this kernel (two plan words)
    const int64_t *offset;
    const void *data;
    float *grid;        // grid (wg_grid, accumulate) or input grid (wg_degrid)
    float2 *vis_out;    // wg_degrid output
    float2 *work;       // wg_degrid per-run dot products
    const wg_stats *stats;
    const double *uvw;
    const float *wt;
    const uint8_t *flag;
};

// Classes per group in a kernel: what one 16-byte load of its table type holds (pairs with
// FP32 tables, quads with 16-bit tables), except pairs for 16-bit tables with four
// polarisations, whose accumulators do not fit four classes per slot in 128 VGPRs.
template <int DT, int NP>
constexpr int kgroup() { return DT == WG_KF32 ? 2 : NP == 4 ? 2 : 4; }

// The samples of a class group as fetched (converted to float only when used, so that a
// wave can keep several loads in flight): two complex FP32 values, or G packed complex
// 16-bit values.
template <int DT, int G> struct GroupRaw { using type = uint4; };
template <> struct GroupRaw<WG_KBF16, 2> { using type = uint2; };
template <> struct GroupRaw<WG_KF16, 2> { using type = uint2; };
template <> struct GroupRaw<WG_KF32, 2> { using type = float4; };

template <int DT>
__device__ inline float2 to_float2(uint32_t u) {
    if constexpr (DT == WG_KBF16) {
        return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xFFFF0000u));
    } else {
        _Float16 lo, hi;
        const uint16_t l16 = (uint16_t)(u & 0xFFFFu), h16 = (uint16_t)(u >> 16);
        __builtin_memcpy(&lo, &l16, 2);
        __builtin_memcpy(&hi, &h16, 2);
        return make_float2((float)lo, (float)hi);
    }
}

// Sample h < G of a group as a complex float.
template <int DT, int G>
__device__ inline float2 group_sample(const typename GroupRaw<DT, G>::type &v, int h) {
    if constexpr (DT == WG_KF32)
        return h == 0 ? make_float2(v.x, v.y) : make_float2(v.z, v.w);
    else if constexpr (G == 2)
        return to_float2<DT>(h == 0 ? v.x : v.y);
    else
        return to_float2<DT>(h == 0 ? v.x : h == 1 ? v.y : h == 2 ? v.z : v.w);
}

// Supports present in the plan, largest first, with their first work unit.
struct UnitTable {
    int n;
    int S[kNumS];
    int first[kNumS + 1];
};

// Built by the first wave of the workgroup: lane l takes the four supports
// kMaxS - 2 (4l + k), k = 0..3 (largest first), and a wave prefix sum over the lanes' unit
// and support counts places them.
static_assert(kNumS == 4 * kWave, "four supports per lane");
__device__ void build_units(const int32_t *plan, int G, int slots, UnitTable *t, int lane) {
    int cnt[4], units[4];
    int u = 0, np = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int S = kMaxS - 2 * (4 * lane + k);
        cnt[k] = plan[kPlanCount + sidx(S)];
        units[k] = cnt[k] * nchunk_groups(S, G, slots);
        u += units[k];
        np += cnt[k] > 0 ? 1 : 0;
    }
    // inclusive prefix sums over the lanes
    int su = u, sn = np;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int pu = __shfl_up(su, d, kWave), pn = __shfl_up(sn, d, kWave);
        if (lane >= d) {
            su += pu;
            sn += pn;
        }
    }
    int first = su - u, m = sn - np;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (cnt[k] > 0) {
            t->S[m] = kMaxS - 2 * (4 * lane + k);
            t->first[m] = first;
            first += units[k];
            ++m;
        }
    if (lane == kWave - 1) {
        t->first[sn] = su;
        t->n = sn;
    }
}

// Run records of up to 64 consecutive runs, one per lane, with everything the per-run loop
// needs precomputed in parallel; the loop then broadcasts run t with v_readlane.
// Tables are read only at non-negative oversample offsets. The kernel is even in u and in v
// (eq. C_W: the taper and the w-screen are even in l and in m), so the matrix of offset -o
// along an axis is the matrix of +o reversed along that axis (position j <-> S - 1 - j).
// Reading the 25 of 64 matrices with o >= 0 per axis, backwards along an axis where the
// run's offset is negative, cuts the samples a plane keeps in the caches by 2.5. Read
// backwards along u, the load of a class group starts at the group's last sample, so the
// samples arrive in reverse order.
template <int NP>
struct RunBatch {
    int cell0, ph, kb, ok;  // ph: footprint origin phases, (row0 mod S) << 16 | (ax mod S)
    int mul;                // signed byte strides of the footprint position in the table,
                            // row << 16 | column (a negative column stride: the group's
                            // samples arrive reversed); kb is the matrix origin read from
    float gr[NP], gi[NP];   // the run's weighted visibility sum per polarisation
};

__device__ inline int rl(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ inline float rlf(float v, int t) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t)); }
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int DT, int NP>
__device__ inline RunBatch<NP> load_batch(const GArgs &a, int S, int j, bool valid, const int64_t *koff) {
    constexpr int esz = (DT == WG_KF32) ? 8 : 4;
    constexpr int G = kgroup<DT, NP>(), P = pad_of(DT);
    static_assert(G - 1 <= P, "the row padding covers a group's wrap");
    RunBatch<NP> b;
    b.ok = 0;
    b.cell0 = b.ph = b.kb = b.mul = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) b.gr[p] = b.gi[p] = 0.f;
    if (valid) {
        const int H = (S - 1) >> 1, half = a.n >> 1, hb = a.beta >> 1;
        const int X = a.x[j], Y = a.y[j], k = a.plane[j];
        const int gid = a.grid_id ? a.grid_id[j] : 0;
        const int ou = a.ou[j], ov = a.ov[j], W = S + 2 * P;  // W: samples per table row
        const int sigma = (abs(ov) + hb - 1) * a.beta + (abs(ou) + hb - 1);
        const int ax = X + half - H, row0 = Y + half - H;
        const int64_t kbase = koff[k] + (int64_t)sigma * S * W;
        // runs from wg_compress with the same geometry and table always pass; anything else
        // is skipped rather than read or written out of bounds
        if (ax >= 0 && ax + S <= a.n && row0 >= 0 && row0 + S <= a.n && kbase >= 0 &&
            kbase + (int64_t)S * W <= a.data_cap && gid >= 0 && gid < a.plan[kPlanGrids]) {
            b.ok = 1;
            b.cell0 = row0 * a.n + ax + (int)(gid * a.cells * NP);
            b.ph = (row0 % S) << 16 | (ax % S);
            // a group whose first class sits in footprint column j loads from row position
            // P + j forwards, P + S - G - j backwards (whose G samples are the columns of
            // footprint positions j + G - 1 down to j); footprint row i reads matrix row i,
            // or S - 1 - i backwards
            const int mu = ou < 0 ? -esz : esz, rv = ov < 0 ? -W * esz : W * esz;
            b.mul = (int)((unsigned)(unsigned short)mu | (unsigned)(unsigned short)rv << 16);
            b.kb = (int)kbase + (ou < 0 ? P + S - G : P) + (ov < 0 ? (S - 1) * W : 0);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const float2 g = a.gamma[(int64_t)j * NP + p];
                b.gr[p] = g.x;
                b.gi[p] = g.y;
            }
        }
    }
    return b;
}

// Buffer resource for the table: 32-bit byte offsets, and reads beyond num_bytes return 0.
__device__ inline __amdgpu_buffer_rsrc_t table_rsrc(const void *data, int64_t num_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(data), (short)0, (int)num_bytes, 0x00020000);
}

template <int DT, int G>
__device__ inline typename GroupRaw<DT, G>::type group_load(__amdgpu_buffer_rsrc_t rs, int off) {
    if constexpr (DT != WG_KF32 && G == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        return make_uint2((unsigned)v[0], (unsigned)v[1]);
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        if constexpr (DT == WG_KF32)
            return make_float4(__int_as_float(v[0]), __int_as_float(v[1]), __int_as_float(v[2]), __int_as_float(v[3]));
        else
            return make_uint4((unsigned)v[0], (unsigned)v[1], (unsigned)v[2], (unsigned)v[3]);
    }
}

// Class positions are handled as two 16-bit halves, column in the low half and row in the
// high half, so that both wraps take three packed integer ops and each linear index one
// v_dot2_u32_u16.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline u16x2 as_u16x2(unsigned v) { return __builtin_bit_cast(u16x2, v); }

// Position (column jj, row ii) of the class cls = (q, p) in a footprint whose origin has the
// phases ph = (ax mod S, row0 mod S): ((q - ax) mod S, (p - row0) mod S).
__device__ inline u16x2 footprint_pos(u16x2 cls, u16x2 ph, u16x2 ss) {
    const u16x2 d = cls - ph;
    return __builtin_elementwise_min(d, d + ss);
}

// w.x * m.x + w.y * m.y + c (v_dot2_u32_u16)
__device__ inline unsigned dot2(u16x2 w, u16x2 m, unsigned c) { return __builtin_amdgcn_udot2(w, m, c, false); }

// A wave-uniform value held in a VGPR, so that an instruction taking it together with a
// per-run scalar needs only one scalar operand.
__device__ inline unsigned in_vgpr(unsigned x) {
    unsigned r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// Table byte offset of footprint position w = (column, row) with signed strides m and a
// wave-uniform origin c in a scalar register: w.x * m.x + w.y * m.y + c as one
// three-operand v_dot2_i32_i16. (From the builtin the compiler selects the two-operand
// v_dot2c_i32_i16, whose addend is its destination, and copies the scalar into it first:
// two operations per slot and run instead of one.)
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ inline unsigned table_off(u16x2 w, unsigned m, unsigned c) {
    int r;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(r) : "v"(__builtin_bit_cast(unsigned, w)), "v"(m), "s"(c));
    return (unsigned)r;
}

// The lane's class groups of a chunk: slot m holds group min(k0 + 64 m + lane, k1 - 1), i.e.
// row p = k / gpr and first column q = G (k mod gpr) with gpr = ceil(S / G) groups per row,
// as (q, p); nval[m] = min(G, S - q) of its classes exist. Only the last slot can lie past
// the lane's share (*idle: the lane then repeats the last group and must neither add nor
// commit), since the slot count is ceil((k1 - k0) / 64).
template <int NS, int G>
__device__ inline void lane_groups(int S, int k0, int k1, int lane, u16x2 *cls, int *nval, bool *idle) {
    const int gpr = groups_per_row(S, G);
    const float rg = 1.0f / (float)gpr;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
        const int k = min(k0 + m * kWave + lane, k1 - 1);
        const int pp = (int)((float)k * rg + 0.5f * rg);
        const int q = G * (k - pp * gpr);
        cls[m] = u16x2{(unsigned short)q, (unsigned short)pp};
        nval[m] = min(G, S - q);
    }
    *idle = k0 + (NS - 1) * kWave + lane >= k1;
}

// Samples and cells of one run for the lane's group slots, fetched one run ahead.
template <int DT, int G>
struct Stage {
    typename GroupRaw<DT, G>::type k[kGroupSlots];
    unsigned yc[kGroupSlots];  // cell of the group's first class; set only when the footprint moved
    int wrap[kGroupSlots];     // classes of the group before it wraps from footprint column S - 1
                               // to column 0 (S minus the first class's column); set with yc
    bool moved;                // wave-uniform: the run's footprint origin differs from the previous run's
    bool swap;                 // wave-uniform: the run reads its matrix backwards along u, so each
                               // load holds the group's samples in reverse order
};

// Cell of class h of a group whose first class has cell c and `wrap` classes before the
// footprint's column S - 1: the next columns, continuing from column 0 after the wrap.
__device__ inline unsigned class_cell(unsigned c, int h, int wrap, int S) {
    return h == 0 ? c : c + (unsigned)h - (h >= wrap ? (unsigned)S : 0u);
}

// Cell base of "no previous run": no footprint starts there (cell bases are below n*n).
constexpr unsigned kNoCell = 0xFFFFFFFFu;

// Static walk over the support-sorted work list (largest supports first): wave w takes
// units w, w + W, ... (W waves in the launch). Waves drift apart, so the units in flight
// spread over much of the list: many baselines and w-planes at once.
template <typename F>
__device__ inline void for_each_unit_static(int nunits, F &&body) {
    const int wpb = blockDim.x / kWave;
    const int stride = gridDim.x * wpb;
    for (int u = uni(blockIdx.x * wpb + (int)(threadIdx.x / kWave)); u < nunits; u += stride) body(u);
}

// Persistent walk over the support-sorted work list (largest supports first) through a
// shared counter: each wave takes the next unit, so the units in flight form a narrow window
// of the list (one or two w-planes at a time: a table working set that stays in L2). Within
// a support the plan lists chunks channel-major, so the window spans many baselines and
// their commits rarely meet on a cell. Every wave leaves once the list is exhausted; the
// last one out resets the counter and the exit count for the next launch.
constexpr int kUnitsPerTicket = 4;  // units handed out per counter increment

template <typename F>
__device__ inline void for_each_unit(int nunits, int32_t *q, F &&body) {
    const int lane = threadIdx.x & (kWave - 1);
    const int nwaves = (int)(gridDim.x * (blockDim.x / kWave));
    for (;;) {
        int u0 = 0;
        if (lane == 0) u0 = atomicAdd(&q[0], kUnitsPerTicket);
        u0 = __builtin_amdgcn_readlane(u0, 0);
        if (u0 >= nunits) break;
        const int u1 = min(u0 + kUnitsPerTicket, nunits);
        for (int u = u0; u < u1; ++u) body(u);
    }
    if (lane == 0) {
        __threadfence();
        if (atomicAdd(&q[1], 1) == nwaves - 1) {
            atomicExch(&q[0], 0);
            atomicExch(&q[1], 0);
        }
    }
}

template <int DT, int NP>
constexpr int grid_slots();

// Words of one wave's commit list (the cells of one footprint move, and their real and
// imaginary values per polarisation): one entry per class the wave owns, and 32 more for
// the entries an earlier move left for the next one.
template <int DT, int NP>
constexpr int commit_words() { return (kgroup<DT, NP>() * grid_slots<DT, NP>() * kWave + 32) * (1 + 2 * NP); }

// KAHAN: compensated sums per owned cell, else plain FP32 sums.
template <int DT, int NP, int NS, bool KAHAN>
__device__ __attribute__((always_inline)) void grid_chunk_ns(const GArgs &a, int S, int k0, int k1, int rb, int re,
                                                             int lane, const int64_t *koff, float *cl_v) {
    constexpr int esz = (DT == WG_KF32) ? 8 : 4;
    constexpr int G = kgroup<DT, NP>();
    const __amdgpu_buffer_rsrc_t rs = table_rsrc(a.data, a.data_cap * esz);

    u16x2 cls[kGroupSlots];
    int nval[kGroupSlots];
    bool idle;
    lane_groups<NS, G>(S, k0, k1, lane, cls, nval, &idle);
    // an idle last slot (past the lane's share of groups) reads past the table's end, which
    // gives zeros: it adds nothing, and it never commits
    const unsigned idle_off = idle ? 0x80000000u : 0u;
    const u16x2 ss = {(unsigned short)S, (unsigned short)S};
    const u16x2 mul_c = {(unsigned short)1, (unsigned short)a.n};  // cell offset in the grid
    // per group slot, class h and polarisation: the owned cell's sum since its last commit
    // and its Kahan compensation (zero throughout with plain sums)
    float acc_r[NS][G][NP], acc_i[NS][G][NP], cmp_r[NS][G][NP], cmp_i[NS][G][NP];
    unsigned cur[kGroupSlots][G];  // owned cells (y*n + x); set from the chunk's first run
    // Footprint positions of the lane's first classes, recomputed only when the footprint moves
    // (consecutive runs of a chunk mostly differ in oversampling offsets or plane alone).
    u16x2 wpos[kGroupSlots];
    unsigned last_cell0 = kNoCell;
#pragma unroll
    for (int m = 0; m < NS; ++m)
#pragma unroll
        for (int h = 0; h < G; ++h)
#pragma unroll
            for (int p = 0; p < NP; ++p) acc_r[m][h][p] = acc_i[m][h][p] = cmp_r[m][h][p] = cmp_i[m][h][p] = 0.f;
    // Commit the cell's compensated sums (acc - cmp) of every polarisation; the next cell
    // starts from acc = cmp, i.e. from the value zero, with the compensation term left as it
    // is (Kahan's recurrence holds from any starting pair). With plain sums cmp stays zero.
    //
    // Commits are compacted. When the footprint moves, each (slot, class) of the wave whose
    // cell leaves writes that cell and its values to the wave's list in LDS (its place from
    // one ballot per class and mbcnt, so the list runs lane by lane, class by class: a row of
    // leaving cells stays a run of neighbouring cells, whereas one atomic per slot and class
    // would cover every G-th cell). Most moves commit one column of the footprint, a few
    // lanes per slot: issued slot by slot, that took about a dozen atomic instructions with
    // three or four active lanes each.
    //
    // The list is then added to the grid 32 entries per atomic instruction, lanes 2e and
    // 2e + 1 taking the real and imaginary parts of entry e: one instruction covers the
    // contiguous values of 32 neighbouring cells (two or three cache lines), where one lane
    // per entry and one instruction per component touched twice as many lines, each half
    // used; the L2's atomic cost goes by the lines an instruction touches. A footprint move
    // adds only the list's whole blocks of 32 entries and moves the rest (at most 31) to its
    // head, for the next move to complete; the chunk's end adds everything. (A move leaves
    // one column or row of the footprint, a few cells per wave: added at once, they took an
    // atomic instruction for about 11 entries.)
    constexpr int kStride = G * NS * kWave + 32;  // entries of one list array: every class of the wave and a carried block
    static_assert(kStride * (1 + 2 * NP) <= commit_words<DT, NP>(), "commit list fits the wave's LDS");
    unsigned *cl_c = (unsigned *)cl_v;
    unsigned nlist = 0;  // wave-uniform
    auto collect = [&](int m, const bool *go) {
        uint64_t bal[G];
        uint64_t any = 0;
#pragma unroll
        for (int h = 0; h < G; ++h) {
            bal[h] = __ballot(go[h]);
            any |= bal[h];
        }
        if (any == 0ull) return;
        unsigned e = nlist;
#pragma unroll
        for (int h = 0; h < G; ++h)
            e = __builtin_amdgcn_mbcnt_hi((unsigned)(bal[h] >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal[h], e));
#pragma unroll
        for (int h = 0; h < G; ++h)
            if (go[h]) {
                cl_c[e] = cur[m][h];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    cl_v[kStride * (1 + 2 * p) + e] = acc_r[m][h][p] - cmp_r[m][h][p];
                    cl_v[kStride * (2 + 2 * p) + e] = acc_i[m][h][p] - cmp_i[m][h][p];
                    acc_r[m][h][p] = cmp_r[m][h][p];
                    acc_i[m][h][p] = cmp_i[m][h][p];
                }
                ++e;
            }
#pragma unroll
        for (int h = 0; h < G; ++h) nlist += (unsigned)__builtin_popcountll(bal[h]);
    };
    auto flush = [&](bool all) {
        const unsigned nf = all ? nlist : (nlist & ~31u);
        const unsigned comp = (unsigned)lane & 1u;
        for (unsigned e = (unsigned)lane >> 1; e < nf; e += kWave / 2) {
            float *val = a.grid + (2u * cl_c[e] + comp);  // cell indices < 2^31
#pragma unroll
            for (int p = 0; p < NP; ++p) unsafeAtomicAdd(val + 2 * p * a.cells, cl_v[kStride * (1 + comp + 2 * p) + e]);
        }
        const unsigned rem = nlist - nf;
        if (nf != 0u && rem != 0u && (unsigned)lane < rem) {
            const unsigned src = nf + (unsigned)lane;
            unsigned c = cl_c[src];
            float v[2 * NP];
#pragma unroll
            for (int q = 0; q < 2 * NP; ++q) v[q] = cl_v[kStride * (1 + q) + src];
            cl_c[lane] = c;
#pragma unroll
            for (int q = 0; q < 2 * NP; ++q) cl_v[kStride * (1 + q) + lane] = v[q];
        }
        nlist = rem;
    };
    // Commits are only for classes that exist: not in an idle last slot, and not past the
    // end of a row's short last group.
    auto owns = [&](int m, int h) { return (m < NS - 1 || !idle) && h < nval[m]; };
    bool first = true;

    for (int base = rb; base < re; base += kWave) {
        const int n = min(kWave, re - base);
        const RunBatch<NP> b = load_batch<DT, NP>(a, S, base + lane, lane < n, koff);

        // cells (when the footprint moved) and sample groups of the lane's slots for run t
        auto fetch = [&](int t, Stage<DT, G> &st) {
            const unsigned cell0 = (unsigned)rl(b.cell0, t);
            const unsigned kbB = (unsigned)rl(b.kb, t) * esz;
            const unsigned mul = (unsigned)rl(b.mul, t);
            const bool ok = rl(b.ok, t) != 0;
            st.swap = (mul & 0x8000u) != 0u;
            st.moved = !ok || cell0 != last_cell0;
            last_cell0 = (unsigned)uni((int)(ok ? cell0 : kNoCell));
            if (st.moved) {
                const u16x2 ph = as_u16x2((unsigned)rl(b.ph, t));
#pragma unroll
                for (int m = 0; m < NS; ++m) {
                    wpos[m] = footprint_pos(cls[m], ph, ss);
                    st.yc[m] = dot2(wpos[m], mul_c, cell0);
                    st.wrap[m] = S - (int)wpos[m].x;
                }
            }
            const unsigned mulv = in_vgpr(mul);
#pragma unroll
            for (int m = 0; m < NS; ++m) {
                const unsigned off = table_off(wpos[m], mulv, kbB);
                st.k[m] = group_load<DT, G>(rs, (int)(m == NS - 1 ? off | idle_off : off));
            }
        };
        // A run that failed load_batch's checks (and lane n, past a batch of odd length n)
        // carries gamma = 0: its step adds zero, so the loop needs no branch on it. Such a
        // failed run counts as moved, with cells inside the first grid's corner, so the next
        // good run commits what was held there (zero) and moves on.
        auto accumulate = [&](int t, const Stage<DT, G> &st, auto fold) {
            float gr[NP], gi[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                gr[p] = rlf(b.gr[p], t);
                gi[p] = rlf(b.gi[p], t);
            }
            // cells that left the footprint are committed under one wave-uniform branch (most
            // runs keep their footprint)
            if (st.moved) {
#pragma unroll
                for (int m = 0; m < NS; ++m) {
                    unsigned yc[G];
                    bool go[G];
#pragma unroll
                    for (int h = 0; h < G; ++h) {
                        yc[h] = class_cell(st.yc[m], h, st.wrap[m], S);
                        go[h] = owns(m, h) && yc[h] != cur[m][h];
                    }
                    collect(m, go);
#pragma unroll
                    for (int h = 0; h < G; ++h) cur[m][h] = yc[h];
                }
                flush(false);
            }
            // Kahan step with the product fused into the compensation:
            // y = gamma*K - c, t = s + y, c = (t - s) - y, s = t, in blocks of two runs: the
            // first run of each pair (`fold`) only subtracts its product from c (two FMAs per
            // component), and the second run's full step absorbs both (the value, s - c, is
            // right after either run, so a commit may come between them). With plain sums
            // s += gamma*K, two FMAs per component. One sample serves every polarisation.
            // Class h takes sample h of the load, or sample G - 1 - h when the run reads
            // backwards along u (one copy of the sums per case, under a wave-uniform branch).
            auto sums = [&](auto swapped) {
                constexpr int sw = decltype(swapped)::value;
#pragma unroll
                for (int m = 0; m < NS; ++m)
#pragma unroll
                    for (int h = 0; h < G; ++h) {
                        const float2 kv = group_sample<DT, G>(st.k[m], sw ? G - 1 - h : h);
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            if constexpr (KAHAN && decltype(fold)::value) {
                                cmp_r[m][h][p] = fmaf(-gr[p], kv.x, fmaf(gi[p], kv.y, cmp_r[m][h][p]));
                                cmp_i[m][h][p] = fmaf(-gr[p], kv.y, fmaf(-gi[p], kv.x, cmp_i[m][h][p]));
                            } else if constexpr (KAHAN) {
                                const float yr = fmaf(gr[p], kv.x, -fmaf(gi[p], kv.y, cmp_r[m][h][p]));
                                const float yi = fmaf(gr[p], kv.y, fmaf(gi[p], kv.x, -cmp_i[m][h][p]));
                                const float tr = acc_r[m][h][p] + yr, ti = acc_i[m][h][p] + yi;
                                cmp_r[m][h][p] = (tr - acc_r[m][h][p]) - yr;
                                cmp_i[m][h][p] = (ti - acc_i[m][h][p]) - yi;
                                acc_r[m][h][p] = tr;
                                acc_i[m][h][p] = ti;
                            } else {
                                acc_r[m][h][p] = fmaf(gr[p], kv.x, fmaf(-gi[p], kv.y, acc_r[m][h][p]));
                                acc_i[m][h][p] = fmaf(gr[p], kv.y, fmaf(gi[p], kv.x, acc_i[m][h][p]));
                            }
                        }
                    }
            };
            // (the two markers differ, so the compiler cannot merge the copies into one with
            // selects on every sample)
            if (st.swap) {
                sums(std::integral_constant<int, 1>{});
                asm volatile("; samples reversed");
            } else {
                sums(std::integral_constant<int, 0>{});
                asm volatile("; samples in order");
            }
        };

        Stage<DT, G> sa, sb;
        fetch(0, sa);
        if (first) {
#pragma unroll
            for (int m = 0; m < NS; ++m)
#pragma unroll
                for (int h = 0; h < G; ++h) cur[m][h] = class_cell(sa.yc[m], h, sa.wrap[m], S);
            first = false;
        }
        // The next run's fetch is issued on every path (past the batch's end it repeats the
        // last run, whose footprint has not moved), so the waits before each accumulation
        // leave that prefetch in flight; a fetch skipped on some path would make them wait
        // for every outstanding load. With n odd, step t + 1 = n repeats run n - 1's
        // footprint with lane n's zero gamma.
        // (the scheduling barriers keep each fetch ahead of the sums it overlaps)
        for (int t = 0; t < n; t += 2) {
            fetch(min(t + 1, n - 1), sb);
            __builtin_amdgcn_sched_barrier(0);
            accumulate(t, sa, std::true_type{});
            fetch(min(t + 2, n - 1), sa);
            __builtin_amdgcn_sched_barrier(0);
            accumulate(t + 1, sb, std::false_type{});
        }
    }
    if (!first) {
#pragma unroll
        for (int m = 0; m < NS; ++m) {
            bool go[G];
#pragma unroll
            for (int h = 0; h < G; ++h) go[h] = owns(m, h);
            collect(m, go);
        }
        flush(true);
    }
}

// Class groups [k0, k1) of share `chunk` of a support-S chunk: the shares are filled in
// order, 64 x slots groups each and the last one the rest, so a run costs the fewest load
// slots, ceil(groups / 64) (an even split left part of a slot idle in every share: S = 35,
// 630 groups over four shares, took 12 slots instead of 10). The slot count per lane is a
// template parameter so the unrolled slot loops carry no guards.
__device__ inline void chunk_groups(int S, int G, int chunk, int slots, int &k0, int &k1, int &ns) {
    const int ng = ngroups(S, G);
    k0 = chunk * kWave * slots;
    k1 = min(ng, k0 + kWave * slots);
    ns = uni((k1 - k0 + kWave - 1) / kWave);
}

// Slot count as a template parameter, instantiated for 1..MAX only (the kernel's register
// allocation is the largest over its instantiations).
template <int DT, int NP, int NS, int MAX, bool KAHAN>
__device__ __attribute__((always_inline)) inline void grid_dispatch(int ns, const GArgs &a, int S, int c0, int c1, int rb, int re, int lane,
                                     const int64_t *koff, float *cl) {
    if constexpr (NS < MAX) {
        if (ns == NS) {
            grid_chunk_ns<DT, NP, NS, KAHAN>(a, S, c0, c1, rb, re, lane, koff, cl);
            return;
        }
        grid_dispatch<DT, NP, NS + 1, MAX, KAHAN>(ns, a, S, c0, c1, rb, re, lane, koff, cl);
    } else {
        grid_chunk_ns<DT, NP, MAX, KAHAN>(a, S, c0, c1, rb, re, lane, koff, cl);
    }
}

// Most class groups per lane of the gridder; the accumulators of more classes per group and
// of more polarisations take the registers of more groups.
template <int DT, int NP>
constexpr int grid_slots() {
    if constexpr (DT == WG_KF32)
        return NP == 4 ? kGridGroupsPol4 : NP == 2 ? kGridGroupsPol2 : kGridGroups;
    else
        return NP == 1 ? kGridGroupsNarrow : kGridGroupsNarrowPol;
}

template <int DT, int NP, bool KAHAN>
__device__ __attribute__((always_inline)) void grid_chunk(const GArgs &a, int S, int chunk, int rb, int re, int lane,
                                                          const int64_t *koff, float *cl) {
    int k0, k1, ns;
    chunk_groups(S, kgroup<DT, NP>(), chunk, grid_slots<DT, NP>(), k0, k1, ns);
    grid_dispatch<DT, NP, 1, grid_slots<DT, NP>(), KAHAN>(ns, a, S, k0, k1, rb, re, lane, koff, cl);
}

// COUNTER: the work list is walked through the counter in a.queue, else statically (one
// walk per instantiation, so the unit body is inlined once). KAHAN: compensated sums.
template <int DT, int NP, bool COUNTER, bool KAHAN>
__global__ __launch_bounds__(256, 4) void k_grid(GArgs a) {
    __shared__ UnitTable ut;
    __shared__ int64_t koff[WG_MAX_PLANES + 1];
    __shared__ float commit_lists[4 * commit_words<DT, NP>()];  // one per wave (256 threads)
    float *cl = commit_lists + (threadIdx.x / kWave) * commit_words<DT, NP>();
    if (threadIdx.x < kWave) build_units(a.plan, kgroup<DT, NP>(), grid_slots<DT, NP>(), &ut, threadIdx.x);
    for (int k = threadIdx.x; k <= a.n_w; k += blockDim.x) koff[k] = a.offset[k];
    __syncthreads();
    const int nunits = uni(ut.first[ut.n]);
    const int lane = threadIdx.x & (kWave - 1);
    auto unit = [&](int u) {
        int m = 0;
        while (u >= ut.first[m + 1]) ++m;
        const int S = uni(ut.S[m]), nch = nchunk_groups(S, kgroup<DT, NP>(), grid_slots<DT, NP>());
        const int rel = u - uni(ut.first[m]);
        const int item = rel / nch, chunk = rel - item * nch;
        const int slot = uni(a.plan[kPlanOff + sidx(S)]) + item;
        grid_chunk<DT, NP, KAHAN>(a, S, chunk, uni(a.items[2 * slot]), uni(a.items[2 * slot + 1]), lane, koff, cl);
    };
    if constexpr (COUNTER)
        for_each_unit(nunits, a.queue, unit);
    else
        for_each_unit_static(nunits, unit);
}

// One DPP move within each row of 16 lanes (all rows and banks on).
template <int CTRL>
__device__ inline float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Wave totals of two complex values at once: after the call, lanes 0-15 hold the total of
// re0, 16-31 of re1, 32-47 of im0 and 48-63 of im1. v_permlane32_swap trades the upper half
// of re for the lower half of im, so the two swapped registers add to re[l] + re[l + 32] in
// the lower half and im[l - 32] + im[l] in the upper half; this for both values, then
// v_permlane16_swap of the two results trades row 1 of the first for row 0 of the second
// and row 3 of the first for row 2 of the second, so one add leaves one value per row and
// the DPP moves inside each row finish all four.
__device__ inline float wave_total_quad(float re0, float im0, float re1, float im1) {
    const auto h0 = __builtin_amdgcn_permlane32_swap(__float_as_int(re0), __float_as_int(im0), false, false);
    const auto h1 = __builtin_amdgcn_permlane32_swap(__float_as_int(re1), __float_as_int(im1), false, false);
    const float v = __int_as_float(h0[0]) + __int_as_float(h0[1]);
    const float w = __int_as_float(h1[0]) + __int_as_float(h1[1]);
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(w), false, false);
    float u = __int_as_float(r[0]) + __int_as_float(r[1]);
    u += dpp_f<0xB1>(u);   // quad_perm [1,0,3,2]
    u += dpp_f<0x4E>(u);   // quad_perm [2,3,0,1]
    u += dpp_f<0x141>(u);  // row_half_mirror
    u += dpp_f<0x140>(u);  // row_mirror
    return u;
}

// Adjoint, with the gridder's decomposition: a wave owns the same cell class groups of a
// local chunk, keeps the grid value of each owned cell in a register and reloads the values
// only when the footprint moves (about one run in seven), and forms per run the partial dot
// product of conj(K) with those values (a short FMA chain per lane, then one lane-swap and
// DPP tree over the wave for the real and imaginary parts of two runs together). The waves
// sharing a chunk add their partial sums into work[run]; k_degrid_finish hands d to the
// run's records.
static_assert(kGridGroups <= kGroupSlots && kGridGroupsNarrow <= kGroupSlots && kGridGroupsPol2 <= kGroupSlots &&
                  kGridGroupsPol4 <= kGroupSlots && kGridGroupsNarrowPol <= kGroupSlots &&
                  kDegridGroups <= kGroupSlots && kDegridGroupsNarrow <= kGroupSlots &&
                  kDegridGroupsPol <= kGroupSlots && kDegridGroupsNarrowPol <= kGroupSlots,
              "per-lane stage arrays hold kGroupSlots groups");
template <int DT, int G>
struct DStage {
    typename GroupRaw<DT, G>::type k[kGroupSlots];
    bool moved;  // wave-uniform: the run's footprint origin differs from the previous run's
    bool swap;   // wave-uniform: the loads hold each group's samples in reverse order
};

// The NP complex values of one cell, one from each polarisation plane ([NP][n][n] grid).
template <int NP>
__device__ inline void load_cell(const float2 *grid, unsigned cell, int64_t cells, float2 *v) {
#pragma unroll
    for (int p = 0; p < NP; ++p) v[p] = grid[cell + p * cells];
}

// Order of the loads per run t: the sample groups of run t + 1 are issued before run t's sums,
// and when run t + 1 moves the footprint its grid values are loaded into the owned-cell
// registers right after run t's last use of them. The wait before run t + 1's sums then
// covers those grid values and run t + 1's samples while run t + 2's samples stay in flight,
// whichever path was taken.
template <int DT, int NP, int NS>
__device__ __attribute__((always_inline)) void degrid_chunk_ns(const GArgs &a, int S, int k0, int k1, int rb,
                                                               int re, int lane, const int64_t *koff) {
    constexpr int esz = (DT == WG_KF32) ? 8 : 4;
    constexpr int G = kgroup<DT, NP>();
    const __amdgpu_buffer_rsrc_t rs = table_rsrc(a.data, a.data_cap * esz);
    const float2 *grid = (const float2 *)a.grid;
    u16x2 cls[kGroupSlots];
    int nval[kGroupSlots];
    bool idle;
    lane_groups<NS, G>(S, k0, k1, lane, cls, nval, &idle);
    // an idle last slot reads its samples past the table's end (zeros)
    const unsigned idle_off = idle ? 0x80000000u : 0u;
    const u16x2 ss = {(unsigned short)S, (unsigned short)S};
    const u16x2 mul_c = as_u16x2(in_vgpr((unsigned)a.n << 16 | 1u));
    float2 gv[NS][G][NP];        // grid values of the owned cells (0 for a class that does not exist)
    unsigned vcell[NS][G];       // the cell whose values gv holds
    u16x2 wpos[kGroupSlots];     // footprint positions of the first classes, when the footprint moves
    unsigned gcell[kGroupSlots]; // first class's cell of the last run that moved the footprint
    unsigned last_cell0 = kNoCell;
#pragma unroll
    for (int m = 0; m < NS; ++m)
#pragma unroll
        for (int h = 0; h < G; ++h) {
            vcell[m][h] = kNoCell;
#pragma unroll
            for (int p = 0; p < NP; ++p) gv[m][h][p] = make_float2(0.f, 0.f);
        }

    for (int base = rb; base < re; base += kWave) {
        const int n = min(kWave, re - base);
        const RunBatch<NP> b = load_batch<DT, NP>(a, S, base + lane, lane < n, koff);

        // footprint positions and cells (when the footprint moved) and sample groups of run t
        auto fetch = [&](int t, DStage<DT, G> &st) {
            const unsigned cell0 = (unsigned)rl(b.cell0, t);
            const unsigned kbB = (unsigned)rl(b.kb, t) * esz;
            const unsigned mul = (unsigned)rl(b.mul, t);
            const bool ok = rl(b.ok, t) != 0;
            st.swap = (mul & 0x8000u) != 0u;
            st.moved = !ok || cell0 != last_cell0;
            last_cell0 = (unsigned)uni((int)(ok ? cell0 : kNoCell));
            if (st.moved) {
                const u16x2 ph = as_u16x2((unsigned)rl(b.ph, t));
#pragma unroll
                for (int m = 0; m < NS; ++m) {
                    wpos[m] = footprint_pos(cls[m], ph, ss);
                    gcell[m] = dot2(wpos[m], mul_c, cell0);
                }
            }
            const unsigned mulv = in_vgpr(mul);
#pragma unroll
            for (int m = 0; m < NS; ++m) {
                const unsigned off = table_off(wpos[m], mulv, kbB);
                st.k[m] = group_load<DT, G>(rs, (int)(m == NS - 1 ? off | idle_off : off));
            }
        };
        // the grid values of the owned cells of the last run that moved the footprint, loaded
        // only for the classes whose cell changed: a footprint that moves by a cell changes the
        // cells of one row or column of classes (1 in S of them), and a load instruction none
        // of whose lanes changed is skipped; a class past the end of a row's short last group
        // keeps the value 0
        auto load_values = [&]() {
#pragma unroll
            for (int m = 0; m < NS; ++m) {
                const int wrap = S - (int)wpos[m].x;
#pragma unroll
                for (int h = 0; h < G; ++h) {
                    const unsigned c = class_cell(gcell[m], h, wrap, S);
                    if (h < nval[m] && c != vcell[m][h]) {
                        load_cell<NP>(grid, c, a.cells, gv[m][h]);
                        vcell[m][h] = c;
                    }
                }
            }
        };
        // this wave's sums, reduced two runs at a time: for the pair of runs 2j and 2j + 1
        // (j = 0..31 in the batch), lane 16k + (j & 15) of lo (j < 16) or hi (j >= 16) holds
        // row k of the pair's totals: the real part of run 2j, of run 2j + 1, the imaginary
        // part of run 2j, of run 2j + 1
        float lo[NP], hi[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) lo[p] = hi[p] = 0.f;
        float qr[2][NP], qi[2][NP];  // the pair's partial sums in this lane
        auto consume = [&](int t, const DStage<DT, G> &st) {
            float *pr = qr[t & 1], *pim = qi[t & 1];
#pragma unroll
            for (int p = 0; p < NP; ++p) pr[p] = pim[p] = 0.f;
            // class h takes sample h of the load, or G - 1 - h when the run reads backwards
            // along u
            auto sums = [&](auto swapped) {
                constexpr int sw = decltype(swapped)::value;
#pragma unroll
                for (int m = 0; m < NS; ++m)
#pragma unroll
                    for (int h = 0; h < G; ++h) {
                        const float2 kv = group_sample<DT, G>(st.k[m], sw ? G - 1 - h : h);
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            pr[p] = fmaf(kv.x, gv[m][h][p].x, fmaf(kv.y, gv[m][h][p].y, pr[p]));
                            pim[p] = fmaf(kv.x, gv[m][h][p].y, fmaf(-kv.y, gv[m][h][p].x, pim[p]));
                        }
                    }
            };
            if (st.swap) {
                sums(std::integral_constant<int, 1>{});
                asm volatile("; samples reversed");
            } else {
                sums(std::integral_constant<int, 0>{});
                asm volatile("; samples in order");
            }
        };
        // the totals of the pair of runs t, t + 1 (t even) into their lanes; two atomics per
        // polarisation and batch add them all
        auto reduce_pair = [&](int t) {
            const int j = t >> 1;
            const bool mine = (lane & 15) == (j & 15);
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const float d = wave_total_quad(qr[0][p], qi[0][p], qr[1][p], qi[1][p]);
                lo[p] = (mine && j < 16) ? d : lo[p];
                hi[p] = (mine && j >= 16) ? d : hi[p];
            }
        };

        DStage<DT, G> sa, sb;
        fetch(0, sa);
        if (sa.moved) load_values();
        // the next run's fetch is issued on every path, as in the gridder
        for (int t = 0; t < n; t += 2) {
            fetch(min(t + 1, n - 1), sb);
            consume(t, sa);
            if (sb.moved) load_values();
            if (t + 1 < n) {
                fetch(min(t + 2, n - 1), sa);
                consume(t + 1, sb);
                if (sa.moved) load_values();
            } else {
#pragma unroll
                for (int p = 0; p < NP; ++p) qr[1][p] = qi[1][p] = 0.f;
            }
            reduce_pair(t);
        }
        const int row = lane >> 4, r = 2 * (lane & 15) + (row & 1), comp = row >> 1;
        const int ok_lo = __shfl(b.ok, r), ok_hi = __shfl(b.ok, r + 32);
        float *w = (float *)(a.work + (int64_t)(base + r) * NP) + comp;
        if (r < n && ok_lo)
#pragma unroll
            for (int p = 0; p < NP; ++p) unsafeAtomicAdd(w + 2 * p, lo[p]);
        if (r + 32 < n && ok_hi)
#pragma unroll
            for (int p = 0; p < NP; ++p) unsafeAtomicAdd(w + 64 * NP + 2 * p, hi[p]);
    }
}

template <int DT, int NP, int NS, int MAX>
__device__ inline void degrid_dispatch(int ns, const GArgs &a, int S, int c0, int c1, int rb, int re, int lane,
                                       const int64_t *koff) {
    if constexpr (NS < MAX) {
        if (ns == NS) {
            degrid_chunk_ns<DT, NP, NS>(a, S, c0, c1, rb, re, lane, koff);
            return;
        }
        degrid_dispatch<DT, NP, NS + 1, MAX>(ns, a, S, c0, c1, rb, re, lane, koff);
    } else {
        degrid_chunk_ns<DT, NP, MAX>(a, S, c0, c1, rb, re, lane, koff);
    }
}

template <int DT, int NP>
constexpr int degrid_slots() {
    if constexpr (DT == WG_KF32)
        return NP == 1 ? kDegridGroups : kDegridGroupsPol;
    else
        return NP == 1 ? kDegridGroupsNarrow : kDegridGroupsNarrowPol;
}

template <int DT, int NP>
__device__ void degrid_chunk(const GArgs &a, int S, int chunk, int rb, int re, int lane, const int64_t *koff) {
    int k0, k1, ns;
    chunk_groups(S, kgroup<DT, NP>(), chunk, degrid_slots<DT, NP>(), k0, k1, ns);
    degrid_dispatch<DT, NP, 1, degrid_slots<DT, NP>()>(ns, a, S, k0, k1, rb, re, lane, koff);
}

template <int DT, int NP>
__global__ __launch_bounds__(256) void k_degrid(GArgs a) {
    __shared__ UnitTable ut;
    __shared__ int64_t koff[WG_MAX_PLANES + 1];
    if (threadIdx.x < kWave) build_units(a.plan, kgroup<DT, NP>(), degrid_slots<DT, NP>(), &ut, threadIdx.x);
    for (int k = threadIdx.x; k <= a.n_w; k += blockDim.x) koff[k] = a.offset[k];
    __syncthreads();
    const int nunits = uni(ut.first[ut.n]);
    const int lane = threadIdx.x & (kWave - 1);
    for_each_unit(nunits, a.queue, [&](int u) {
        int m = 0;
        while (u >= ut.first[m + 1]) ++m;
        const int S = uni(ut.S[m]);
        // share-major within a support: the waves in flight take the same share of different
        // chunks, so the partial sums they add into work[] go to different runs (a chunk of
        // large support has hundreds of shares, all adding into the same runs' entries)
        const int rel = u - uni(ut.first[m]);
        const int nit = uni(a.plan[kPlanCount + sidx(S)]);
        const int chunk = rel / nit, item = rel - chunk * nit;
        const int slot = uni(a.plan[kPlanOff + sidx(S)]) + item;
        degrid_chunk<DT, NP>(a, S, chunk, uni(a.items[2 * slot]), uni(a.items[2 * slot + 1]), lane, koff);
    });
}

// Clears the per-run accumulators (n_runs * npol entries, read on the device).
__global__ void k_zero_work(GArgs a) {
    const int64_t n = a.stats->n_runs * a.npol;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        a.work[j] = make_float2(0.f, 0.f);
}

// Hands each run's dot products to its records: polarisation p gets weight * (1 - flag) *
// (d[p], or conj d[s] when w < 0, s the slot its value went to). A wave takes 64 runs (in
// record order) and its lanes walk their records in order, so that neighbouring lanes write
// neighbouring records; each lane finds its record's run among the 64 by a shuffle search.
// The wave writes every record from its first run's start (record 0 for the first wave) to
// the next wave's first run's start (the last record for the last wave), so each record is
// written once: records in no run (not griddable) get 0.
template <int NP>
__global__ void k_degrid_finish(GArgs a) {
    const int64_t n = a.stats->n_runs;
    const int64_t seglen = (int64_t)a.nt * a.nc;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
    if (n == 0) {  // no runs: every record gets 0
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.n_rec * NP;
             e += (int64_t)gridDim.x * blockDim.x)
            a.vis_out[e] = make_float2(0.f, 0.f);
        return;
    }
    for (int64_t j0 = ((int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave; j0 < n;
         j0 += nwaves * kWave) {
        const int nv = (int)min((int64_t)kWave, n - j0);
        const bool v = lane < nv;
        const int st = v ? a.start[j0 + lane] : 0x7FFFFFFF;  // runs are in record order
        const int ln = v ? a.len[j0 + lane] : 0;
        const int64_t r_begin = j0 == 0 ? 0 : (int64_t)__shfl(st, 0, kWave);
        const int64_t r_end = j0 + kWave < n ? (int64_t)a.start[j0 + kWave] : a.n_rec;
        for (int64_t base = r_begin; base < r_end; base += kWave) {  // wave-uniform trip count
            const int64_t r = base + lane;
            int l = 0;  // the last of the 64 runs that starts at or before r
            for (int step = kWave / 2; step >= 1; step >>= 1) {
                const int c = l + step;
                const int sc = __shfl(st, c < kWave ? c : kWave - 1, kWave);
                if (c < nv && sc <= r) l = c;
            }
            const int sl = __shfl(st, l, kWave), ll = __shfl(ln, l, kWave);
            if (r >= r_end) continue;
            if (r < sl || r >= (int64_t)sl + ll) {  // in no run
#pragma unroll
                for (int p = 0; p < NP; ++p) a.vis_out[r * NP + p] = make_float2(0.f, 0.f);
                continue;
            }
            const int64_t j = j0 + l;
            const int64_t bb = r / seglen, tt = r - (r / a.nt) * a.nt;
            const double wm = a.uvw[(bb * a.nt + tt) * 3 + 2];
            const int psi = (wm >= 0.0) ? 1 : -1;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const int64_t e = r * NP + p;
                float w = a.wt ? a.wt[e] : 1.0f;
                if (NP > 1 && a.flag && a.flag[e]) w = 0.0f;
                const float2 d = a.work[j * NP + pol_source<NP>(p, psi)];
                a.vis_out[e] = make_float2(w * d.x, w * (psi > 0 ? d.y : -d.y));
            }
        }
    }
}

GArgs make_args(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs) {
    GArgs a;
    a.n = g->n;
    a.beta = g->beta;
    a.n_w = g->n_w;
    a.nc = a.nt = 0;
    a.n_rec = 0;
    a.data_cap = kt->data_cap;
    a.start = runs->start;
    a.len = runs->len;
    a.x = runs->x;
    a.y = runs->y;
    a.plane = runs->plane;
    a.ou = runs->ou;
    a.ov = runs->ov;
    a.gamma = (const float2 *)runs->gamma;
    a.plan = runs->plan;
    a.grid_id = (g->flags & (WG_GRID_PER_CHANNEL | WG_W_STACKING)) ? runs->grid : nullptr;
    a.cells = (int64_t)g->n * g->n;
    a.queue = nullptr;
    a.items = runs->plan + plan_items_at();
    a.offset = kt->offset;
    a.data = kt->data;
    a.grid = nullptr;
    a.vis_out = nullptr;
    a.work = (float2 *)runs->work;
    a.stats = nullptr;
    a.uvw = nullptr;
    a.wt = nullptr;
    a.flag = nullptr;
    a.npol = npol_of(g);
    return a;
}

int check_runs(const wg_geom *g, const wg_runs *runs) {
    if (!runs || !runs->start || !runs->len || !runs->x || !runs->y || !runs->plane || !runs->ou ||
        !runs->ov || !runs->gamma || !runs->plan || runs->capacity < 1)
        return WG_EINVAL;
    if ((g->flags & (WG_GRID_PER_CHANNEL | WG_W_STACKING)) && !runs->grid) return WG_EINVAL;
    return WG_OK;
}

// Workgroups of four waves per launch. The gridder's static walk gains from more waves than
// fit at once (later ones start as early ones finish); a work counter is best served by one
// resident round (four waves per SIMD).
constexpr int kGridBlocks = 8192;
constexpr int kDegridBlocks = 1024;
constexpr int kGridCounterBlocks = 1024;
// The gridder walks its work list through the counter (a narrow window of the support-sorted
// list: one or two planes of table samples in flight, which stay in L2) on grids of at least
// this side, and statically (a wide spread of baselines and planes in flight) on smaller
// ones, where the narrow window's commits meet on the same cells too often. Measured: 4096^2,
// 64 planes, 11.9 M runs: 10.8 ms against 11.8; 2048^2, 32 planes: 3.6 against 3.1 ms.
constexpr int kGridCounterMinSide = 4096;

// The gridder for a table type, polarisation count, walk and summation.
template <int DT, bool COUNTER, bool KAHAN>
void (*pick_grid_np(int npol))(GArgs) {
    return npol == 4   ? k_grid<DT, 4, COUNTER, KAHAN>
           : npol == 2 ? k_grid<DT, 2, COUNTER, KAHAN>
                       : k_grid<DT, 1, COUNTER, KAHAN>;
}
template <bool COUNTER, bool KAHAN>
void (*pick_grid_dt(int dtype, int npol))(GArgs) {
    return dtype == WG_KF32    ? pick_grid_np<WG_KF32, COUNTER, KAHAN>(npol)
           : dtype == WG_KBF16 ? pick_grid_np<WG_KBF16, COUNTER, KAHAN>(npol)
                               : pick_grid_np<WG_KF16, COUNTER, KAHAN>(npol);
}
void (*pick_grid(int dtype, int npol, bool counter, bool kahan))(GArgs) {
    if (kahan) return counter ? pick_grid_dt<true, true>(dtype, npol) : pick_grid_dt<false, true>(dtype, npol);
    return counter ? pick_grid_dt<true, false>(dtype, npol) : pick_grid_dt<false, false>(dtype, npol);
}

// The degridder kernel for a table type and polarisation count.
void (*pick_degrid(int dtype, int npol))(GArgs) {
    if (dtype == WG_KF32)
        return npol == 4 ? k_degrid<WG_KF32, 4> : npol == 2 ? k_degrid<WG_KF32, 2> : k_degrid<WG_KF32, 1>;
    if (dtype == WG_KBF16)
        return npol == 4 ? k_degrid<WG_KBF16, 4> : npol == 2 ? k_degrid<WG_KBF16, 2> : k_degrid<WG_KBF16, 1>;
    return npol == 4 ? k_degrid<WG_KF16, 4> : npol == 2 ? k_degrid<WG_KF16, 2> : k_degrid<WG_KF16, 1>;
}

}  // namespace
}  // namespace wg

extern "C" int wg_grid(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs, const wg_stats *stats,
                       float *grid, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_table(g, kt)) != WG_OK) return st;
    if ((st = check_runs(g, runs)) != WG_OK) return st;
    if (!grid || !stats) return WG_EINVAL;
    if (kt->data_cap >= ((int64_t)1 << 28)) return WG_EUNSUPPORTED;  // byte offsets stay 32-bit
    GArgs a = make_args(g, kt, runs);
    a.grid = grid;
    const bool counter = g->n >= kGridCounterMinSide;
    a.queue = counter ? runs->plan + kPlanQueueGrid : nullptr;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(pick_grid(kt->dtype, a.npol, counter, !(g->flags & WG_PLAIN_SUMS)),
                       dim3(counter ? kGridCounterBlocks : kGridBlocks), dim3(256), 0, s, a);
    return launch_status();
}

extern "C" int wg_degrid(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs, const wg_stats *stats,
                         const float *grid, const double *uvw, const float *weight, const uint8_t *flag,
                         int64_t nb, int32_t nc, int32_t nt, float *vis_out, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_table(g, kt)) != WG_OK) return st;
    if ((st = check_runs(g, runs)) != WG_OK) return st;
    if (!grid || !stats || !uvw || !vis_out || !runs->work || nb < 1 || nc < 1 || nt < 1) return WG_EINVAL;
    if (kt->data_cap >= ((int64_t)1 << 28)) return WG_EUNSUPPORTED;  // byte offsets stay 32-bit
    const int64_t n_rec = nb * (int64_t)nc * nt;
    if (n_rec > runs->capacity) return WG_ECAPACITY;
    GArgs a = make_args(g, kt, runs);
    a.grid = (float *)grid;
    a.vis_out = (float2 *)vis_out;
    a.queue = runs->plan + kPlanQueueDegrid;
    a.uvw = uvw;
    a.wt = weight;
    a.flag = flag;
    a.nc = nc;
    a.nt = nt;
    a.n_rec = n_rec;
    a.stats = stats;
    hipStream_t s = (hipStream_t)stream;
    // clear the per-run accumulators first (k_degrid_finish writes every record)
    hipLaunchKernelGGL(k_zero_work, dim3(2048), dim3(256), 0, s, a);
    hipLaunchKernelGGL(pick_degrid(kt->dtype, a.npol), dim3(kDegridBlocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(a.npol == 4 ? k_degrid_finish<4> : a.npol == 2 ? k_degrid_finish<2> : k_degrid_finish<1>,
                       dim3(2048), dim3(256), 0, s, a);
    return launch_status();
}
