// WImager preparation phase on the GPU: PreProcessUVW (discrete choices per record),
// compression (eqs. compression, ci), index creation/filtering, compressed/weighted
// visibilities (eqs. compress1, conjugatetake), the plan of equal-support local chunks, the
// statistics and the normaliser (eq. normalizer).
//
// One wavefront walks one (baseline, channel) segment, 64 records per step. Each lane
// computes its record's key in FP64; the predecessor's key arrives by a lane shuffle (the
// last lane's key is carried to the next step); compression and run starts are ballots; run
// indices are popcounts; gamma is a segmented wave scan headed at run starts, with an open
// run's partial sum carried across steps. Two passes: the first counts runs per segment and
// local chunks per support, a scan turns counts into offsets, the second writes everything.
// The index arithmetic must round exactly like its definition, so this file is compiled
// without floating-point contraction.
#include "wg_common.hpp"

#pragma clang fp contract(off)

namespace wg {
namespace {

struct CArgs {
    int n, beta, lb, n_w, nc, nt, compress;
    int stack;  // w-stacking: every record takes plane 0's kernel; its w-plane picks its grid
    int npol;   // polarisations per record (1, 2 or 4): vis, wt, flag are [record][npol]
    int64_t n_seg;
    double uv_scale;
    const double *uvw;
    const double *il;
    const float2 *vis;
    const float *wt;
    const uint8_t *flag;
    const double *wbound;
    const int32_t *support;
    const double *zeta;
    int32_t *start, *len, *x, *y;
    int16_t *plane;
    int8_t *ou, *ov;
    float2 *gamma;
    int32_t *plan, *items, *segcnt, *tiles;
    wg_stats *stats;
    int16_t *grid_id;  // the grid of each run (its channel, or its w-plane when stacking), else NULL
    double *norm;      // normalisers [grid][npol] (per-channel grids or npol > 1), else NULL
    int norm_per_ch;   // norm has one row per channel (per-channel grids), else one row
    int vec;           // npol > 1 with vis, wt and flag aligned to a record's values: each
                       // record's products are read with vector loads
};

struct Key {
    int X, Y, k, ou, ov, psi, ok;
};

// Cross-lane moves on the DPP path (no LDS): the previous lane's value (wave_shr:1; lane 0
// gets `old`), and lane 63's value in every lane.
__device__ inline int from_prev_lane(int v, int old) { return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xF, 0xF, false); }
__device__ inline int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ inline float lane63f(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }

// Segmented inclusive sum over the wave: lane l receives the sum of v over lanes
// [max(seg, 0), l], where seg = seg_start(l) is the last segment head at or below l (-1:
// none). Shifts by 1, 2, 4, 8 within each row of 16 lanes, then the row broadcasts carry
// lane 15 into rows 1 and 3 and lane 31 into rows 2 and 3; each step is taken only where
// its source lane lies in the receiving lane's segment.
template <int CTRL, int ROWS, bool BC>
__device__ inline float dpp_mv(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, BC));
}
__device__ inline float seg_scan(float v, int seg, int lane) {
    const int r = lane & 15;
    float u;
    u = dpp_mv<0x111, 0xF, true>(v); v += (r >= 1 && lane - 1 >= seg) ? u : 0.f;  // row_shr:1
    u = dpp_mv<0x112, 0xF, true>(v); v += (r >= 2 && lane - 2 >= seg) ? u : 0.f;  // row_shr:2
    u = dpp_mv<0x114, 0xF, true>(v); v += (r >= 4 && lane - 4 >= seg) ? u : 0.f;  // row_shr:4
    u = dpp_mv<0x118, 0xF, true>(v); v += (r >= 8 && lane - 8 >= seg) ? u : 0.f;  // row_shr:8
    u = dpp_mv<0x142, 0xA, false>(v);                                              // row_bcast:15
    v += ((lane & 16) && ((lane | 15) - 16) >= seg) ? u : 0.f;
    u = dpp_mv<0x143, 0xC, false>(v);                                              // row_bcast:31
    v += (lane >= 32 && 31 >= seg) ? u : 0.f;
    return v;
}

// A record's NP flag bytes, byte q in bits 8q..8q+7 (0 without flags).
template <int NP>
__device__ inline unsigned load_flags(const CArgs &a, int64_t r) {
    if (!a.flag) return 0u;
    if constexpr (NP == 4)
        if (a.vec) return *(const unsigned *)(a.flag + 4 * r);
    if constexpr (NP == 2)
        if (a.vec) return *(const unsigned short *)(a.flag + 2 * r);
    unsigned f = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) f |= (unsigned)a.flag[r * NP + q] << (8 * q);
    return f;
}

// A record's NP visibilities and weights (weights 1 without them).
template <int NP>
__device__ inline void load_values(const CArgs &a, int64_t r, float2 *v, float *w) {
    if (NP > 1 && a.vec) {
        const float4 *vp = (const float4 *)(a.vis + r * NP);
#pragma unroll
        for (int h = 0; h < NP / 2; ++h) {
            const float4 x = vp[h];
            v[2 * h] = make_float2(x.x, x.y);
            v[2 * h + 1] = make_float2(x.z, x.w);
        }
        if constexpr (NP == 4) {
            const float4 x = a.wt ? *(const float4 *)(a.wt + 4 * r) : make_float4(1.f, 1.f, 1.f, 1.f);
            w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
        } else {
            const float2 x = a.wt ? *(const float2 *)(a.wt + 2 * r) : make_float2(1.f, 1.f);
            w[0] = x.x; w[1] = x.y;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        v[q] = a.vis[r * NP + q];
        w[q] = a.wt ? a.wt[r * NP + q] : 1.0f;
    }
}

// t with t - 1/2 < x <= t + 1/2 (eq. sat at the fine interval), exact for |x| < 2^30.
__device__ inline int fine_index(double x) {
    double t = ceil(x - 0.5);
    if (!(t - 0.5 < x))
        t -= 1.0;
    else if (!(x <= t + 0.5))
        t += 1.0;
    return (int)t;
}

__device__ inline Key index_record(double um, double vm, double wm, double il, bool flagged,
                                   const CArgs &a, const double *s_wb, const int *s_sup) {
    Key r;
    r.X = r.Y = r.k = r.ou = r.ov = 0;
    const double ul = um * il, vl = vm * il, wl = wm * il;
    r.psi = (wm >= 0.0) ? 1 : -1;
    const double sg = (double)r.psi;
    const double uf = sg * ul, vf = sg * vl, wa = sg * wl;
    const double pu = uf * a.uv_scale, pv = vf * a.uv_scale;
    if (!(fabs(pu) < 1073741824.0) || !(fabs(pv) < 1073741824.0) || !isfinite(wa)) {
        r.ok = 0;
        return r;
    }
    const int tu = fine_index(pu), tv = fine_index(pv);
    const int hb = a.beta >> 1;
    r.X = (tu + hb - 1) >> a.lb;  // floor division by a power of two
    r.Y = (tv + hb - 1) >> a.lb;
    r.ou = tu - (r.X << a.lb);
    r.ov = tv - (r.Y << a.lb);
    int lo = 1, hi = a.n_w;  // #{j >= 1 : wa >= wbound[j]}
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_wb[mid] <= wa)
            lo = mid + 1;
        else
            hi = mid;
    }
    r.k = lo - 1;
    const int S = s_sup[r.k], H = (S - 1) >> 1;
    const int ax = r.X + a.n / 2 - H, row0 = r.Y + a.n / 2 - H;
    r.ok = !flagged && ax >= 0 && ax + S <= a.n && row0 >= 0 && row0 + S <= a.n;
    return r;
}

__global__ void k_init(CArgs a, int64_t n_records) {
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < kPlanHdr; i += blockDim.x)
            a.plan[i] = i == kPlanGrids ? (a.grid_id ? (a.stack ? a.n_w : a.nc) : 1) : 0;
        if (a.norm)
            for (int c = threadIdx.x; c < (a.norm_per_ch ? a.nc : 1) * a.npol; c += blockDim.x) a.norm[c] = 0.0;
        if (threadIdx.x == 0) {
            a.stats->n_records = n_records;
            a.stats->n_griddable = 0;
            a.stats->n_runs = 0;
            a.stats->n_compressed = 0;
            a.stats->upd_real = 0;
            a.stats->upd_saved = 0;
            a.stats->normaliser = 0.0;
            a.stats->n_items = 0;
        }
    }
}

// Local chunks and statistics are gathered per workgroup in LDS and published with one
// global atomic per counter (per-support counters and the statistics words are shared by
// every wave of the launch, so per-wave atomics would serialise on a few addresses). In the
// emit pass the chunk records are staged in LDS and given slots per support at the end; a
// chunk that does not fit the stage takes its slot directly.
constexpr int kStage = 1024;
constexpr int kSegWaves = 16;  // segments (one per wave) per k_segments workgroup

struct BlockAgg {
    int cnt[kNumS];    // chunks per support (index S >> 1)
    int fill[kNumS];   // emit: slots handed out per support
    int base[kNumS];   // emit: first slot reserved per support
    int nstaged;
    int2 items[kStage];
    int itemS[kStage];
    unsigned long long st[4];
    double norm;  // the first polarisation's normaliser (the statistics word)
};

template <bool EMIT>
__device__ inline void close_item(const CArgs &a, BlockAgg &agg, int S, int begin, int end) {
    if (!EMIT) {
        atomicAdd(&agg.cnt[sidx(S)], 1);
        return;
    }
    const int i = atomicAdd(&agg.nstaged, 1);
    if (i < kStage) {
        agg.items[i] = make_int2(begin, end);
        agg.itemS[i] = S;
        atomicAdd(&agg.cnt[sidx(S)], 1);
    } else {
        const int slot = atomicAdd(&a.plan[kPlanCur + sidx(S)], 1);
        a.items[2 * slot] = begin;
        a.items[2 * slot + 1] = end;
    }
}

template <bool EMIT, int NP>
__device__ void walk_segment(const CArgs &a, int64_t seg, const double *s_wb, const int *s_sup, BlockAgg &agg);

template <bool EMIT, int NP>
__global__ __launch_bounds__(1024) void k_segments(CArgs a) {
    __shared__ double s_wb[WG_MAX_PLANES];
    __shared__ int s_sup[WG_MAX_PLANES];
    __shared__ BlockAgg agg;
    for (int i = threadIdx.x; i < a.n_w; i += blockDim.x) {
        s_wb[i] = a.wbound[i];
        s_sup[i] = a.support[a.stack ? 0 : i];  // stacking: plane 0's support for every plane
    }
    static_assert(kNumS <= 1024, "one thread per support counter");
    if (threadIdx.x < kNumS) {
        agg.cnt[threadIdx.x] = 0;
        agg.fill[threadIdx.x] = 0;
    }
    if (threadIdx.x < 4) agg.st[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        agg.nstaged = 0;
        agg.norm = 0.0;
    }
    __syncthreads();
    // Waves take segments in (channel, baseline) order, so that the local chunks each
    // workgroup appends to the plan come from different baselines: neighbouring work units
    // of the gridder then sweep different regions of the grid. (Run numbering follows the
    // record order and does not depend on this.)
    const int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (g < a.n_seg) {
        const int64_t nb = a.n_seg / a.nc, ch = g / nb, b = g - ch * nb;
        walk_segment<EMIT, NP>(a, b * a.nc + ch, s_wb, s_sup, agg);
    }
    __syncthreads();
    if (!EMIT) {
        if (threadIdx.x < kNumS && agg.cnt[threadIdx.x]) atomicAdd(&a.plan[kPlanCount + threadIdx.x], agg.cnt[threadIdx.x]);
        if (threadIdx.x == 0) {
            if (agg.st[0]) atomicAdd((unsigned long long *)&a.stats->n_griddable, agg.st[0]);
            if (agg.st[1]) atomicAdd((unsigned long long *)&a.stats->n_compressed, agg.st[1]);
            if (agg.st[2]) atomicAdd((unsigned long long *)&a.stats->upd_real, agg.st[2]);
            if (agg.st[3]) atomicAdd((unsigned long long *)&a.stats->upd_saved, agg.st[3]);
        }
    } else {
        if (threadIdx.x < kNumS && agg.cnt[threadIdx.x])
            agg.base[threadIdx.x] = atomicAdd(&a.plan[kPlanCur + threadIdx.x], agg.cnt[threadIdx.x]);
        if (threadIdx.x == 0 && agg.norm != 0.0) atomicAdd(&a.stats->normaliser, agg.norm);
        __syncthreads();
        const int nst = min(agg.nstaged, kStage);
        for (int i = threadIdx.x; i < nst; i += blockDim.x) {
            const int S = agg.itemS[i];
            const int slot = agg.base[sidx(S)] + atomicAdd(&agg.fill[sidx(S)], 1);
            a.items[2 * slot] = agg.items[i].x;
            a.items[2 * slot + 1] = agg.items[i].y;
        }
    }
}

template <bool EMIT, int NP>
__device__ void walk_segment(const CArgs &a, int64_t seg, const double *s_wb, const int *s_sup, BlockAgg &agg) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t b = seg / a.nc;
    const int ch = (int)(seg - b * a.nc);
    const double il = a.il[ch];
    const uint64_t lt = lanemask_lt();
    const int nbeta2 = a.beta * a.beta;

    int cX = 0, cY = 0, cK = 0, cOu = 0, cOv = 0, cOk = 0;  // key of the previous step's last record
    int runs_before = 0, lastS = -1;
    int item_begin = -1, item_S = 0;
    bool open = false;  // EMIT: a run still open at the end of the previous step
    int open_idx = 0, open_len = 0;
    float og_r[NP], og_i[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) og_r[q] = og_i[q] = 0.f;
    int run_base = 0;
    if (EMIT) run_base = a.segcnt[seg] + a.tiles[seg / kScanTile];
    int64_t my_real = 0, my_saved = 0;
    int n_ok = 0, n_c = 0;
    double my_norm[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) my_norm[q] = 0.0;

    // uvw of the lane's record one step ahead: each step's loads are in flight while the
    // previous step is indexed
    const double *uvw_b = a.uvw + b * a.nt * 3;
    double nu = 0.0, nv = 0.0, nw = 0.0;
    if (lane < a.nt) {
        nu = uvw_b[lane * 3];
        nv = uvw_b[lane * 3 + 1];
        nw = uvw_b[lane * 3 + 2];
    }
    for (int t0 = 0; t0 < a.nt; t0 += kWave) {
        const int t = t0 + lane;
        const bool valid = t < a.nt;
        const int64_t r = seg * a.nt + t;
        const double cu = nu, cv = nv, cw = nw;
        if (t + kWave < a.nt) {
            nu = uvw_b[(t + kWave) * 3];
            nv = uvw_b[(t + kWave) * 3 + 1];
            nw = uvw_b[(t + kWave) * 3 + 2];
        }
        Key key;
        key.ok = 0;
        key.X = key.Y = key.k = key.ou = key.ov = 0;
        key.psi = 1;
        unsigned fw = 0;  // the record's flag bytes
        if (valid) {
            fw = load_flags<NP>(a, r);
            bool fl = a.flag != nullptr;  // dropped only when every polarisation is flagged
#pragma unroll
            for (int q = 0; q < NP; ++q)
                if (((fw >> (8 * q)) & 0xFFu) == 0) fl = false;
            key = index_record(cu, cv, cw, il, fl, a, s_wb, s_sup);
        }
        // the previous record's key; lane 0 takes the carried one
        const int pX = from_prev_lane(key.X, cX), pY = from_prev_lane(key.Y, cY);
        const int pK = from_prev_lane(key.k, cK), pOu = from_prev_lane(key.ou, cOu);
        const int pOv = from_prev_lane(key.ov, cOv), pOk = from_prev_lane(key.ok, cOk);
        const bool same = key.X == pX && key.Y == pY && key.k == pK && key.ou == pOu && key.ov == pOv;
        const bool c = a.compress && t > 0 && key.ok && pOk && same;
        const bool g = key.ok && !c;
        const uint64_t gm = __ballot(g), cm = __ballot(c), okm = __ballot(key.ok);
        const int S = key.ok ? s_sup[key.k] : 0;

        if (EMIT && open && !(cm & 1ull)) {  // the carried run ended with the previous step
            if (lane == 0) {
                a.len[open_idx] = open_len;
#pragma unroll
                for (int q = 0; q < NP; ++q) a.gamma[(int64_t)open_idx * NP + q] = make_float2(og_r[q], og_i[q]);
            }
            open = false;
        }

        // local chunks: a run starts a new chunk when its support differs from the previous run's
        const uint64_t gbelow = gm & lt;
        const int src = gbelow ? 63 - __clzll(gbelow) : 0;
        const int sprev_l = __shfl(S, src, kWave);
        const int prevS = gbelow ? sprev_l : lastS;
        uint64_t ism = __ballot(g && S != prevS);
        while (ism) {
            const int L = __ffsll((unsigned long long)ism) - 1;
            ism &= ism - 1;
            const int SL = __shfl(S, L, kWave);
            const int jL = runs_before + __popcll(gm & ((1ull << L) - 1ull));
            if (item_begin >= 0 && lane == 0) close_item<EMIT>(a, agg, item_S, run_base + item_begin, run_base + jL);
            item_begin = jL;
            item_S = SL;
        }

        n_ok += __popcll(okm);
        n_c += __popcll(cm);
        if (!EMIT) {
            if (g) my_real += (int64_t)S * S;
            if (c) my_saved += (int64_t)S * S;
        } else {
            // slot q: weight * (1 - flag) * (vis, conjugated when flipped) of its source slot
            float sr[NP], si[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) sr[q] = si[q] = 0.f;
            if (key.ok) {
                const int sigma = (key.ov + (a.beta >> 1) - 1) * a.beta + (key.ou + (a.beta >> 1) - 1);
                const double z = a.zeta[(int64_t)(a.stack ? 0 : key.k) * nbeta2 + sigma];
                float2 vv[NP];
                float ww[NP];
                load_values<NP>(a, r, vv, ww);
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const int src = pol_source<NP>(q, key.psi);
                    // q is a compile-time index after unrolling: src is q or, four products
                    // with a flipped record, 3 - q
                    float w = ww[q];
                    float2 v = vv[q];
                    if constexpr (NP == 4) {
                        w = src != q ? ww[3 - q] : w;
                        v = src != q ? vv[3 - q] : v;
                    }
                    if (NP > 1 && ((fw >> (8 * src)) & 0xFFu)) w = 0.0f;
                    sr[q] = w * v.x;
                    si[q] = w * ((float)key.psi * v.y);
                    my_norm[q] += (double)w * z;
                }
            }
            const uint64_t gle = gm & (lt | (1ull << lane));
            const int seg_start = gle ? 63 - __clzll(gle) : -1;
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                sr[q] = seg_scan(sr[q], seg_start, lane);
                si[q] = seg_scan(si[q], seg_start, lane);
            }
            if (seg_start < 0 && open) {
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    sr[q] += og_r[q];
                    si[q] += og_i[q];
                }
            }
            if (g) {
                const int j = run_base + runs_before + __popcll(gbelow);
                a.start[j] = (int32_t)r;
                a.x[j] = key.X;
                a.y[j] = key.Y;
                a.plane[j] = (int16_t)(a.stack ? 0 : key.k);
                a.ou[j] = (int8_t)key.ou;
                a.ov[j] = (int8_t)key.ov;
                if (a.grid_id) a.grid_id[j] = (int16_t)(a.stack ? key.k : ch);
            }
            const int cnext = __shfl_down((int)c, 1, kWave);
            const bool last_in_seg = (t == a.nt - 1);
            const bool is_end = key.ok && (last_in_seg || (lane < kWave - 1 && !cnext));
            if (is_end) {
                int j, ln;
                if (seg_start >= 0) {
                    j = run_base + runs_before + __popcll(gle) - 1;
                    ln = lane - seg_start + 1;
                } else {
                    j = open_idx;
                    ln = open_len + lane + 1;
                }
                a.len[j] = ln;
#pragma unroll
                for (int q = 0; q < NP; ++q) a.gamma[(int64_t)j * NP + q] = make_float2(sr[q], si[q]);
            }
            const int carry = lane63((int)(key.ok && !is_end));
            const int ss63 = lane63(seg_start);
            float cr[NP], ci[NP];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                cr[q] = lane63f(sr[q]);
                ci[q] = lane63f(si[q]);
            }
            if (carry) {
                if (ss63 >= 0) {
                    open_idx = run_base + runs_before + __popcll(gm) - 1;
                    open_len = kWave - ss63;
                } else {
                    open_len += kWave;
                }
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    og_r[q] = cr[q];
                    og_i[q] = ci[q];
                }
                open = true;
            } else {
                open = false;
            }
        }
        cX = lane63(key.X);
        cY = lane63(key.Y);
        cK = lane63(key.k);
        cOu = lane63(key.ou);
        cOv = lane63(key.ov);
        cOk = lane63(key.ok);
        if (gm) lastS = __shfl(S, 63 - __clzll(gm), kWave);
        runs_before += __popcll(gm);
    }
    if (item_begin >= 0 && lane == 0) close_item<EMIT>(a, agg, item_S, run_base + item_begin, run_base + runs_before);
    if (!EMIT) {
        const int64_t real = wave_sum(my_real), saved = wave_sum(my_saved);
        if (lane == 0) {
            a.segcnt[seg] = runs_before;
            atomicAdd(&agg.st[0], (unsigned long long)n_ok);
            atomicAdd(&agg.st[1], (unsigned long long)n_c);
            atomicAdd(&agg.st[2], (unsigned long long)real);
            atomicAdd(&agg.st[3], (unsigned long long)saved);
        }
    } else {
        double nsum[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) nsum[q] = wave_sum(my_norm[q]);
        if (lane == 0) {
            atomicAdd(&agg.norm, nsum[0]);
            if (a.norm)
#pragma unroll
                for (int q = 0; q < NP; ++q)
                    if (nsum[q] != 0.0) atomicAdd(&a.norm[(a.norm_per_ch ? ch : 0) * NP + q], nsum[q]);
        }
    }
}

// Exclusive scan of up to 1024 per-thread values; returns the thread's offset, *total = sum.
__device__ int block_exclusive_scan(int v, int *s_wave, int *total) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int xs = v;
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(xs, d, kWave);
        if (lane >= d) xs += y;
    }
    if (lane == kWave - 1) s_wave[wid] = xs;
    __syncthreads();
    if (wid == 0) {
        int w = lane < nw ? s_wave[lane] : 0;
        for (int d = 1; d < kWave; d <<= 1) {
            const int y = __shfl_up(w, d, kWave);
            if (lane >= d) w += y;
        }
        if (lane < nw) s_wave[lane] = w;
    }
    __syncthreads();
    const int off = (wid ? s_wave[wid - 1] : 0) + xs - v;
    *total = s_wave[nw - 1];
    __syncthreads();
    return off;
}

// Per-tile exclusive scan of runs-per-segment (in place) and tile totals.
__global__ __launch_bounds__(1024) void k_scan_tiles(CArgs a) {
    __shared__ int s_wave[16];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    int v[4], sum = 0;
    for (int i = 0; i < 4; ++i) {
        v[i] = (base + i < a.n_seg) ? a.segcnt[base + i] : 0;
        sum += v[i];
    }
    int total;
    int off = block_exclusive_scan(sum, s_wave, &total);
    for (int i = 0; i < 4; ++i) {
        if (base + i < a.n_seg) a.segcnt[base + i] = off;
        off += v[i];
    }
    if (threadIdx.x == 0) a.tiles[blockIdx.x] = total;
}

// Scan of tile totals; run count; local-chunk offsets per support (largest support first).
__global__ __launch_bounds__(1024) void k_scan_top(CArgs a, int64_t n_tiles) {
    __shared__ int s_wave[16];
    int carry = 0;
    for (int64_t c0 = 0; c0 < n_tiles; c0 += blockDim.x) {
        const int64_t i = c0 + threadIdx.x;
        const int v = i < n_tiles ? a.tiles[i] : 0;
        int total;
        const int off = block_exclusive_scan(v, s_wave, &total);
        if (i < n_tiles) a.tiles[i] = carry + off;
        carry += total;
    }
    if (threadIdx.x == 0) {
        a.tiles[n_tiles] = carry;
        a.stats->n_runs = carry;
        int acc = 0;
        for (int S = kMaxS; S >= 1; S -= 2) {
            a.plan[kPlanOff + sidx(S)] = acc;
            a.plan[kPlanCur + sidx(S)] = acc;
            acc += a.plan[kPlanCount + sidx(S)];
        }
        a.plan[kPlanOff + kNumS] = acc;
        a.stats->n_items = acc;
    }
}

}  // namespace
}  // namespace wg

extern "C" int wg_compress(const wg_geom *g, const wg_ktable *kt, const double *uvw,
                           const double *inv_lambda, const float *vis, const float *weight,
                           const uint8_t *flag, int64_t nb, int32_t nc, int32_t nt, wg_runs *runs,
                           wg_stats *stats, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    st = check_table(g, kt);
    if (st != WG_OK) return st;
    if (!uvw || !inv_lambda || !vis || !runs || !stats) return WG_EINVAL;
    if (nb < 1 || nc < 1 || nt < 1) return WG_EINVAL;
    const int64_t n_rec = nb * (int64_t)nc * nt;
    if (n_rec >= (int64_t)1 << 31) return WG_EUNSUPPORTED;
    if (!runs->start || !runs->len || !runs->x || !runs->y || !runs->plane || !runs->ou || !runs->ov ||
        !runs->gamma || !runs->plan)
        return WG_EINVAL;
    const int64_t n_seg = nb * nc;
    const bool per_channel = (g->flags & WG_GRID_PER_CHANNEL) != 0;
    const bool stack = (g->flags & WG_W_STACKING) != 0;
    const int npol = npol_of(g);
    if (npol > 1 && !runs->norm) return WG_EINVAL;
    if (per_channel) {
        if (!runs->grid || !runs->norm) return WG_EINVAL;
        if (nc > 32767 || (int64_t)nc * npol * g->n * g->n >= ((int64_t)1 << 31)) return WG_EUNSUPPORTED;
    }
    if (stack) {
        if (!runs->grid) return WG_EINVAL;
        if ((int64_t)g->n_w * npol * g->n * g->n >= ((int64_t)1 << 31)) return WG_EUNSUPPORTED;
    }
    if (runs->capacity < n_rec) return WG_ECAPACITY;
    if (runs->plan_elems < wg_plan_elems(runs->capacity, n_seg)) return WG_ECAPACITY;

    CArgs a;
    a.n = g->n;
    a.beta = g->beta;
    a.lb = 0;
    while ((1 << a.lb) < g->beta) ++a.lb;
    a.n_w = g->n_w;
    a.nc = nc;
    a.nt = nt;
    a.compress = (g->flags & WG_COMPRESS) ? 1 : 0;
    a.stack = stack ? 1 : 0;
    a.npol = npol;
    a.n_seg = n_seg;
    a.uv_scale = (double)g->beta / g->du;
    a.uvw = uvw;
    a.il = inv_lambda;
    a.vis = (const float2 *)vis;
    a.wt = weight;
    a.flag = flag;
    a.vec = npol > 1 && (uintptr_t)vis % 16 == 0 && (uintptr_t)weight % (4 * npol) == 0 &&
            (uintptr_t)flag % npol == 0;
    a.wbound = kt->wbound;
    a.support = kt->support;
    a.zeta = kt->zeta;
    a.start = runs->start;
    a.len = runs->len;
    a.x = runs->x;
    a.y = runs->y;
    a.plane = runs->plane;
    a.ou = runs->ou;
    a.ov = runs->ov;
    a.gamma = (float2 *)runs->gamma;
    a.plan = runs->plan;
    a.items = runs->plan + plan_items_at();
    a.segcnt = runs->plan + plan_segcnt_at(runs->capacity);
    a.tiles = runs->plan + plan_tiles_at(runs->capacity, n_seg);
    a.stats = stats;
    a.grid_id = (per_channel || stack) ? runs->grid : nullptr;
    a.norm = (per_channel || npol > 1) ? runs->norm : nullptr;
    a.norm_per_ch = per_channel ? 1 : 0;

    hipStream_t s = (hipStream_t)stream;
    const int64_t n_tiles = n_scan_tiles(n_seg);
    // 16 segments (waves) per workgroup: the per-support chunk counters and the statistics
    // take one global atomic per workgroup each, and these few addresses serialise them
    // (4 waves per workgroup: 0.31 ms for the compress step of a 15,136-segment batch; 16: 0.19)
    const int64_t seg_blocks = (n_seg + kSegWaves - 1) / kSegWaves;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, a, n_rec);
    auto segments = [&](bool emit) {
        void (*k)(CArgs) = npol == 4   ? (emit ? k_segments<true, 4> : k_segments<false, 4>)
                           : npol == 2 ? (emit ? k_segments<true, 2> : k_segments<false, 2>)
                                       : (emit ? k_segments<true, 1> : k_segments<false, 1>);
        hipLaunchKernelGGL(k, dim3((unsigned)seg_blocks), dim3(kSegWaves * kWave), 0, s, a);
    };
    segments(false);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_tiles), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, a, n_tiles);
    segments(true);
    return launch_status();
}
