// Gridding phase (eq. gridding) and its adjoint on gfx950.
//
// Work unit = one local chunk (consecutive runs of one baseline/channel trajectory with a
// common support S) x one slice of its rows. Inside a wavefront, lane l owns the column
// class q = l mod S of every footprint and a few row classes p (cells with x = q mod S and
// y = p mod S): as the footprint slides along the trajectory a lane keeps updating the same
// cell, accumulating gamma*K in registers with Kahan compensation, and commits (one FP32
// atomic add per component) only when its cell leaves the footprint -- the ownership idea of
// Romein's gridder, applied per wavefront. Kernel samples are read straight into registers:
// for a fixed row class the 64 lanes read a contiguous (rotated) row of the S x S matrix.
#include "wg_common.hpp"

#pragma clang fp contract(off)

namespace wg {
namespace {

struct GArgs {
    int n, beta, n_w, nc, nt;
    int64_t n_rec, data_cap;
    const int32_t *start, *len, *x, *y;
    const int16_t *plane;
    const int8_t *ou, *ov;
    const float2 *gamma;
    const int32_t *plan, *items;
    const int64_t *offset;
    const void *data;
    float *grid;        // grid (wg_grid, accumulate) or input grid (wg_degrid)
    float2 *vis_out;    // wg_degrid output
    const double *uvw;
    const float *wt;
};

template <int DT>
__device__ inline float2 load_k(const void *data, int64_t idx) {
    if (DT == WG_KF32) return ((const float2 *)data)[idx];
    const uint32_t u = ((const uint32_t *)data)[idx];
    if (DT == WG_KBF16) return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xFFFF0000u));
    _Float16 lo, hi;
    const uint16_t l16 = (uint16_t)(u & 0xFFFFu), h16 = (uint16_t)(u >> 16);
    __builtin_memcpy(&lo, &l16, 2);
    __builtin_memcpy(&hi, &h16, 2);
    return make_float2((float)lo, (float)hi);
}

__device__ inline void kahan_add(float &s, float &c, float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Supports present in the plan, largest first, with their first work unit.
struct UnitTable {
    int n;
    int S[33];
    int first[34];
};

__device__ void build_units(const int32_t *plan, bool per_row_chunk, UnitTable *t) {
    int u = 0, m = 0;
    for (int S = kMaxS; S >= 1; S -= 2) {
        const int c = plan[kPlanCount + S];
        if (c > 0) {
            t->S[m] = S;
            t->first[m] = u;
            u += c * (per_row_chunk ? nchunk_of(S) : 1);
            ++m;
        }
    }
    t->first[m] = u;
    t->n = m;
}

template <int DT>
__device__ void grid_chunk(const GArgs &a, int S, int chunk, int rb, int re, int lane,
                           const int64_t *koff) {
    const int G = groups_of(S), R = nchunk_of(S) * G;
    const int grp = lane / S, q = lane - grp * S;
    const bool active = grp < G;
    const int p0 = chunk * G + grp;
    const float rS = 1.0f / (float)S;
    const int H = (S - 1) >> 1, S2 = S * S, half = a.n >> 1, hb = a.beta >> 1;

    float acc_r[kSlots], acc_i[kSlots], cmp_r[kSlots], cmp_i[kSlots];
    int cur_y[kSlots];
#pragma unroll
    for (int m = 0; m < kSlots; ++m) {
        acc_r[m] = acc_i[m] = cmp_r[m] = cmp_i[m] = 0.f;
        cur_y[m] = -1;
    }
    int cur_x = -1;

    auto commit = [&](int m) {
        float *cell = a.grid + 2 * ((int64_t)cur_y[m] * a.n + cur_x);
        unsafeAtomicAdd(cell, acc_r[m] - cmp_r[m]);
        unsafeAtomicAdd(cell + 1, acc_i[m] - cmp_i[m]);
        acc_r[m] = acc_i[m] = cmp_r[m] = cmp_i[m] = 0.f;
    };

    for (int j = rb; j < re; ++j) {
        const int X = a.x[j], Y = a.y[j], k = a.plane[j];
        const int sigma = (a.ov[j] + hb - 1) * a.beta + (a.ou[j] + hb - 1);
        const float2 gam = a.gamma[j];
        const int ax = X + half - H, row0 = Y + half - H;
        const int64_t kbase = koff[k] + (int64_t)sigma * S2;
        // runs from wg_compress with the same geometry and table always pass; anything else
        // is skipped rather than read or written out of bounds
        if (ax < 0 || ax + S > a.n || row0 < 0 || row0 + S > a.n || kbase < 0 || kbase + S2 > a.data_cap)
            continue;
        const int am = mod_small(ax, S, rS), r0m = mod_small(row0, S, rS);
        int jj = q - am;
        jj += (jj < 0) ? S : 0;
        const int xc = ax + jj;
        if (active && xc != cur_x) {
#pragma unroll
            for (int m = 0; m < kSlots; ++m)
                if (cur_y[m] >= 0) {
                    commit(m);
                    cur_y[m] = -1;
                }
            cur_x = xc;
        }
        int p = p0;
        int ii = p0 - r0m;
        ii += (ii < 0) ? S : 0;
#pragma unroll
        for (int m = 0; m < kSlots; ++m) {
            if (active && p < S) {
                const int yc = row0 + ii;
                if (yc != cur_y[m]) {
                    if (cur_y[m] >= 0) commit(m);
                    cur_y[m] = yc;
                }
                const float2 kv = load_k<DT>(a.data, kbase + ii * S + jj);
                const float pr = fmaf(gam.x, kv.x, -(gam.y * kv.y));
                const float pi = fmaf(gam.x, kv.y, gam.y * kv.x);
                kahan_add(acc_r[m], cmp_r[m], pr);
                kahan_add(acc_i[m], cmp_i[m], pi);
            }
            p += R;
            ii += R;
            ii -= (ii >= S) ? S : 0;
        }
    }
    if (active) {
#pragma unroll
        for (int m = 0; m < kSlots; ++m)
            if (cur_y[m] >= 0) commit(m);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_grid(GArgs a) {
    __shared__ UnitTable ut;
    __shared__ int64_t koff[WG_MAX_PLANES + 1];
    if (threadIdx.x == 0) build_units(a.plan, true, &ut);
    for (int k = threadIdx.x; k <= a.n_w; k += blockDim.x) koff[k] = a.offset[k];
    __syncthreads();
    const int nunits = ut.first[ut.n];
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    for (int u = blockIdx.x * wpb + threadIdx.x / kWave; u < nunits; u += gridDim.x * wpb) {
        int m = 0;
        while (u >= ut.first[m + 1]) ++m;
        const int S = ut.S[m], nch = nchunk_of(S);
        const int rel = u - ut.first[m];
        const int item = rel / nch, chunk = rel - item * nch;
        const int slot = a.plan[kPlanOff + S] + item;
        grid_chunk<DT>(a, S, chunk, a.items[2 * slot], a.items[2 * slot + 1], lane, koff);
    }
}

// Adjoint: one wavefront per local chunk; per run the S x S dot product with conj(K) is
// accumulated per lane (Kahan), reduced across the wave, and broadcast to the run's records.
template <int DT>
__device__ void degrid_chunk(const GArgs &a, int S, int rb, int re, int lane, const int64_t *koff) {
    const int G = groups_of(S);
    const int grp = lane / S, q = lane - grp * S;
    const bool active = grp < G;
    const float rS = 1.0f / (float)S;
    const int H = (S - 1) >> 1, S2 = S * S, half = a.n >> 1, hb = a.beta >> 1;
    const int64_t seglen = (int64_t)a.nt * a.nc;
    const float2 *grid = (const float2 *)a.grid;
    for (int j = rb; j < re; ++j) {
        const int X = a.x[j], Y = a.y[j], k = a.plane[j];
        const int sigma = (a.ov[j] + hb - 1) * a.beta + (a.ou[j] + hb - 1);
        const int ax = X + half - H, row0 = Y + half - H;
        const int64_t kbase = koff[k] + (int64_t)sigma * S2;
        if (ax < 0 || ax + S > a.n || row0 < 0 || row0 + S > a.n || kbase < 0 || kbase + S2 > a.data_cap)
            continue;
        const int am = mod_small(ax, S, rS), r0m = mod_small(row0, S, rS);
        int jj = q - am;
        jj += (jj < 0) ? S : 0;
        float sr = 0.f, si = 0.f, cr = 0.f, ci = 0.f;
        if (active) {
            int ii = grp - r0m;
            ii += (ii < 0) ? S : 0;
            for (int p = grp; p < S; p += G) {
                const float2 kv = load_k<DT>(a.data, kbase + ii * S + jj);
                const float2 gv = grid[(int64_t)(row0 + ii) * a.n + ax + jj];
                const float pr = fmaf(kv.x, gv.x, kv.y * gv.y);
                const float pi = fmaf(kv.x, gv.y, -(kv.y * gv.x));
                kahan_add(sr, cr, pr);
                kahan_add(si, ci, pi);
                ii += G;
                ii -= (ii >= S) ? S : 0;
            }
        }
        const float dr = wave_sum(sr - cr), di = wave_sum(si - ci);
        const int r0 = a.start[j], n = a.len[j];
        for (int m = lane; m < n; m += kWave) {
            const int64_t r = (int64_t)r0 + m;
            if (r < 0 || r >= a.n_rec) break;
            const int64_t b = r / seglen;
            const int64_t t = r - (r / a.nt) * a.nt;
            const double wm = a.uvw[(b * a.nt + t) * 3 + 2];
            const float e = a.wt ? a.wt[r] : 1.0f;
            a.vis_out[r] = make_float2(e * dr, e * ((wm >= 0.0) ? di : -di));
        }
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_degrid(GArgs a) {
    __shared__ UnitTable ut;
    __shared__ int64_t koff[WG_MAX_PLANES + 1];
    if (threadIdx.x == 0) build_units(a.plan, false, &ut);
    for (int k = threadIdx.x; k <= a.n_w; k += blockDim.x) koff[k] = a.offset[k];
    __syncthreads();
    const int nunits = ut.first[ut.n];
    const int lane = threadIdx.x & (kWave - 1);
    const int wpb = blockDim.x / kWave;
    for (int u = blockIdx.x * wpb + threadIdx.x / kWave; u < nunits; u += gridDim.x * wpb) {
        int m = 0;
        while (u >= ut.first[m + 1]) ++m;
        const int S = ut.S[m];
        const int slot = a.plan[kPlanOff + S] + (u - ut.first[m]);
        degrid_chunk<DT>(a, S, a.items[2 * slot], a.items[2 * slot + 1], lane, koff);
    }
}

__global__ void k_zero(float2 *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float2(0.f, 0.f);
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
    a.items = runs->plan + plan_items_at();
    a.offset = kt->offset;
    a.data = kt->data;
    a.grid = nullptr;
    a.vis_out = nullptr;
    a.uvw = nullptr;
    a.wt = nullptr;
    return a;
}

int check_runs(const wg_runs *runs) {
    if (!runs || !runs->start || !runs->len || !runs->x || !runs->y || !runs->plane || !runs->ou ||
        !runs->ov || !runs->gamma || !runs->plan || runs->capacity < 1)
        return WG_EINVAL;
    return WG_OK;
}

constexpr int kPersistentBlocks = 4096;

}  // namespace
}  // namespace wg

extern "C" int wg_grid(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs, const wg_stats *stats,
                       float *grid, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_table(g, kt)) != WG_OK) return st;
    if ((st = check_runs(runs)) != WG_OK) return st;
    if (!grid || !stats) return WG_EINVAL;
    GArgs a = make_args(g, kt, runs);
    a.grid = grid;
    hipStream_t s = (hipStream_t)stream;
    switch (kt->dtype) {
    case WG_KF32: hipLaunchKernelGGL(k_grid<WG_KF32>, dim3(kPersistentBlocks), dim3(256), 0, s, a); break;
    case WG_KBF16: hipLaunchKernelGGL(k_grid<WG_KBF16>, dim3(kPersistentBlocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_grid<WG_KF16>, dim3(kPersistentBlocks), dim3(256), 0, s, a); break;
    }
    return launch_status();
}

extern "C" int wg_degrid(const wg_geom *g, const wg_ktable *kt, const wg_runs *runs, const wg_stats *stats,
                         const float *grid, const double *uvw, const float *weight, int64_t nb, int32_t nc,
                         int32_t nt, float *vis_out, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_table(g, kt)) != WG_OK) return st;
    if ((st = check_runs(runs)) != WG_OK) return st;
    if (!grid || !stats || !uvw || !vis_out || nb < 1 || nc < 1 || nt < 1) return WG_EINVAL;
    const int64_t n_rec = nb * (int64_t)nc * nt;
    if (n_rec > runs->capacity) return WG_ECAPACITY;
    GArgs a = make_args(g, kt, runs);
    a.grid = (float *)grid;
    a.vis_out = (float2 *)vis_out;
    a.uvw = uvw;
    a.wt = weight;
    a.nc = nc;
    a.nt = nt;
    a.n_rec = n_rec;
    hipStream_t s = (hipStream_t)stream;
    // records in no run get 0: clear the output first
    hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, s, (float2 *)vis_out, n_rec);
    switch (kt->dtype) {
    case WG_KF32: hipLaunchKernelGGL(k_degrid<WG_KF32>, dim3(kPersistentBlocks), dim3(256), 0, s, a); break;
    case WG_KBF16: hipLaunchKernelGGL(k_degrid<WG_KBF16>, dim3(kPersistentBlocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_degrid<WG_KF16>, dim3(kPersistentBlocks), dim3(256), 0, s, a); break;
    }
    return launch_status();
}
