// Image finaliser (Algorithm finalizer), one polarisation, on gfx950.
//
//   1. inverse 2-D FFT of the UV-grid: img[q][p] = sum_cells G[y][x] e^{+2 pi i ((x - N/2)(p - N/2)
//      + (y - N/2)(q - N/2)) / N}, so pixel [q][p] holds (l, m) = ((p - N/2), (q - N/2)) / (N du);
//   2. real part (each record is gridded once, at its w >= 0 representative of eq. conj) over
//      the normaliser N_p of eq. normalizer, giving Jy/beam;
//   3. division by the taper c(l) c(m) of sec. convgriddingmath (psi_0(3 pi, 2 l du)),
//      normalised to 1 at the centre;
//   4. division by sinc(pi l du / beta) sinc(pi m du / beta) (eq. coversampled).
// Pixels where the taper is zero (the first row and column, l or m = -FOV/2) are 0, and the
// whole image is 0 when the normaliser is 0 (nothing was gridded).
//
// Polarised grids ([P][n][n], P = 2 or 4): each polarisation is transformed on its own and
// divided by its normaliser, and the Stokes images are the real parts of the linear
// combinations given by the feed relations (XX = I + Q, XY = U + iV, YX = U - iV, YY = I - Q;
// RR = I + V, RL = Q + iU, LR = Q - iU, LL = I - V), accumulated pixel by pixel in FP32 as
// the polarisations are transformed one after the other.
//
// W-stacking (eq. stacking) adds, before step 2, the sum over the w-plane grids of their
// transforms times the plane's image-plane w-term correction exp(+2 pi i w_k (n - 1)),
// n = sqrt(1 - l^2 - m^2): the factor that the w-projection kernel of plane k carries
// (eq. C_W), applied after the transform instead of by the kernel.
//
// Layout of the work: row transforms (one workgroup per row, an N-point FP32 Stockham FFT in
// LDS with radix-16 passes in registers), a tiled transpose, row transforms again, and a
// tiled transposing pass that applies steps 2-4 while writing the image row-major. The
// ifftshift of the input and the fftshift of the output are index XORs with N/2.
#include <math.h>

#include "prolate.hpp"
#include "wg_common.hpp"

#pragma clang fp contract(off)

namespace wg {
namespace {

constexpr int kMaxImageN = 8192;  // one row of FP32 complex values in 64 KB of LDS

__device__ inline float2 fmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 faddc(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 fsubc(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// exp(+2 pi i j / 16), j < 8
constexpr float kC1 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508977173f;  // sin(pi/8)
constexpr float kH = 0.70710678118654752440f;

__device__ inline float2 rot16_inv(float2 d, int j) {
    switch (j) {
    case 0: return d;
    case 1: return fmulc(d, make_float2(kC1, kS1));
    case 2: return fmulc(d, make_float2(kH, kH));
    case 3: return fmulc(d, make_float2(kS1, kC1));
    case 4: return make_float2(-d.y, d.x);
    case 5: return fmulc(d, make_float2(-kS1, kC1));
    case 6: return fmulc(d, make_float2(-kH, kH));
    default: return fmulc(d, make_float2(-kC1, kS1));
    }
}

constexpr int bitrev_i(int k, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((k >> i) & 1) << (bits - 1 - i);
    return r;
}

// Inverse DFT (e^{+2 pi i}) of R <= 16 points starting at v[o], natural order in and out.
template <int R>
__device__ inline void idft_reg(float2 *v) {
    constexpr int bits = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int s0 = 0; s0 < R; s0 += 2 * h) {
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const float2 x = v[s0 + i], y = v[s0 + i + h];
                v[s0 + i] = faddc(x, y);
                v[s0 + i + h] = rot16_inv(fsubc(x, y), i * (16 / (2 * h)));
            }
        }
    }
    float2 t[R];
#pragma unroll
    for (int k = 0; k < R; ++k) t[k] = v[bitrev_i(k, bits)];
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = t[k];
}

// One radix-R pass of an N-point inverse Stockham FFT for the lane's 16 values: 16/R
// butterflies j = t + b*T (T = N/16 active threads). Butterfly j reads elements j + r*N/R
// (times exp(+2 pi i (j mod ns) r / (ns R))) and writes element r to (j - j mod ns) R +
// (j mod ns) + r ns. The pass reads from `in` (global, shifted) when first, else from LDS,
// and writes to `out` (global, shifted) when last, else back to LDS.
template <int R>
__device__ inline void ifft_pass(float2 *buf, const float2 *in, float2 *out, int n, int ns, bool first,
                                 bool last, bool active, const float2 *tw) {
    const int T = n >> 4, t = threadIdx.x, nb = n / R, half = n >> 1;
    float2 v[16];
    if (active) {
#pragma unroll
        for (int b = 0; b < 16 / R; ++b) {
            const int j = t + b * T, jm = j & (ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = j + r * nb;
                float2 x = first ? in[e ^ half] : buf[e];
                if (r > 0 && ns > 1) x = fmulc(x, tw[jm * r * (n / (ns * R))]);
                v[b * R + r] = x;
            }
            idft_reg<R>(v + b * R);
        }
    }
    if (!first) __syncthreads();  // every read of buf precedes the writes below
    if (active) {
#pragma unroll
        for (int b = 0; b < 16 / R; ++b) {
            const int j = t + b * T, jm = j & (ns - 1);
            const int d0 = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = d0 + r * ns;
                if (last)
                    out[e ^ half] = v[b * R + r];
                else
                    buf[e] = v[b * R + r];
            }
        }
    }
    __syncthreads();
}

// The passes of an N = 2^LG point transform with their radices fixed at compile time (the
// first pass takes the LG mod 4 leftover bits, the others radix 16), so that every array
// index and stride is a constant and the lane's 16 values stay in registers.
template <int LG, int PASS, int NS_LOG>
__device__ inline void ifft_passes(float2 *buf, const float2 *in, float2 *out, bool active, const float2 *tw) {
    constexpr int kBits = PASS == 0 && (LG & 3) ? (LG & 3) : 4;
    constexpr int kDone = NS_LOG + kBits;
    ifft_pass<1 << kBits>(buf, in, out, 1 << LG, 1 << NS_LOG, PASS == 0, kDone == LG, active, tw);
    if constexpr (kDone < LG) ifft_passes<LG, PASS + 1, kDone>(buf, in, out, active, tw);
}

// Rows of src (N x N complex, one grid plane) -> inverse transforms in dst; ifftshift on input
// and fftshift on output. blockDim >= N/16.
template <int LG>
__global__ __launch_bounds__(512) void k_ifft_rows(const float2 *__restrict__ src, float2 *__restrict__ dst,
                                                   const float2 *__restrict__ tw) {
    extern __shared__ float2 buf[];
    constexpr int n = 1 << LG;
    const float2 *in = src + (size_t)blockIdx.x * n;
    float2 *out = dst + (size_t)blockIdx.x * n;
    const bool active = (int)threadIdx.x < (n >> 4);
    ifft_passes<LG, 0, 0>(buf, in, out, active, tw);
}

using RowFft = void (*)(const float2 *, float2 *, const float2 *);

RowFft row_fft(int lg) {
    switch (lg) {
    case 4: return k_ifft_rows<4>;
    case 5: return k_ifft_rows<5>;
    case 6: return k_ifft_rows<6>;
    case 7: return k_ifft_rows<7>;
    case 8: return k_ifft_rows<8>;
    case 9: return k_ifft_rows<9>;
    case 10: return k_ifft_rows<10>;
    case 11: return k_ifft_rows<11>;
    case 12: return k_ifft_rows<12>;
    default: return k_ifft_rows<13>;
    }
}

// dst[c][r] = src[r][c] for an N x N complex matrix, 32 x 32 tiles through LDS.
__global__ void k_transpose(const float2 *__restrict__ src, float2 *__restrict__ dst, int n) {
    __shared__ float2 tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int i = threadIdx.y; i < 32; i += blockDim.y) {
        const int r = by + i, c = bx + threadIdx.x;
        if (r < n && c < n) tile[i][threadIdx.x] = src[(size_t)r * n + c];
    }
    __syncthreads();
    for (int i = threadIdx.y; i < 32; i += blockDim.y) {
        const int r = bx + i, c = by + threadIdx.x;
        if (r < n && c < n) dst[(size_t)r * n + c] = tile[threadIdx.x][i];
    }
}

// Twiddles exp(+2 pi i j / N), j < N, and the per-axis correction
// corr[p] = taper(2 (p - N/2) / N) / taper(0) * sinc(pi (p - N/2) / (N beta)).
__global__ void k_fin_setup(float2 *tw, double *corr, int n, int beta, TaperCoef tc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s, c;
    sincospi(2.0 * (double)j / (double)n, &s, &c);
    tw[j] = make_float2((float)c, (float)s);
    const double x = 2.0 * (double)(j - n / 2) / (double)n;
    const double y = (double)(j - n / 2) / ((double)n * (double)beta);
    const double sinc = (j == n / 2) ? 1.0 : sinpi(y) / (M_PI * y);
    corr[j] = taper(x, tc) / taper(0.0, tc) * sinc;
}

// Stokes coefficients of each polarisation: image s += Re(c[s][p] * T_p) / N_p.
struct StokesCoef {
    float re[4][4], im[4][4];
    int ns;
};

// acc[s][p][q] (+)= Re(c[s][pol] * T[p][q] * W) / normaliser[pol] for the Stokes images s, T
// the transformed, transposed grid of polarisation `pol`, W = exp(+2 pi i w (n - 1)) with
// w-stacking (0 where l^2 + m^2 > 1) and 1 otherwise; `first` writes. A zero normaliser
// adds 0.
__global__ void k_stokes_acc(const float2 *__restrict__ T, float *__restrict__ acc, int n,
                             const double *__restrict__ normaliser, int pol, StokesCoef c, int stacked, double du,
                             double w, int first) {
    const int64_t nn = (int64_t)n * n;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    const double np = normaliser[pol];
    const double inv = np != 0.0 ? 1.0 / np : 0.0;
    double tx = T[e].x, ty = T[e].y;
    if (stacked) {
        const int p = (int)(e / n), q = (int)(e - (int64_t)p * n);
        const double l = (double)(p - n / 2) / ((double)n * du), m = (double)(q - n / 2) / ((double)n * du);
        const double rr = 1.0 - l * l - m * m;
        double sn = 0.0, cs = 0.0;
        if (rr >= 0.0) sincospi(2.0 * w * (sqrt(rr) - 1.0), &sn, &cs);
        const double ux = tx * cs - ty * sn, uy = tx * sn + ty * cs;
        tx = ux;
        ty = uy;
    }
    for (int s = 0; s < c.ns; ++s) {
        const float v = (float)(((double)c.re[s][pol] * tx - (double)c.im[s][pol] * ty) * inv);
        float *a = acc + (size_t)s * nn + e;
        *a = first ? v : *a + v;
    }
}

__device__ inline float re_of(float2 v) { return v.x; }
__device__ inline float re_of(float v) { return v; }

// W-stacking: acc[p][q] (+)= Re(T[p][q] * exp(+2 pi i w (n - 1))) for plane k's transformed,
// transposed grid T (row p = l index, column q = m index); the first plane writes. The
// correction is 0 where l^2 + m^2 > 1 (no direction there).
__global__ void k_stack_acc(const float2 *__restrict__ T, float *__restrict__ acc, int n, double du, double w,
                            int first) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int p = (int)(e / n), q = (int)(e - (int64_t)p * n);
    const double l = (double)(p - n / 2) / ((double)n * du), m = (double)(q - n / 2) / ((double)n * du);
    const double rr = 1.0 - l * l - m * m;
    float v = 0.0f;
    if (rr >= 0.0) {
        double s, c;
        sincospi(2.0 * w * (sqrt(rr) - 1.0), &s, &c);
        const float2 t = T[e];
        v = (float)((double)t.x * c - (double)t.y * s);
    }
    acc[e] = first ? v : acc[e] + v;
}

// image[q][p] = Re(T[p][q]) / (normaliser * corr[q] * corr[p]) (0 where the product is 0 or
// the normaliser is 0), T the twice-transformed, transposed grid (or the w-stacking sum of
// real parts); 32 x 32 tiles.
template <typename In>
__global__ void k_fin_out(const In *__restrict__ T, const double *__restrict__ corr,
                          const double *__restrict__ normaliser, float *__restrict__ image, int n) {
    __shared__ float tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int i = threadIdx.y; i < 32; i += blockDim.y) {
        const int r = by + i, c = bx + threadIdx.x;  // T row r = l index p, column c = m index q
        if (r < n && c < n) tile[i][threadIdx.x] = re_of(T[(size_t)r * n + c]);
    }
    __syncthreads();
    const double norm = normaliser ? *normaliser : 1.0;  // NULL: the input is normalised
    for (int i = threadIdx.y; i < 32; i += blockDim.y) {
        const int q = bx + i, p = by + threadIdx.x;
        if (q < n && p < n) {
            const double d = norm * corr[q] * corr[p];
            image[(size_t)q * n + p] = d != 0.0 ? (float)((double)tile[threadIdx.x][i] / d) : 0.0f;
        }
    }
}

struct FinLayout {
    size_t a, b, acc, tw, corr, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FinLayout fin_layout(int n, int npol) {
    FinLayout l;
    const size_t nn = (size_t)n * n;
    l.a = 0;
    l.b = align256(l.a + sizeof(float2) * nn);
    l.acc = align256(l.b + sizeof(float2) * nn);
    l.tw = align256(l.acc + sizeof(float) * nn * npol);
    l.corr = align256(l.tw + sizeof(float2) * n);
    l.total = align256(l.corr + sizeof(double) * n);
    return l;
}

int image_lg(int n) {
    if (n < 16 || n > kMaxImageN || (n & (n - 1))) return -1;
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    return lg;
}

}  // namespace
}  // namespace wg

extern "C" int wg_finalise_ws_bytes(const wg_geom *g, size_t *ws_bytes) {
    using namespace wg;
    const int st = check_geom(g);
    if (st != WG_OK) return st;
    if (!ws_bytes) return WG_EINVAL;
    if (image_lg(g->n) < 0) return WG_EUNSUPPORTED;
    *ws_bytes = fin_layout(g->n, npol_of(g)).total;
    return WG_OK;
}

namespace wg {
namespace {

// Coefficients of the Stokes images (feed relations above), in the order I, Q, U, V of those
// the polarisations give.
StokesCoef stokes_coef(int npol, bool circular) {
    StokesCoef c;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) c.re[i][j] = c.im[i][j] = 0.f;
    if (npol == 2) {  // (XX, YY) -> I, Q; (RR, LL) -> I, V
        c.ns = 2;
        c.re[0][0] = c.re[0][1] = 0.5f;
        c.re[1][0] = 0.5f;
        c.re[1][1] = -0.5f;
    } else {  // four products -> I, Q, U, V
        c.ns = 4;
        c.re[0][0] = c.re[0][3] = 0.5f;  // I
        if (!circular) {
            c.re[1][0] = 0.5f;  // Q = (XX - YY) / 2
            c.re[1][3] = -0.5f;
            c.re[2][1] = c.re[2][2] = 0.5f;  // U = (XY + YX) / 2
            c.im[3][1] = -0.5f;  // V = -i (XY - YX) / 2
            c.im[3][2] = 0.5f;
        } else {
            c.re[1][1] = c.re[1][2] = 0.5f;  // Q = (RL + LR) / 2
            c.im[2][1] = -0.5f;  // U = -i (RL - LR) / 2
            c.im[2][2] = 0.5f;
            c.re[3][0] = 0.5f;  // V = (RR - LL) / 2
            c.re[3][3] = -0.5f;
        }
    }
    return c;
}

// Both finalisers: one grid (stacked = false) or the n_w w-plane grids of w-stacking.
int finalise(const wg_geom *g, const float *grid, const double *normaliser, float *image, void *ws,
             size_t ws_bytes, wg_stream_t stream, bool stacked) {
    const int st = check_geom(g);
    if (st != WG_OK) return st;
    if (!grid || !normaliser || !image || !ws) return WG_EINVAL;
    if (stacked && !(g->flags & WG_W_STACKING)) return WG_EINVAL;
    const int n = g->n, lg = image_lg(n);
    if (lg < 0) return WG_EUNSUPPORTED;
    const int npol = npol_of(g);
    const FinLayout lay = fin_layout(n, npol);
    if (ws_bytes < lay.total) return WG_ECAPACITY;
    char *base = (char *)ws;
    float2 *A = (float2 *)(base + lay.a), *B = (float2 *)(base + lay.b), *tw = (float2 *)(base + lay.tw);
    double *corr = (double *)(base + lay.corr);
    hipStream_t s = (hipStream_t)stream;

    TaperCoef tc;
    prolate_coefficients(kTaperC, &tc);
    const int threads = n / 16 > 64 ? n / 16 : 64;
    const RowFft rows = row_fft(lg);
    const size_t lds = sizeof(float2) * (size_t)n;
    const dim3 tiles((n + 31) / 32, (n + 31) / 32), tb(32, 8);
    hipLaunchKernelGGL(k_fin_setup, dim3((n + 255) / 256), dim3(256), 0, s, tw, corr, n, g->beta, tc);
    const int64_t nn = (int64_t)n * n;
    float *acc = (float *)(base + lay.acc);
    if (npol > 1) {
        // polarised grids ([P][n][n], or [n_w][P][n][n] stacked): every (plane, product)
        // transform adds its share to the Stokes accumulators
        StokesCoef c = stokes_coef(npol, (g->flags & WG_POL_CIRCULAR) != 0);
        const int planes = stacked ? g->n_w : 1;
        for (int k = 0; k < planes; ++k) {
            const double q = g->n_w > 1 ? (double)k / (double)(g->n_w - 1) : 0.0;
            const double w = stacked ? g->w_max * (q * q) : 0.0;
            for (int p = 0; p < npol; ++p) {
                const float2 *G = (const float2 *)grid + ((size_t)k * npol + p) * nn;
                hipLaunchKernelGGL(rows, dim3(n), dim3(threads), lds, s, G, A, tw);
                hipLaunchKernelGGL(k_transpose, tiles, tb, 0, s, A, B, n);
                hipLaunchKernelGGL(rows, dim3(n), dim3(threads), lds, s, B, A, tw);
                hipLaunchKernelGGL(k_stokes_acc, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, A, acc, n,
                                   normaliser, p, c, stacked ? 1 : 0, g->du, w, (k == 0 && p == 0) ? 1 : 0);
            }
        }
        for (int k = 0; k < c.ns; ++k)
            hipLaunchKernelGGL(k_fin_out<float>, tiles, tb, 0, s, (const float *)(acc + (size_t)k * nn), corr,
                               (const double *)nullptr, image + (size_t)k * nn, n);
        return launch_status();
    }
    const int planes = stacked ? g->n_w : 1;
    for (int k = 0; k < planes; ++k) {
        const float2 *G = (const float2 *)grid + (size_t)k * nn;
        hipLaunchKernelGGL(rows, dim3(n), dim3(threads), lds, s, G, A, tw);
        hipLaunchKernelGGL(k_transpose, tiles, tb, 0, s, A, B, n);
        hipLaunchKernelGGL(rows, dim3(n), dim3(threads), lds, s, B, A, tw);
        if (stacked) {
            // the plane's w, computed as the table generator places its planes
            const double q = g->n_w > 1 ? (double)k / (double)(g->n_w - 1) : 0.0;
            const double w = g->w_max * (q * q);
            hipLaunchKernelGGL(k_stack_acc, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, A, acc, n, g->du, w,
                               k == 0 ? 1 : 0);
        }
    }
    if (stacked)
        hipLaunchKernelGGL(k_fin_out<float>, tiles, tb, 0, s, (const float *)acc, corr, normaliser, image, n);
    else
        hipLaunchKernelGGL(k_fin_out<float2>, tiles, tb, 0, s, A, corr, normaliser, image, n);
    return launch_status();
}

}  // namespace
}  // namespace wg

extern "C" int wg_finalise(const wg_geom *g, const float *grid, const double *normaliser, float *image, void *ws,
                           size_t ws_bytes, wg_stream_t stream) {
    return wg::finalise(g, grid, normaliser, image, ws, ws_bytes, stream, false);
}

extern "C" int wg_finalise_stacked(const wg_geom *g, const float *grids, const double *normaliser, float *image,
                                   void *ws, size_t ws_bytes, wg_stream_t stream) {
    return wg::finalise(g, grids, normaliser, image, ws, ws_bytes, stream, true);
}
