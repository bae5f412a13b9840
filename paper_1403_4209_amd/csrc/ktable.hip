// Convolution-function table on the GPU (Convolution Function Generator, Algorithm convgen).
//
// Per w-plane: evaluate the image-plane function (separable prolate spheroidal taper times
// the inverse w-screen) on m_img x m_img samples, zero-pad to L = beta*m_img, apply a
// forward 2-D DFT (row pass, then column pass), normalise by the w=0 plane's centre value,
// find the natural support from the 1e-3 magnitude threshold, then trim/reorder into one
// S x S matrix per oversample offset pair, round to the table's storage type and sum real
// parts (eq. sum).
//
// Each L-point transform of a zero-padded line of M samples x[n], n in [-M/2, M/2), is
// computed as beta transforms of M points: X[beta*k1 + b] = sum_n (x[n] w_L^(n b)) w_M^(n k1)
// with w_N = exp(-2 pi i / N). The M-point transforms are Stockham auto-sort FFTs whose
// passes (radix 16, and one radix-2/4/8 pass when log2 M is not a multiple of 4) run in
// registers and exchange through LDS between passes.
//
// The prolate spheroidal taper psi_0(3 pi, x) comes from prolate.hpp.
#include <math.h>
#include <string.h>

#include <vector>

#include "prolate.hpp"
#include "wg_common.hpp"

#pragma clang fp contract(off)

namespace wg {
namespace {

constexpr double kThreshold = 1e-3;


struct BuildArgs {
    int M, L, lgM, beta, n_w, Wf, W, dtype;
    double du, w_max;
    const double2 *tw;
    double2 *A;    // [n_w][L][M]  row-pass output, column-major per plane
    double2 *win;  // [n_w][W][W]  normalised central window
    double *c00;
    int *kmax;
    double *tap;   // [M] taper at the image samples
};

// Work index of block b in a launch of `total` blocks: blocks are dealt to the 8 XCDs in
// turn, so XCD x takes the x-th eighth of the work range (neighbouring lines and columns,
// whose values share cache lines, then meet in one L2); the last total % 8 blocks keep
// their own index.
__device__ inline int xcd_work_index(int b, int total) {
    const int q = total >> 3;
    return b >= 8 * q ? b : (b & 7) * q + (b >> 3);
}

__device__ inline double plane_w(int k, int n_w, double w_max) {
    if (n_w == 1) return 0.0;
    double q = (double)k / (double)(n_w - 1);
    return w_max * (q * q);
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// exp(-2 pi i j / 16), j < 8: cos and sin of multiples of pi/8
constexpr double kCos1 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kSin1 = 0.38268343236508977173;  // sin(pi/8)
constexpr double kHalfRt2 = 0.70710678118654752440;

// d * exp(-2 pi i j / 16) for a compile-time j after unrolling
__device__ inline double2 rot16(double2 d, int j) {
    switch (j) {
    case 0: return d;
    case 1: return cmul(d, make_double2(kCos1, -kSin1));
    case 2: return cmul(d, make_double2(kHalfRt2, -kHalfRt2));
    case 3: return cmul(d, make_double2(kSin1, -kCos1));
    case 4: return make_double2(d.y, -d.x);
    case 5: return cmul(d, make_double2(-kSin1, -kCos1));
    case 6: return cmul(d, make_double2(-kHalfRt2, -kHalfRt2));
    default: return cmul(d, make_double2(-kCos1, -kSin1));
    }
}

constexpr int bitrev_c(int k, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((k >> i) & 1) << (bits - 1 - i);
    return r;
}

// Forward DFT of R <= 16 points in registers, natural order in and out (radix-2
// decimation in frequency, then the bit-reversal permutation).
template <int R>
__device__ inline void dft_reg(double2 (&v)[R]) {
    constexpr int bits = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int s0 = 0; s0 < R; s0 += 2 * h) {
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const double2 x = v[s0 + i], y = v[s0 + i + h];
                v[s0 + i] = cadd(x, y);
                v[s0 + i + h] = rot16(csub(x, y), i * (16 / (2 * h)));
            }
        }
    }
    double2 t[R];
#pragma unroll
    for (int k = 0; k < R; ++k) t[k] = v[bitrev_c(k, bits)];
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = t[k];
}

// One radix-R Stockham pass over nsub independent M-point transforms. ns is the product of
// the radices of the earlier passes. Butterfly j of a transform reads elements j + r*M/R,
// multiplies element r by exp(-2 pi i (j mod ns) r / (ns R)), transforms, and writes
// element r to (j - j mod ns) R + (j mod ns) + r ns. ld(b, e) and st(b, e, v) access
// element e of transform b.
template <int R, class Ld, class St>
__device__ inline void stockham_pass(int M, int nsub, int ns, int L, const double2 *__restrict__ tw, Ld ld, St st) {
    const int nb = M / R;
    const int step = L / (ns * R);
    for (int t = threadIdx.x; t < nsub * nb; t += blockDim.x) {
        const int b = t / nb, j = t - b * nb;
        const int jm = j & (ns - 1);
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r] = ld(b, j + r * nb);
            if (r > 0 && ns > 1) v[r] = cmul(v[r], tw[jm * r * step]);
        }
        dft_reg<R>(v);
        const int d0 = (j - jm) * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) st(b, d0 + r * ns, v[r]);
    }
}

// Passes of an M-point transform (M = 2^lgM): radix 2^(lgM mod 4) first when lgM is not a
// multiple of 4, radix 16 after that.
__host__ __device__ inline int n_passes(int lgM) { return (lgM + 3) / 4; }

// The L = beta*M outputs of the zero-padded transform of the centred line x (M values in
// LDS or global memory, x[n + M/2] = sample n): first(b, e) = x[n] w_L^(n b) feeds the first
// pass, out(b, k1, v) receives X[beta*k1 + b]. buf0 and buf1 hold beta*M values each in LDS
// (buf1 only with three or more passes; it may alias x, which the first pass alone reads).
// Pass PASS of the M = 2^LGM point transforms, its radix fixed at compile time (the first
// pass takes the LGM mod 4 leftover bits, the others radix 16), then the passes after it.
template <int LGM, int PASS, int NS_LOG, class First, class Out>
__device__ inline void dft_passes(const BuildArgs &a, const double2 *src, double2 *dst, double2 *buf0, double2 *buf1,
                                  First first, Out out) {
    constexpr int kBits = PASS == 0 && (LGM & 3) ? (LGM & 3) : 4;
    constexpr int kDone = NS_LOG + kBits;
    constexpr bool kLast = kDone == LGM;
    constexpr int M = 1 << LGM, R = 1 << kBits, ns = 1 << NS_LOG;
    // exchange positions swizzled within each 16 x 16 block of a transform: a radix-16
    // pass stores its outputs 16 apart, which would put 16 neighbouring lanes on one LDS bank
    auto swz = [](int e) { return e ^ ((e >> 4) & 15); };
    auto lds_ld = [&](int b, int e) { return src[b * M + swz(e)]; };
    auto lds_st = [&](int b, int e, double2 v) { dst[b * M + swz(e)] = v; };
    if constexpr (PASS == 0 && kLast)
        stockham_pass<R>(M, a.beta, ns, a.L, a.tw, first, out);
    else if constexpr (PASS == 0)
        stockham_pass<R>(M, a.beta, ns, a.L, a.tw, first, lds_st);
    else if constexpr (kLast)
        stockham_pass<R>(M, a.beta, ns, a.L, a.tw, lds_ld, out);
    else
        stockham_pass<R>(M, a.beta, ns, a.L, a.tw, lds_ld, lds_st);
    __syncthreads();
    if constexpr (!kLast)
        dft_passes<LGM, PASS + 1, kDone>(a, dst, dst == buf0 ? buf1 : buf0, buf0, buf1, first, out);
}

template <int LGM, class Out>
__device__ void oversampled_dft(const BuildArgs &a, const double2 *x, double2 *buf0, double2 *buf1, Out out) {
    constexpr int M = 1 << LGM;
    const int L = a.L;
    const double2 *tw = a.tw;
    auto first = [&](int b, int e) {
        const int n = e - ((e >= M / 2) ? M : 0);
        return cmul(x[(e + M / 2) & (M - 1)], tw[(n * b) & (L - 1)]);
    };
    dft_passes<LGM, 0, 0>(a, nullptr, buf0, buf0, buf1, first, out);
}

__global__ void k_twiddle(double2 *tw, int L) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < L) {
        double s, c;
        sincospi(-2.0 * (double)j / (double)L, &s, &c);
        tw[j] = make_double2(c, s);
    }
}

// The taper at the M image samples, x_p = 2(p - M/2)/M.
__global__ void k_taper(BuildArgs a, TaperCoef tc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < a.M) a.tap[p] = taper(2.0 * (double)(p - a.M / 2) / (double)a.M, tc);
}

// LDS of the row and column kernels: beta*M values of buf0, then max(M, beta*M when a
// second exchange buffer is needed) values of the input line / buf1.
inline size_t dft_lds_bytes(int M, int L, int lgM) {
    return sizeof(double2) * (size_t)(L + (n_passes(lgM) >= 3 ? L : M));
}

// LDS of the column kernel: with two passes it reads its column from global memory and
// needs buf0 alone (beta*M values: 32 KB at M = 256, five blocks per CU); with three or
// more, as the row kernel.
inline size_t col_lds_bytes(int M, int L, int lgM) {
    return n_passes(lgM) >= 3 ? dft_lds_bytes(M, L, lgM) : sizeof(double2) * (size_t)L;
}

// Row pass: image row q of plane k -> L-point transform along u; stores the centred
// spectrum column-major so the column pass reads contiguous values.
//
// The image-plane function is even in l and in m on the sample grid, bit for bit: the taper
// is a series of even Legendre polynomials, the w-screen depends on l^2 and m^2, and the one
// unpaired sample (x = -1) has taper 0. So row M - q equals row q, row 0 is zero, and each row
// transform is even in u. Only rows q >= M/2 are transformed (each stored also as row M - q)
// and only the columns the column pass reads (u >= 0 and the Nyquist column -L/2) are stored.
template <int LGM>
__global__ __launch_bounds__(128) void k_rows(BuildArgs a) {
    extern __shared__ double2 lds[];
    double2 *buf0 = lds, *xin = lds + a.L;
    const int t = xcd_work_index((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    const int q = a.M / 2 + t % (int)gridDim.x, k = t / (int)gridDim.x;
    const double xq = 2.0 * (double)(q - a.M / 2) / (double)a.M;
    const double m = xq / (2.0 * a.du);
    const double tq = a.tap[q];
    const double w = plane_w(k, a.n_w, a.w_max);
    for (int p = threadIdx.x; p < a.M; p += blockDim.x) {
        const double xp = 2.0 * (double)(p - a.M / 2) / (double)a.M;
        const double l = xp / (2.0 * a.du);
        const double tp = a.tap[p];
        const double rr = (1.0 - l * l) - m * m;
        double2 v = make_double2(0.0, 0.0);
        if (rr >= 0.0) {
            const double nm1 = sqrt(rr) - 1.0;
            const double th = (2.0 * M_PI * w) * nm1;
            double sn, cs;
            sincos(th, &sn, &cs);
            const double t2 = tq * tp;
            v = make_double2(t2 * cs, t2 * sn);
        }
        xin[p] = v;
    }
    __syncthreads();
    double2 *plane = a.A + (size_t)k * a.L * a.M;
    const int L = a.L, M = a.M, beta = a.beta;
    oversampled_dft<LGM>(a, xin, buf0, xin, [&](int b, int k1, double2 v) {
        const int cu = (k1 * beta + b + L / 2) & (L - 1);
        if (cu != 0 && cu < L / 2) return;  // u < 0: the column pass uses the mirror column
        double2 *col = plane + (size_t)cu * M;
        col[q] = v;
        if (q > M / 2)
            col[M - q] = v;
        else
            col[0] = make_double2(0.0, 0.0);  // row 0 (taper zero), written once per column
    });
}

__global__ void k_c00_and_reset(BuildArgs a, double *wbound) {
    __shared__ double red[256];
    // lower |w| edge of every plane: nearest plane in sqrt(w)
    for (int j = threadIdx.x; j < a.n_w; j += blockDim.x) {
        double wb = 0.0;
        if (j > 0) {
            const double q = ((double)j - 0.5) / (double)(a.n_w - 1);
            wb = a.w_max * (q * q);
        }
        wbound[j] = wb;
    }
    double acc = 0.0;
    const double2 *col = a.A + (size_t)(a.L / 2) * a.M;  // plane 0, zero frequency in u
    for (int q = threadIdx.x; q < a.M; q += blockDim.x) acc += col[q].x;
    red[threadIdx.x] = acc;
    for (int k = threadIdx.x; k < a.n_w; k += blockDim.x) a.kmax[k] = 0;
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *a.c00 = red[0];
}

// Column pass for column cu of plane k: transform along v, normalise, support search over
// the whole plane, and keep the central window the matrices are cut from. The plane is even
// in u (see the row pass): columns u >= 0 and the Nyquist column -L/2 are transformed, and
// each window column u > 0 is stored also as column -u.
//
// The support test |C/c00| > 1e-3 is decided on |C|^2 against (1e-3 c00)^2 wherever the two
// differ by more than a relative 1e-9 (far beyond the rounding of either side); only values
// closer than that take the exact quotient and hypot, so every decision equals the exact one.
template <int LGM>
__global__ __launch_bounds__(128) void k_cols(BuildArgs a) {
    extern __shared__ double2 lds[];
    constexpr bool kStage = (LGM + 3) / 4 >= 3;  // three or more passes: the column goes to LDS
    double2 *buf0 = lds, *xin = lds + a.L;
    const int t = xcd_work_index((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    const int bx = t % (int)gridDim.x, k = t / (int)gridDim.x;
    const int fu_b = bx == a.L / 2 ? -a.L / 2 : bx;
    const int cu = fu_b + a.L / 2;
    const double2 *in = a.A + ((size_t)k * a.L + cu) * a.M;
    if constexpr (kStage) {
        for (int q = threadIdx.x; q < a.M; q += blockDim.x) xin[q] = in[q];
        __syncthreads();
    }
    const double c00 = *a.c00;
    const double t2 = (kThreshold * c00) * (kThreshold * c00);
    const double t2_hi = t2 * (1.0 + 1e-9), t2_lo = t2 * (1.0 - 1e-9);
    const int fu = cu - a.L / 2;
    const bool keep_u = fu >= -a.Wf && fu <= a.Wf;
    const int L = a.L, beta = a.beta, Wf = a.Wf, W = a.W;
    double2 *win = a.win + (size_t)k * W * W + (fu + Wf);
    const int mirror = -2 * fu;  // column -fu relative to column fu
    int dmax = 0;
    oversampled_dft<LGM>(a, kStage ? xin : in, buf0, xin, [&](int b, int k1, double2 s) {
        const int fv = ((k1 * beta + b + L / 2) & (L - 1)) - L / 2;
        const double r2 = s.x * s.x + s.y * s.y;
        bool above = r2 > t2_hi;
        if (!above && r2 >= t2_lo) above = hypot(s.x / c00, s.y / c00) > kThreshold;
        if (above) dmax = max(dmax, max(abs(fu), abs(fv)));
        if (keep_u && fv >= -Wf && fv <= Wf) {
            const double2 v = make_double2(s.x / c00, s.y / c00);
            win[(size_t)(fv + Wf) * W] = v;
            if (fu > 0) win[(size_t)(fv + Wf) * W + mirror] = v;
        }
    });
    // the transform ended with a barrier: its LDS now holds the block's maxima
    int *red = (int *)lds;
    red[threadIdx.x] = dmax;
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + d]);
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > 0) atomicMax(&a.kmax[k], red[0]);
}

// Supports from the natural support (1e-3 threshold) and the configured law, and plane
// offsets in complex elements.
__global__ void k_supports(BuildArgs a, int s_lo, int s_hi, int32_t *support, int64_t *offset) {
    if (threadIdx.x != 0) return;
    int64_t acc = 0;
    for (int k = 0; k < a.n_w; ++k) {
        const int over = a.kmax[k] - a.beta / 2;
        const int r = over <= 0 ? 0 : (over + a.beta - 1) / a.beta;
        const int snat = 2 * r + 1;
        const int law = a.n_w == 1 ? s_lo : s_lo + 2 * (((s_hi - s_lo) * k + (a.n_w - 1)) / (2 * (a.n_w - 1)));
        const int S = min(s_hi, max(snat, law));
        support[k] = S;
        offset[k] = acc;
        acc += (int64_t)a.beta * a.beta * S * (S + 2 * pad_of(a.dtype));
    }
    offset[a.n_w] = acc;
}

// Round-to-nearest-even of an FP64 value to a format with `sig` significant bits and
// smallest quantum 2^qmin; returns the rounded value (exactly representable).
__device__ inline double round_sig(double x, int sig, int qmin) {
    if (!(x != 0.0) || isinf(x) || isnan(x)) return x;
    const int e = ilogb(x);
    const int qe = max(e - (sig - 1), qmin);
    return ldexp(rint(ldexp(x, -qe)), qe);
}

__device__ inline uint16_t to_bf16_bits(double x, double *rounded) {
    double r = round_sig(x, 8, -133);
    if (fabs(r) > 0x1.FEp127) r = copysign(INFINITY, r);
    *rounded = r;
    const float f = (float)r;  // exact
    return (uint16_t)(__float_as_uint(f) >> 16);
}

__device__ inline uint16_t to_f16_bits(double x, double *rounded) {
    double r = round_sig(x, 11, -24);
    if (fabs(r) > 65504.0) r = copysign(INFINITY, r);
    *rounded = r;
    const _Float16 h = (_Float16)(float)r;  // exact
    uint16_t bits;
    memcpy(&bits, &h, 2);
    return bits;
}

__global__ void k_slices(BuildArgs a, const int32_t *__restrict__ support,
                         const int64_t *__restrict__ offset, void *data, double *zeta) {
    __shared__ double red[256];
    const int t = xcd_work_index((int)(blockIdx.y * gridDim.x + blockIdx.x), (int)(gridDim.x * gridDim.y));
    const int sigma = t % (int)gridDim.x, k = t / (int)gridDim.x;
    const int beta = a.beta;
    const int ov = sigma / beta - beta / 2 + 1, ou = sigma % beta - beta / 2 + 1;
    const int P = pad_of(a.dtype);
    const int S = support[k], H = (S - 1) / 2, W = S + 2 * P;
    const int64_t base = offset[k] + (int64_t)sigma * S * W;
    double acc = 0.0;
    // rows of S + 2P values (P = 1 for FP32, 3 for 16-bit): column j of the matrix at
    // position P + j, with columns S - P..S - 1 repeated before the row and 0..P - 1 after
    // it, so that P + 1 neighbouring columns of a row, read forwards or (for a mirrored
    // matrix) backwards, are adjacent also where they wrap; zeta sums the S columns once.
    // (Positions wrap only by less than one row: P < S, or P >= S only for S = 1, where
    // every position holds the single column.)
    for (int e = threadIdx.x; e < S * W; e += blockDim.x) {
        const int i = e / W, jw = e - (e / W) * W;
        int j = jw - P;
        while (j < 0) j += S;
        while (j >= S) j -= S;
        const bool counted = jw >= P && jw < P + S;
        const int fv = (i - H) * beta - ov, fu = (j - H) * beta - ou;
        const double2 v = a.win[((size_t)k * a.W + (fv + a.Wf)) * a.W + (fu + a.Wf)];
        if (a.dtype == WG_KF32) {
            const float2 f = make_float2((float)v.x, (float)v.y);
            ((float2 *)data)[base + e] = f;
            if (counted) acc += (double)f.x;
        } else if (a.dtype == WG_KBF16) {
            double rr, ri;
            const uint32_t lo = to_bf16_bits(v.x, &rr), hi = to_bf16_bits(v.y, &ri);
            ((uint32_t *)data)[base + e] = lo | (hi << 16);
            if (counted) acc += rr;
        } else {
            double rr, ri;
            const uint32_t lo = to_f16_bits(v.x, &rr), hi = to_f16_bits(v.y, &ri);
            ((uint32_t *)data)[base + e] = lo | (hi << 16);
            if (counted) acc += rr;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) zeta[(size_t)k * beta * beta + sigma] = red[0];
}

struct WsLayout {
    size_t tw, A, win, c00, kmax, tap, total;
    int L, Wf, W;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout ws_layout(const wg_geom *g) {
    WsLayout w;
    w.L = g->beta * g->m_img;
    w.Wf = (g->s_hi - 1) / 2 * g->beta + g->beta / 2;
    w.W = 2 * w.Wf + 1;
    size_t o = 0;
    w.tw = o;
    o = align256(o + sizeof(double2) * w.L);
    w.A = o;
    o = align256(o + sizeof(double2) * (size_t)g->n_w * w.L * g->m_img);
    w.win = o;
    o = align256(o + sizeof(double2) * (size_t)g->n_w * w.W * w.W);
    w.c00 = o;
    o = align256(o + sizeof(double));
    w.kmax = o;
    o = align256(o + sizeof(int) * g->n_w);
    w.tap = o;
    o = align256(o + sizeof(double) * g->m_img);
    w.total = o;
    return w;
}


}  // namespace
}  // namespace wg

namespace wg {
namespace {

// The row (ROWS) or column kernel for M = 2^lgM image samples (16..1024).
template <bool ROWS>
void (*line_kernel(int lgM))(BuildArgs) {
    switch (lgM) {
    case 4: return ROWS ? k_rows<4> : k_cols<4>;
    case 5: return ROWS ? k_rows<5> : k_cols<5>;
    case 6: return ROWS ? k_rows<6> : k_cols<6>;
    case 7: return ROWS ? k_rows<7> : k_cols<7>;
    case 8: return ROWS ? k_rows<8> : k_cols<8>;
    case 9: return ROWS ? k_rows<9> : k_cols<9>;
    default: return ROWS ? k_rows<10> : k_cols<10>;
    }
}

}  // namespace
}  // namespace wg

extern "C" int wg_ktable_sizes(const wg_geom *g, int64_t *data_elems_max, size_t *ws_bytes) {
    int st = wg::check_geom(g);
    if (st != WG_OK) return st;
    if (!data_elems_max || !ws_bytes) return WG_EINVAL;
    *data_elems_max = (int64_t)g->n_w * g->beta * g->beta * g->s_hi * (g->s_hi + 2 * wg::kPadMax);
    *ws_bytes = wg::ws_layout(g).total;
    return WG_OK;
}

extern "C" int wg_ktable_build(const wg_geom *g, wg_ktable *kt, void *ws, size_t ws_bytes,
                               int32_t *support_out, int64_t *offset_out, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if (!kt || !ws || kt->dtype < WG_KF32 || kt->dtype > WG_KF16) return WG_EINVAL;
    if (kt->n_w != g->n_w || kt->beta != g->beta) return WG_EINVAL;
    if (!kt->support || !kt->offset || !kt->wbound || !kt->zeta || !kt->data) return WG_EINVAL;
    const WsLayout lay = ws_layout(g);
    if (ws_bytes < lay.total) return WG_ECAPACITY;
    hipStream_t s = (hipStream_t)stream;

    TaperCoef tc;
    prolate_coefficients(kTaperC, &tc);

    char *base = (char *)ws;
    BuildArgs a;
    a.M = g->m_img;
    a.L = lay.L;
    a.lgM = 0;
    while ((1 << a.lgM) < a.M) ++a.lgM;
    a.beta = g->beta;
    a.n_w = g->n_w;
    a.Wf = lay.Wf;
    a.W = lay.W;
    a.dtype = kt->dtype;
    a.du = g->du;
    a.w_max = g->w_max;
    a.tw = (const double2 *)(base + lay.tw);
    a.A = (double2 *)(base + lay.A);
    a.win = (double2 *)(base + lay.win);
    a.c00 = (double *)(base + lay.c00);
    a.kmax = (int *)(base + lay.kmax);
    a.tap = (double *)(base + lay.tap);

    const size_t lds = dft_lds_bytes(a.M, a.L, a.lgM);
    hipLaunchKernelGGL(k_twiddle, dim3((a.L + 255) / 256), dim3(256), 0, s, (double2 *)a.tw, a.L);
    hipLaunchKernelGGL(k_taper, dim3((a.M + 255) / 256), dim3(256), 0, s, a, tc);
    hipLaunchKernelGGL(line_kernel<true>(a.lgM), dim3(a.M / 2, a.n_w), dim3(128), lds, s, a);
    hipLaunchKernelGGL(k_c00_and_reset, dim3(1), dim3(256), 0, s, a, kt->wbound);
    hipLaunchKernelGGL(line_kernel<false>(a.lgM), dim3(a.L / 2 + 1, a.n_w), dim3(128), col_lds_bytes(a.M, a.L, a.lgM),
                       s, a);
    hipLaunchKernelGGL(k_supports, dim3(1), dim3(64), 0, s, a, g->s_lo, g->s_hi, kt->support, kt->offset);
    if (hipGetLastError() != hipSuccess) return WG_EHIP;

    // With room for every plane at s_hi and no host copies requested, nothing waits: the
    // matrices are cut on the device right away and s_max reports the upper bound s_hi.
    const int64_t cap_max = (int64_t)g->n_w * g->beta * g->beta * g->s_hi * (g->s_hi + 2 * wg::pad_of(kt->dtype));
    const bool sync = support_out || offset_out || kt->data_cap < cap_max;
    if (sync) {
        std::vector<int32_t> sup(g->n_w);
        std::vector<int64_t> off(g->n_w + 1);
        WG_HIP_CHECK(hipMemcpyAsync(sup.data(), kt->support, sizeof(int32_t) * g->n_w, hipMemcpyDeviceToHost, s));
        WG_HIP_CHECK(hipMemcpyAsync(off.data(), kt->offset, sizeof(int64_t) * (g->n_w + 1), hipMemcpyDeviceToHost, s));
        WG_HIP_CHECK(hipStreamSynchronize(s));
        if (off[g->n_w] > kt->data_cap) return WG_ECAPACITY;
        int smax = 1;
        for (int k = 0; k < g->n_w; ++k) smax = sup[k] > smax ? sup[k] : smax;
        kt->s_max = smax;
        if (support_out) memcpy(support_out, sup.data(), sizeof(int32_t) * g->n_w);
        if (offset_out) memcpy(offset_out, off.data(), sizeof(int64_t) * (g->n_w + 1));
    } else {
        kt->s_max = g->s_hi;
    }
    hipLaunchKernelGGL(k_slices, dim3(g->beta * g->beta, g->n_w), dim3(256), 0, s, a,
                       (const int32_t *)kt->support, (const int64_t *)kt->offset, kt->data, kt->zeta);
    if (hipGetLastError() != hipSuccess) return WG_EHIP;
    if (sync) WG_HIP_CHECK(hipStreamSynchronize(s));
    return WG_OK;
}
