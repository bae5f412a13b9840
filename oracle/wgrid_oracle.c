/*
 * wgrid_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU reference of w-projection gridding with the
 * thesis's "compression". Only the tests, the package's smoke check and the benchmark's
 * CPU-baseline leg may call it; the product path never does. It shares no code, header or
 * table with the GPU library.
 *
 * Source: D. Muscat, "High-Performance Image Synthesis for Radio Interferometry"
 * (arXiv:1403.4209), ch.4 sec. "The WImager Component".
 *
 * Every function follows the thesis's definitions in their plain form:
 *   or_compress : the WImager preparation phase -- PreProcessUVW outputs (position tuple,
 *                 data pointer, take-conjugate eq. conj, compression indicator eq. ci), the
 *                 gridding indicator (WImager inputs/outputs), the visibility weighting and
 *                 compression of eqs. compress1 and conjugatetake, the statistics logic and
 *                 the normaliser of eq. normalizer.
 *   or_grid     : eq. gridding (gridding1 + gridding2), one run at a time, in run order.
 *   or_degrid   : the exact adjoint of or_grid (not in the thesis; derived from eq. gridding).
 *
 * Readings where the thesis is silent or garbled:
 *   - nearest-sample choice is two-stage: fine index t with t - 1/2 < x <= t + 1/2 where
 *     x = fl(u * beta/du) (eq. sat's half-open interval, ties go down), then pixel X and
 *     oversample offset o = t - beta*X with o in (-beta/2, beta/2];
 *   - row index of a kernel matrix follows v, column follows u (eq. choose swaps them);
 *   - w-plane = nearest plane in sqrt(w), via boundaries w_max*((j-1/2)/(n_w-1))^2;
 *   - the flip takes (-u,-v,-w) with the conjugate, decided on the sign of w in metres;
 *   - the compression key is the full position and kernel choice (X,Y,plane,o_u,o_v); the
 *     predecessor must itself be griddable; runs never cross a (baseline, channel) segment;
 *   - a record any of whose taps falls outside the grid is dropped whole.
 *
 * Polarisations (WImager inputs: per-polarisation flags, weights and visibilities; eqs.
 * gridding, normalizer, compress1 and conjugatetake). P = 1, 2 or 4 values per record,
 * [record][p]: P = 2 holds the two parallel hands (XX, YY or RR, LL), P = 4 the four
 * products (XX, XY, YX, YY or RR, RL, LR, LL). A record is griddable when it is on the grid
 * and at least one polarisation is unflagged; a flagged polarisation adds 0 (its (1 - f)
 * factor). The grid is [P][n][n], one plane per polarisation; the normaliser one value
 * per polarisation.
 * Reading for the flip: the measurement equation gives V_pq(-u) = conj V_qp(u) for a
 * polarised record, so with P = 4 a flipped record puts conj of its YX value (with YX's
 * weight and flag) into the XY slot and conj of XY into the YX slot; the parallel hands are
 * conjugated in place, which is eq. conjugatetake.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n, beta, n_w;
    double uv_scale;          /* beta / du: fine samples per wavelength */
    const double *wbound;     /* [n_w], entry j>=1 is the lower edge of plane j */
    const int32_t *support;   /* [n_w] odd supports */
} geom_t;

typedef struct {
    int32_t X, Y, k, ou, ov, psi, ok;
} rec_t;

/* Polarisation slot whose value (weight, flag) a record puts into slot p: the cross hands
 * exchange places when a four-product record is flipped. */
static int pol_source(int p, int npol, int psi)
{
    if (npol == 4 && psi < 0 && (p == 1 || p == 2))
        return 3 - p;
    return p;
}

/* 1 when every polarisation of record r is flagged. */
static int all_flagged(const uint8_t *flag, int64_t r, int npol)
{
    if (!flag)
        return 0;
    for (int p = 0; p < npol; ++p)
        if (flag[r * npol + p] == 0)
            return 0;
    return 1;
}

static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

/* The integer t with t - 1/2 < x <= t + 1/2 (eq. sat's interval at the fine sampling
 * interval). ceil(x - 1/2) can be one off when x - 1/2 rounds (x just above -1/2), so the
 * result is checked with exact comparisons (t +- 1/2 is exact for |t| < 2^52). */
static int64_t fine_index(double x)
{
    double t = ceil(x - 0.5);
    if (!(t - 0.5 < x))
        t -= 1.0;
    else if (!(x <= t + 0.5))
        t += 1.0;
    return (int64_t)t;
}

/* Discrete choices for one record: Convolution Function Generator eqs. choose and sat,
 * the gridding phase's Convolution Position tuple, eq. conj. `flagged` is the
 * single-polarisation flag. */
static rec_t index_record(const geom_t *g, double um, double vm, double wm, double il, int flagged)
{
    rec_t r;
    memset(&r, 0, sizeof r);
    double ul = um * il, vl = vm * il, wl = wm * il;
    r.psi = (wm >= 0.0) ? 1 : -1;
    double s = (double)r.psi;
    double uf = s * ul, vf = s * vl, wa = s * wl;
    double pu = uf * g->uv_scale;
    double pv = vf * g->uv_scale;
    const double lim = 1073741824.0; /* 2^30 fine samples */
    if (!(fabs(pu) < lim) || !(fabs(pv) < lim) || !isfinite(wa)) {
        r.ok = 0;
        return r;
    }
    int64_t iu = fine_index(pu), iv = fine_index(pv);
    int64_t hb = g->beta / 2;
    int64_t X = floor_div(iu + hb - 1, g->beta);
    int64_t Y = floor_div(iv + hb - 1, g->beta);
    r.X = (int32_t)X;
    r.Y = (int32_t)Y;
    r.ou = (int32_t)(iu - (int64_t)g->beta * X);
    r.ov = (int32_t)(iv - (int64_t)g->beta * Y);
    int k = 0;
    for (int j = 1; j < g->n_w; ++j)
        if (wa >= g->wbound[j])
            k = j;
    r.k = k;
    int64_t S = g->support[k];
    int64_t H = (S - 1) / 2;
    int64_t a = X + g->n / 2 - H;
    int64_t row0 = Y + g->n / 2 - H;
    r.ok = !flagged && a >= 0 && a + S <= g->n && row0 >= 0 && row0 + S <= g->n;
    return r;
}

/*
 * Index + compress + statistics over records in [b][ch][t] order.
 * Outputs runs (start, len, X, Y, plane, o_u, o_v, gamma[2]) and returns the run count.
 * stats[0..5] = n_records, n_griddable, n_gridded(=runs), n_compressed, upd_real, upd_saved;
 * *normaliser = sum over griddable records of weight * zeta(plane, slice).
 * zeta is [n_w][beta*beta]. compress=0 makes every griddable record its own run.
 */
int64_t or_compress(int32_t n, int32_t beta, int32_t n_w, double uv_scale,
                    const double *wbound, const int32_t *support, const double *zeta,
                    const double *uvw, const double *inv_lambda,
                    const float *vis, const float *weight, const uint8_t *flag,
                    int64_t nb, int32_t nc, int32_t nt, int32_t npol, int32_t compress,
                    int32_t *start, int32_t *len, int32_t *X, int32_t *Y, int32_t *plane,
                    int32_t *ou, int32_t *ov, double *gamma, int64_t *stats, double *normaliser)
{
    geom_t g = {n, beta, n_w, uv_scale, wbound, support};
    int64_t nruns = 0, n_grid = 0, n_comp = 0, upd_real = 0, upd_saved = 0;
    for (int p = 0; p < npol; ++p)
        normaliser[p] = 0.0;
    for (int64_t b = 0; b < nb; ++b)
        for (int32_t ch = 0; ch < nc; ++ch) {
            rec_t prev;
            memset(&prev, 0, sizeof prev);
            for (int32_t t = 0; t < nt; ++t) {
                int64_t r = (b * nc + ch) * (int64_t)nt + t;
                const double *p = uvw + (b * nt + t) * 3;
                rec_t cur = index_record(&g, p[0], p[1], p[2], inv_lambda[ch], all_flagged(flag, r, npol));
                if (cur.ok) {
                    int c = compress && t > 0 && prev.ok && cur.X == prev.X && cur.Y == prev.Y &&
                            cur.k == prev.k && cur.ou == prev.ou && cur.ov == prev.ov;
                    int64_t S = support[cur.k];
                    int sigma = (cur.ov + beta / 2 - 1) * beta + (cur.ou + beta / 2 - 1);
                    double z = zeta[(int64_t)cur.k * beta * beta + sigma];
                    /* slot q of this record: eps (1 - f) (v, conjugated when flipped) of its source */
                    double vr[4], vi[4];
                    for (int q = 0; q < npol; ++q) {
                        int64_t e = r * npol + pol_source(q, npol, cur.psi);
                        double eps = weight ? (double)weight[e] : 1.0;
                        if (flag && flag[e])
                            eps = 0.0;
                        vr[q] = eps * (double)vis[2 * e];
                        vi[q] = eps * (double)cur.psi * (double)vis[2 * e + 1];
                        normaliser[q] += eps * z;
                    }
                    n_grid++;
                    if (c) {
                        len[nruns - 1] += 1;
                        for (int q = 0; q < npol; ++q) {
                            gamma[2 * ((nruns - 1) * npol + q)] += vr[q];
                            gamma[2 * ((nruns - 1) * npol + q) + 1] += vi[q];
                        }
                        n_comp++;
                        upd_saved += S * S;
                    } else {
                        start[nruns] = (int32_t)r;
                        len[nruns] = 1;
                        X[nruns] = cur.X;
                        Y[nruns] = cur.Y;
                        plane[nruns] = cur.k;
                        ou[nruns] = cur.ou;
                        ov[nruns] = cur.ov;
                        for (int q = 0; q < npol; ++q) {
                            gamma[2 * (nruns * npol + q)] = vr[q];
                            gamma[2 * (nruns * npol + q) + 1] = vi[q];
                        }
                        upd_real += S * S;
                        nruns++;
                    }
                }
                prev = cur;
            }
        }
    stats[0] = nb * nc * (int64_t)nt;
    stats[1] = n_grid;
    stats[2] = nruns;
    stats[3] = n_comp;
    stats[4] = upd_real;
    stats[5] = upd_saved;
    return nruns;
}

/* Per-record discrete choices, for pin tests: X, Y, plane, o_u, o_v, psi, griddable. */
void or_index(int32_t n, int32_t beta, int32_t n_w, double uv_scale,
              const double *wbound, const int32_t *support,
              const double *uvw, const double *inv_lambda, const uint8_t *flag,
              int64_t nb, int32_t nc, int32_t nt, int32_t npol, int32_t *out /* [N_rec][7] */)
{
    geom_t g = {n, beta, n_w, uv_scale, wbound, support};
    for (int64_t b = 0; b < nb; ++b)
        for (int32_t ch = 0; ch < nc; ++ch)
            for (int32_t t = 0; t < nt; ++t) {
                int64_t r = (b * nc + ch) * (int64_t)nt + t;
                const double *p = uvw + (b * nt + t) * 3;
                rec_t c = index_record(&g, p[0], p[1], p[2], inv_lambda[ch], all_flagged(flag, r, npol));
                int32_t *o = out + r * 7;
                o[0] = c.X; o[1] = c.Y; o[2] = c.k; o[3] = c.ou; o[4] = c.ov; o[5] = c.psi; o[6] = c.ok;
            }
}

/* eq. gridding: G[p][row0+i][a+j] += gamma[p] * K_plane[slice][i][j] for every run and
 * polarisation, FP64.
 * table: interleaved complex FP64, plane k starting at offset[k] complex elements; each
 * plane holds beta^2 slices of S_k x S_k row-major matrices, slice index
 * (o_v + beta/2 - 1)*beta + (o_u + beta/2 - 1). gamma: [nruns][npol] complex;
 * grid: [npol][n][n] complex, accumulated. */
void or_grid(int32_t n, int32_t beta, int32_t npol, const int32_t *support, const int64_t *offset,
             const double *table, int64_t nruns, const int32_t *X, const int32_t *Y,
             const int32_t *plane, const int32_t *ou, const int32_t *ov,
             const double *gamma, double *grid)
{
    for (int64_t q = 0; q < nruns; ++q) {
        int64_t S = support[plane[q]], H = (S - 1) / 2;
        int64_t a = X[q] + n / 2 - H, row0 = Y[q] + n / 2 - H;
        int64_t sigma = (int64_t)(ov[q] + beta / 2 - 1) * beta + (ou[q] + beta / 2 - 1);
        const double *K = table + 2 * (offset[plane[q]] + sigma * S * S);
        for (int p = 0; p < npol; ++p) {
            double gr = gamma[2 * (q * npol + p)], gi = gamma[2 * (q * npol + p) + 1];
            for (int64_t i = 0; i < S; ++i)
                for (int64_t j = 0; j < S; ++j) {
                    double kr = K[2 * (i * S + j)], ki = K[2 * (i * S + j) + 1];
                    double *G = grid + 2 * ((int64_t)p * n * n + (row0 + i) * n + a + j);
                    G[0] += gr * kr - gi * ki;
                    G[1] += gr * ki + gi * kr;
                }
        }
    }
}

/* Adjoint of or_grid followed by the adjoint of the visibility weighting:
 * per run and polarisation d[p] = sum_ij conj(K[i][j]) * G[p][row0+i][a+j]; polarisation p
 * of every member record x of the run gets weight_{x,p} (1 - f_{x,p}) times d[p], or, when
 * x is flipped, conj d[s] with s the slot its value went to (the cross hands exchange with
 * P = 4). Records in no run get 0. vis_out: [N_rec][npol] complex; weight, flag
 * [N_rec][npol] or NULL. */
void or_degrid(int32_t n, int32_t beta, int32_t npol, const int32_t *support, const int64_t *offset,
               const double *table, int64_t nruns, const int32_t *start, const int32_t *len,
               const int32_t *X, const int32_t *Y, const int32_t *plane,
               const int32_t *ou, const int32_t *ov, const double *grid,
               const double *uvw, const float *weight, const uint8_t *flag, int64_t nb, int32_t nc,
               int32_t nt, double *vis_out)
{
    memset(vis_out, 0, sizeof(double) * 2 * (size_t)(nb * nc * (int64_t)nt * npol));
    for (int64_t q = 0; q < nruns; ++q) {
        int64_t S = support[plane[q]], H = (S - 1) / 2;
        int64_t a = X[q] + n / 2 - H, row0 = Y[q] + n / 2 - H;
        int64_t sigma = (int64_t)(ov[q] + beta / 2 - 1) * beta + (ou[q] + beta / 2 - 1);
        const double *K = table + 2 * (offset[plane[q]] + sigma * S * S);
        double dr[4], di[4];
        for (int p = 0; p < npol; ++p) {
            dr[p] = di[p] = 0.0;
            for (int64_t i = 0; i < S; ++i)
                for (int64_t j = 0; j < S; ++j) {
                    double kr = K[2 * (i * S + j)], ki = K[2 * (i * S + j) + 1];
                    const double *G = grid + 2 * ((int64_t)p * n * n + (row0 + i) * n + a + j);
                    dr[p] += kr * G[0] + ki * G[1];
                    di[p] += kr * G[1] - ki * G[0];
                }
        }
        for (int32_t m = 0; m < len[q]; ++m) {
            int64_t r = (int64_t)start[q] + m;
            int64_t t = r % nt, b = r / ((int64_t)nt * nc);
            double wm = uvw[(b * nt + t) * 3 + 2];
            int psi = (wm >= 0.0) ? 1 : -1;
            for (int p = 0; p < npol; ++p) {
                int64_t e = r * npol + p;
                double eps = weight ? (double)weight[e] : 1.0;
                if (flag && flag[e])
                    eps = 0.0;
                int s = pol_source(p, npol, psi); /* the exchange is its own inverse */
                vis_out[2 * e] = eps * dr[s];
                vis_out[2 * e + 1] = eps * (double)psi * di[s];
            }
        }
    }
}
