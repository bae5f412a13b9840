// Host-side argument checks and small entry points of the C ABI.
#include "wg_common.hpp"

namespace wg {

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int check_geom(const wg_geom *g) {
    if (!g) return WG_EINVAL;
    if (g->n < 2 || (g->n & 1) || g->beta < 2 || !is_pow2(g->beta) || g->n_w < 1) return WG_EINVAL;
    if (g->s_lo < 1 || g->s_hi < g->s_lo || !(g->s_lo & 1) || !(g->s_hi & 1)) return WG_EINVAL;
    if (!(g->du > 0.0) || !(g->w_max >= 0.0) || g->du != g->du) return WG_EINVAL;
    if (g->m_img < 16 || !is_pow2(g->m_img)) return WG_EINVAL;
    if ((g->flags & ~(WG_COMPRESS | WG_GRID_PER_CHANNEL | WG_W_STACKING | WG_POL_CIRCULAR | WG_PLAIN_SUMS)) != 0)
        return WG_EINVAL;
    if ((g->flags & WG_GRID_PER_CHANNEL) && (g->flags & WG_W_STACKING)) return WG_EINVAL;
    if (g->n_pol != 0 && g->n_pol != 1 && g->n_pol != 2 && g->n_pol != 4) return WG_EINVAL;
    if (g->n > 32768 || g->beta > 32 || g->n_w > WG_MAX_PLANES || g->s_hi > WG_MAX_SUPPORT)
        return WG_EUNSUPPORTED;
    const int64_t L = (int64_t)g->beta * g->m_img;
    if (L > WG_MAX_FFT) return WG_EUNSUPPORTED;
    // the widest matrix must stay inside the oversampled plane
    if ((int64_t)(g->s_hi - 1) / 2 * g->beta + g->beta / 2 >= L / 2) return WG_EINVAL;
    return WG_OK;
}

int check_table(const wg_geom *g, const wg_ktable *kt) {
    if (!kt) return WG_EINVAL;
    if (kt->dtype < WG_KF32 || kt->dtype > WG_KF16) return WG_EINVAL;
    if (kt->n_w != g->n_w || kt->beta != g->beta) return WG_EINVAL;
    if (!kt->support || !kt->offset || !kt->wbound || !kt->zeta || !kt->data) return WG_EINVAL;
    if (kt->s_max < 1 || kt->s_max > g->s_hi) return WG_EINVAL;
    return WG_OK;
}

}  // namespace wg

extern "C" {

const char *wg_status_str(int s) {
    switch (s) {
    case WG_OK: return "ok";
    case WG_EINVAL: return "invalid argument";
    case WG_ECAPACITY: return "buffer too small";
    case WG_EHIP: return "HIP runtime error";
    case WG_EUNSUPPORTED: return "unsupported size";
    default: return "unknown status";
    }
}

int wg_version(void) { return 100; }

int64_t wg_plan_elems(int64_t capacity, int64_t n_segments) {
    if (capacity < 0 || n_segments < 0) return -1;
    return wg::plan_tiles_at(capacity, n_segments) + wg::n_scan_tiles(n_segments) + 1;
}

}  // extern "C"
