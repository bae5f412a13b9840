// One call from records to grid: the WImager component as a whole (inputs I-1..I-5 and the
// generator's outputs C-1..C-3 in; the grid O-1 and the normaliser O-2 out), i.e. the
// preparation phase (wg_compress) followed by the gridding phase (wg_grid), with the run
// list and plan carved out of one caller-owned workspace.
#include <mutex>

#include "wg_common.hpp"

namespace wg {
namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout of the workspace for nb x nc x nt records: the run arrays of wg_runs (capacity =
// records, so the run list cannot overflow), the per-run grid ids, the normalisers and the
// plan, each starting on a 256-byte boundary. With `base` NULL only the size is computed.
size_t carve(const wg_geom *g, int64_t nb, int32_t nc, int32_t nt, char *base, wg_runs *r) {
    const int64_t cap = nb * (int64_t)nc * nt;
    const int64_t npol = npol_of(g);
    const bool ids = (g->flags & (WG_GRID_PER_CHANNEL | WG_W_STACKING)) != 0;
    const int64_t n_norm = ((g->flags & WG_GRID_PER_CHANNEL) ? nc : 1) * npol;
    const int64_t plan = wg_plan_elems(cap, nb * nc);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? base + off : nullptr;
        off += round_up(bytes);
        return p;
    };
    wg_runs v;
    v.capacity = cap;
    v.start = (int32_t *)take(4 * cap);
    v.len = (int32_t *)take(4 * cap);
    v.x = (int32_t *)take(4 * cap);
    v.y = (int32_t *)take(4 * cap);
    v.plane = (int16_t *)take(2 * cap);
    v.ou = (int8_t *)take(cap);
    v.ov = (int8_t *)take(cap);
    v.gamma = (float *)take(8 * cap * npol);
    v.work = (float *)take(8 * cap * npol);
    v.grid = ids ? (int16_t *)take(2 * cap) : nullptr;
    v.norm = (double *)take(8 * n_norm);
    v.plan = (int32_t *)take(4 * plan);
    v.plan_elems = plan;
    if (r) *r = v;
    return off;
}

int check_sizes(int64_t nb, int32_t nc, int32_t nt) {
    if (nb < 1 || nc < 1 || nt < 1) return WG_EINVAL;
    if (nb * (int64_t)nc * nt >= ((int64_t)1 << 31)) return WG_EUNSUPPORTED;
    return WG_OK;
}

}  // namespace

// Shared by wg_grid_records and its workspace-free variant: compress into the runs `r`
// (views of a workspace) and grid them.
int grid_records_into(const wg_geom *g, const wg_ktable *kt, const double *uvw, const double *inv_lambda,
                      const float *vis, const float *weight, const uint8_t *flag, int64_t nb, int32_t nc,
                      int32_t nt, float *grid, wg_stats *stats, wg_runs *r, wg_stream_t stream) {
    if (!grid) return WG_EINVAL;
    int st = wg_compress(g, kt, uvw, inv_lambda, vis, weight, flag, nb, nc, nt, r, stats, stream);
    if (st != WG_OK) return st;
    return wg_grid(g, kt, r, stats, grid, stream);
}

}  // namespace wg

extern "C" int wg_grid_records_ws(const wg_geom *g, int64_t nb, int32_t nc, int32_t nt, void *ws,
                                  size_t *ws_bytes, wg_runs *runs) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_sizes(nb, nc, nt)) != WG_OK) return st;
    if (!ws_bytes) return WG_EINVAL;
    const size_t need = carve(g, nb, nc, nt, nullptr, nullptr);
    if (!ws) {
        *ws_bytes = need;
        return WG_OK;
    }
    if ((uintptr_t)ws % kAlign != 0) return WG_EINVAL;
    if (*ws_bytes < need) return WG_ECAPACITY;
    if (runs) carve(g, nb, nc, nt, (char *)ws, runs);
    return WG_OK;
}

extern "C" int wg_grid_records(const wg_geom *g, const wg_ktable *kt, const double *uvw, const double *inv_lambda,
                               const float *vis, const float *weight, const uint8_t *flag, int64_t nb, int32_t nc,
                               int32_t nt, float *grid, wg_stats *stats, void *ws, size_t ws_bytes,
                               wg_runs *runs_out, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_table(g, kt)) != WG_OK) return st;
    if ((st = check_sizes(nb, nc, nt)) != WG_OK) return st;
    if (!grid || !stats || !ws) return WG_EINVAL;
    if ((uintptr_t)ws % kAlign != 0) return WG_EINVAL;
    if (kt->data_cap >= ((int64_t)1 << 28)) return WG_EUNSUPPORTED;  // as wg_grid, checked before any work
    if (ws_bytes < carve(g, nb, nc, nt, nullptr, nullptr)) return WG_ECAPACITY;
    wg_runs r;
    carve(g, nb, nc, nt, (char *)ws, &r);
    if (runs_out) *runs_out = r;
    return grid_records_into(g, kt, uvw, inv_lambda, vis, weight, flag, nb, nc, nt, grid, stats, &r, stream);
}

// ---------------------------------------------------------------------------------------
// Workspace-free variant: the run list, plan and normalisers live in `scratch`, a fixed
// array of this library on each GPU (held until the process ends). In host code the
// array's name stands for no device address: its address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current, and only that
// address is handed to the kernels.
namespace wg {
namespace {

constexpr size_t kScratchBytes = WG_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex scratch_mu;
void *scratch_at[kMaxDevices];

// The device address of `scratch` on the current device, or NULL on a HIP error.
void *scratch_address(int dev) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_at[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        scratch_at[dev] = p;
    }
    return scratch_at[dev];
}

}  // namespace
}  // namespace wg

extern "C" int wg_grid_records_static(const wg_geom *g, const wg_ktable *kt, const double *uvw,
                                      const double *inv_lambda, const float *vis, const float *weight,
                                      const uint8_t *flag, int64_t nb, int32_t nc, int32_t nt, float *grid,
                                      wg_stats *stats, wg_runs *runs_out, wg_stream_t stream) {
    using namespace wg;
    int st = check_geom(g);
    if (st != WG_OK) return st;
    if ((st = check_table(g, kt)) != WG_OK) return st;
    if ((st = check_sizes(nb, nc, nt)) != WG_OK) return st;
    if (!grid || !stats) return WG_EINVAL;
    if (kt->data_cap >= ((int64_t)1 << 28)) return WG_EUNSUPPORTED;
    if (carve(g, nb, nc, nt, nullptr, nullptr) > kScratchBytes) return WG_ECAPACITY;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return WG_EHIP;
    if (dev >= kMaxDevices) return WG_EUNSUPPORTED;
    void *base = scratch_address(dev);
    if (!base) return WG_EHIP;
    wg_runs r;
    carve(g, nb, nc, nt, (char *)base, &r);
    if (runs_out) *runs_out = r;
    return grid_records_into(g, kt, uvw, inv_lambda, vis, weight, flag, nb, nc, nt, grid, stats, &r, stream);
}
