"""MI355X-native w-projection gridding with compression (HIP library + thin binding).

Method: D. Muscat, High-Performance Image Synthesis for Radio Interferometry (arXiv:1403.4209).
The compute runs in libwgrid.so (csrc/, C ABI in include/wgrid.h); `wgrid` is its binding.
"""
from .wgrid import (DTYPES, GridFn, Gridder, KernelTable, Runs, Stats, WgError, WgGeom, finalise,  # noqa: F401
                    geom_from_dict, make_geom, wg_compress, wg_degrid, wg_finalise, wg_finalise_ws_bytes, wg_grid,
                    wg_ktable_build, wg_ktable_sizes, wg_plan_elems, wg_status_str, wg_version)
