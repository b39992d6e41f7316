// eu_kset.hpp -- per-precision kernel launchers (one table per state type).
#pragma once

#include "eu_internal.hpp"

namespace eu {

// Initial data parameters (host values passed by value to the kernel).
struct InitArgs {
    int kind;          // 0 quadrants, 1 ellipsoid, 2 1D Riemann, 3 uniform
    int axis;
    double lo, hi;
    double x0, y0;
    double quad[4][4];
    double ell[8];
    double es[4];
    double lr[6];
    double split;
    double uni[5];
};

// Which state array a launcher works on.
enum { ARR_Q = 0, ARR_QS = 1, ARR_QO = 2 };

constexpr int FV_VARIANTS = 10;  // schedules of the stage kernel (autotuned)
// Schedules 6-9 (grids of one level: a uniform grid or a batch) run the
// strip kernels.  2D: 6, 7 one stage per launch, 8, 9 both stages in one
// launch (outflow boundaries only); 6 and 8 strips of 32 rows, 7 and 9 of
// 128.  3D (one stage per launch): workgroups of 8 output rows (6, 8) or 16
// (7, 9), strips of 32 planes (6, 7) or 64 (8, 9).
constexpr int FV_STRIP0 = 6;
inline bool strip_variant(int var) { return var >= FV_STRIP0; }
inline bool strip_fused(int var) { return var >= FV_STRIP0 + 2; }
inline int strip_rows(int var) { return (var - FV_STRIP0) % 2 ? 128 : 32; }
inline int strip3_waves(int var) { return (var - FV_STRIP0) % 2 ? 16 : 8; }
inline int strip3_planes(int var) { return var >= FV_STRIP0 + 2 ? 64 : 32; }
inline int strip_width(bool fused) { return fused ? 56 : 60; }   // columns written per strip
inline int strip_halo(bool fused) { return fused ? 4 : 2; }
// The AMR scheme on a hierarchy runs the Hancock tile kernel: schedules 0,
// 1, 2 with 128, 192, 256 threads per tile in 2D; 0, 1 with 256, 512 in 3D
// (its LDS holds one tile per CU).
inline int hancock_tile_variants(int dim) { return dim == 2 ? 3 : 2; }

struct KSet {
    size_t elem;  // bytes per state value
    void (*init)(const View &, const InitArgs &, int grid, int64_t ncell, hipStream_t);
    void (*restrict_full)(const View &, int arr, int grid_coarse, int64_t ncell, hipStream_t);
    void (*restrict_cov)(const View &, int arr, int lvl, int maxblocks, hipStream_t);
    void (*restrict2)(const View &, int arr, int lvl, int nlev, int ghosts, int64_t ndetails, int maxblocks,
                      hipStream_t);   // 2D, nlev = 1 or 2
    // cfl: also the CFL slots of the state it leaves (mode 3 on the state,
    // the launch of the finest levels; the slots must be zero)
    void (*predict)(const View &, int arr, int lvl, int nlev, int mode, double theta, int cfl, int maxblocks,
                    hipStream_t);
    // fineproj (2D hierarchy, global step): tiles of level L-1 also write the
    // projection of their cells onto level L-2
    void (*fv_stage)(const View &, int stage, int lvl, int sub, int record, int maxtiles, int variant,
                     int fineproj, hipStream_t);
    // strip kernels: one stage (fused = 0; own_base: the base state is the
    // source) or both (fused = 1) over count strips; cfl = 1: the launch
    // adds the CFL partials of the state it writes (zero partials needed),
    // cfl = 2: computes them without publishing
    void (*fv_strip)(const View &, int fused, int own_base, int cfl, const Strip *list, int count, const void *src,
                     const void *base, void *out, double fac, hipStream_t);
    // 3D strip kernel: one stage over count strips with workgroups of waves
    // rows (8 or 16)
    void (*fv_strip3)(const View &, int waves, int own_base, int cfl, const Strip *list, int count, const void *src,
                      const void *base, void *out, double fac, hipStream_t);
    // the AMR scheme's MUSCL-Hancock step over count strips (src -> out)
    void (*hancock_strip)(const View &, int cfl, const Strip *list, int count, const void *src, void *out,
                          hipStream_t);
    // the AMR scheme's MUSCL-Hancock step (Q -> Qs) on every leaf of a
    // hierarchy or uniform grid (lvl < 0; past t_end the whole state of nstate elements is
    // copied) or on the patches of level lvl (local time stepping; record:
    // flux registers of substep sub)
    void (*hancock_tile)(const View &, int variant, int fineproj, int64_t nstate, int maxtiles, int lvl, int sub,
                         int record, hipStream_t);
    // the patch cells of level lvl: Q -> Qo, or Qs -> Q (back)
    void (*copy_level)(const View &, int lvl, int maxblocks, int back, hipStream_t);
    void (*reflux)(const View &, int lvl, int maxblocks, hipStream_t);
    void (*cfl_slots)(const View &, int maxtiles, hipStream_t);     // into zero CFL slots / batch maxima
    void (*totals)(const View &, int maxtiles, hipStream_t);
    void (*details)(const View &, int64_t ncell_coarse_levels, hipStream_t);
    void (*gradient)(const View &, int64_t ncell_coarse_levels, hipStream_t);
    void (*composite)(const View &, int lvl, int64_t ncell, hipStream_t);
};

// workgroups of a prediction launch over maxblocks blocks
inline int predict_grid(int64_t maxblocks)
{
    constexpr int CAP = 1024;
    return maxblocks < 1 ? 1 : maxblocks > CAP ? CAP : (int)maxblocks;
}

extern const KSet kset_f64;
extern const KSet kset_f32;

// precision-independent mesh kernels (eu_mesh.hip)
void launch_flag_tile(const View &, int lvl, int nblocks, hipStream_t);
// every flagged level in one launch (workgroups of level L-2-k from wg0[k] on,
// nflag of them), optionally followed by the list build in the same launch
bool flag_chain_ok(const View &);
bool flag_chain_lists(const View &, int64_t nblocks_total);
void launch_flag_chain(const View &, const int *wg0, int nseg, int nflag, int64_t nblocks_total, bool lists,
                       hipStream_t);
void launch_build_lists(const View &, int64_t nblocks_total, hipStream_t);
void launch_cfl_final(const View &, hipStream_t);
void launch_fill_u8(uint8_t *p, int64_t n, uint8_t val, hipStream_t);
void launch_totals_final(const View &, int ngroups, hipStream_t);
void launch_set_dt(const View &, const double *dt_ext, hipStream_t);
void launch_copy_f64(double *dst, const double *src, int n, hipStream_t);
void launch_threshold(const View &, int64_t ncell, hipStream_t);

}  // namespace eu
