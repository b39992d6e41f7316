// eu_kset_impl.hpp -- launcher bodies, instantiated once per state type by
// eu_fp64.hip and eu_fp32.hip.
#pragma once

#include "eu_kernels.hpp"

namespace eu {
namespace impl {

inline int clamp_grid(int64_t want, int cap)
{
    if (want < 1) return 1;
    return want > cap ? cap : (int)want;
}

// grid for XCD-aware walks: a multiple of 8 once there are 8 items or more
inline int xcd_grid(int64_t want, int cap)
{
    int g = clamp_grid(want, cap);
    return g < 8 ? g : (g + 7) / 8 * 8;
}

template <typename T> T *arr(const View &v, int a)
{
    return (T *)(a == ARR_Q ? v.Q : a == ARR_QS ? v.Qs : v.Qo);
}

template <typename T> void init(const View &v, const InitArgs &a, int grid, int64_t ncell, hipStream_t s)
{
    const int nblk = clamp_grid((ncell + 255) / 256, 8192);
    if (v.dim == 2) k_init<T, 2><<<nblk, 256, 0, s>>>(v, a, grid, (T *)v.Q);
    else k_init<T, 3><<<nblk, 256, 0, s>>>(v, a, grid, (T *)v.Q);
}

template <typename T> void restrict_full(const View &v, int a, int gc, int64_t ncell, hipStream_t s)
{
    const int nblk = clamp_grid((ncell + 255) / 256, 8192);
    if (v.dim == 2) k_restrict_full<T, 2><<<nblk, 256, 0, s>>>(v, arr<T>(v, a), gc);
    else k_restrict_full<T, 3><<<nblk, 256, 0, s>>>(v, arr<T>(v, a), gc);
}

template <typename T> void restrict_cov(const View &v, int a, int lvl, int maxb, hipStream_t s)
{
    const int nblk = clamp_grid(maxb, 1024);
    if (v.dim == 2) k_restrict_cov<T, 2><<<nblk, 64, 0, s>>>(v, arr<T>(v, a), lvl);
    else k_restrict_cov<T, 3><<<nblk, 256, 0, s>>>(v, arr<T>(v, a), lvl);
}

// one or two levels per launch (2D only), optionally with the ghost fill of
// every level or the MR details of levels 0 .. L-2
template <typename T> void restrict2(const View &v, int a, int lvl, int nlev, int ghosts, int64_t ndet, int maxb,
                                     hipStream_t s)
{
    const int nblk = clamp_grid(maxb, 2048);
    k_restrict2<T><<<nblk, 64, 0, s>>>(v, arr<T>(v, a), lvl, nlev, ghosts, ndet);
}

template <typename T> void predict(const View &v, int a, int lvl, int nlev, int mode, double theta, int cfl,
                                   int maxb, hipStream_t s)
{
    // the launch that also reduces the CFL speeds takes up to 2048
    // workgroups: the ones without a prediction then take the leaf tiles in
    // one round of two
    const int nblk = cfl && v.dim == 2 && mode == 3 ? clamp_grid(maxb, 2048) : predict_grid(maxb);
    const Grid Gl = v.gt[mode == 1 ? 0 : lvl], Cl = v.gt[mode == 1 ? 0 : lvl - 1];
    const Grid Gh = v.gt[nlev == 2 ? lvl + 1 : (mode == 1 ? 0 : lvl)];
    // the blocks of the levels walked directly when one pass takes them all
    const int direct = mode == 3 && !cfl && maxb <= nblk ? 1 : 0;
    if (v.dim == 2)
        k_predict<T, 2><<<nblk, 64, 0, s>>>(v, arr<T>(v, a), lvl, mode, theta, nlev, Gl, Cl, Gh, cfl, direct);
    else
        k_predict<T, 3><<<nblk, 256, 0, s>>>(v, arr<T>(v, a), lvl, mode, theta, nlev, Gl, Cl, Gh, cfl, direct);
}

// Stage-kernel schedules the autotuner chooses from (variant index):
//   2D: 0 = 64 threads, per-axis faces; 1 = 64 threads, merged faces;
//       2 = 128 threads, per-axis;      3 = 128 threads, merged;
//       4 = 192 threads, merged (one face per thread, 144 faces);
//       5 = 128 threads, per-axis with per-cell face states.
//   3D: 0-3 and 5 the same with 256 and 512 threads; 4 = 256 threads,
//       per-axis with per-cell face states.
template <typename T, int D, int NT, int M>
void fv_launch(const View &v, int nblk, const T *src, T *out, double fac, int lvl, int sub, int record,
               int fineproj, int blend, hipStream_t s)
{
    k_fv_stage<T, D, NT, M><<<nblk, NT, 0, s>>>(v, src, (const T *)v.Q, out, fac, lvl, sub, record, fineproj,
                                                blend);
}

template <typename T> void fv_stage(const View &v, int stage, int lvl, int sub, int record, int maxt,
                                    int variant, int fineproj, hipStream_t s)
{
    // a 2D hierarchy has at most a few thousand leaf tiles: 2048 workgroups
    // take them all at once, and fewer idle workgroups are dispatched (a
    // batch or a 3D grid needs the larger grid to fill the chip)
    const int nblk = xcd_grid(maxt, v.dim == 2 && v.mode == MODE_HIER ? 2048 : 16384);
    // stage 3: the second stage's form reading Q and writing the stage array
    // (timing passes that leave the state unchanged)
    const T *src = (const T *)(stage == 2 ? v.Qs : v.Q);
    T *out = (T *)(stage == 2 ? v.Q : v.Qs);
    // midpoint rule: dt/2 then dt; Heun: dt, then dt/2 from the mean of the
    // base and the stage state
    const double fac = stage == 1 ? (v.rk ? 1.0 : 0.5) : (v.rk ? 0.5 : 1.0);
    const int blend = stage != 1 && v.rk ? 1 : 0;
    if (v.dim == 2) {
        switch (variant) {
        case 1: fv_launch<T, 2, 64, 1>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 2: fv_launch<T, 2, 128, 0>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 3: fv_launch<T, 2, 128, 1>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 4: fv_launch<T, 2, 192, 1>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 5: fv_launch<T, 2, 128, 2>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        default: fv_launch<T, 2, 64, 0>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        }
    } else {
        switch (variant) {
        case 1: fv_launch<T, 3, 256, 1>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 2: fv_launch<T, 3, 512, 0>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 3: fv_launch<T, 3, 512, 1>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 4: fv_launch<T, 3, 256, 2>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        case 5: fv_launch<T, 3, 512, 2>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        default: fv_launch<T, 3, 256, 0>(v, nblk, src, out, fac, lvl, sub, record, fineproj, blend, s); break;
        }
    }
}

template <typename T> void fv_strip(const View &v, int fused, int own_base, int cfl, const Strip *list, int count,
                                    const void *src, const void *base, void *out, double fac, hipStream_t s)
{
    const int nblk = xcd_grid((count + 3) / 4, 16384);
    if (fused)
        k_fv_strip<T, 1><<<nblk, 256, 0, s>>>(v, list, count, (const T *)src, (const T *)base, (T *)out, fac, 0,
                                              cfl);
    else
        k_fv_strip<T, 0><<<nblk, 256, 0, s>>>(v, list, count, (const T *)src, (const T *)base, (T *)out, fac,
                                              own_base, cfl);
}

template <typename T> void fv_strip3(const View &v, int waves, int own_base, int cfl, const Strip *list, int count,
                                     const void *src, const void *base, void *out, double fac, hipStream_t s)
{
    const int nblk = xcd_grid(count, 16384);
    if (waves == 16)
        k_fv_strip3<T, 16><<<nblk, 1024, 0, s>>>(v, list, count, (const T *)src, (const T *)base, (T *)out, fac,
                                                 own_base, cfl);
    else
        k_fv_strip3<T, 8><<<nblk, 512, 0, s>>>(v, list, count, (const T *)src, (const T *)base, (T *)out, fac,
                                               own_base, cfl);
}

template <typename T> void hancock_strip(const View &v, int cfl, const Strip *list, int count, const void *src,
                                         void *out, hipStream_t s)
{
    const int nblk = xcd_grid((count + 3) / 4, 16384);
    k_hancock_strip<T><<<nblk, 256, 0, s>>>(v, list, count, (const T *)src, (T *)out, cfl);
}

template <typename T> void hancock_tile(const View &v, int variant, int fineproj, int64_t nstate, int maxt, int lvl,
                                        int sub, int record, hipStream_t s)
{
    const T *src = (const T *)v.Q;
    T *out = (T *)v.Qs;
    if (v.dim == 3) {
        const int nb3 = xcd_grid(maxt, 16384);
        if (variant == 1) k_hancock_tile3<T, 512><<<nb3, 512, 0, s>>>(v, src, out, nstate, lvl, sub, record);
        else k_hancock_tile3<T, 256><<<nb3, 256, 0, s>>>(v, src, out, nstate, lvl, sub, record);
        return;
    }
    const int nblk = xcd_grid(maxt, 2048);
    switch (variant) {
    case 1: k_hancock_tile<T, 192><<<nblk, 192, 0, s>>>(v, src, out, fineproj, nstate, lvl, sub, record); break;
    case 2: k_hancock_tile<T, 256><<<nblk, 256, 0, s>>>(v, src, out, fineproj, nstate, lvl, sub, record); break;
    default: k_hancock_tile<T, 128><<<nblk, 128, 0, s>>>(v, src, out, fineproj, nstate, lvl, sub, record); break;
    }
}

template <typename T> void copy_level(const View &v, int lvl, int maxb, int back, hipStream_t s)
{
    const int nblk = clamp_grid(maxb, 2048);
    const T *src = (const T *)(back ? v.Qs : v.Q);
    T *dst = (T *)(back ? v.Q : v.Qo);
    if (v.dim == 2) k_copy_level<T, 2><<<nblk, 64, 0, s>>>(v, lvl, src, dst);
    else k_copy_level<T, 3><<<nblk, 256, 0, s>>>(v, lvl, src, dst);
}

template <typename T> void reflux(const View &v, int lvl, int maxb, hipStream_t s)
{
    const int nblk = clamp_grid(maxb, 1024);
    if (v.dim == 2) k_reflux<T, 2><<<nblk, 64, 0, s>>>(v, lvl);
    else k_reflux<T, 3><<<nblk, 256, 0, s>>>(v, lvl);
}

// The CFL maxima of the current state added into the slots (hierarchy) or
// the per-instance maxima (batch), which must be zero (one wave per tile;
// 2D tiles are light: fewer workgroups suffice)
template <typename T> void cfl_slots(const View &v, int maxt, hipStream_t s)
{
    // (a batch's hundreds of thousands of tiles need the chip: more workgroups)
    const int cap = v.mode == MODE_BATCH ? 8192 : v.dim == 2 ? 512 : CFL_MAXBLK;
    const int nblk = clamp_grid((maxt + 3) / 4, cap);
    if (v.dim == 2) k_cfl<T, 2><<<nblk, 256, 0, s>>>(v, (const T *)v.Q);
    else k_cfl<T, 3><<<nblk, 256, 0, s>>>(v, (const T *)v.Q);
}

template <typename T> void totals(const View &v, int maxt, hipStream_t s)
{
    const int nblk = clamp_grid(maxt, 8192);
    if (v.dim == 2) k_totals<T, 2><<<nblk, 256, 0, s>>>(v, (const T *)v.Q);
    else k_totals<T, 3><<<nblk, 256, 0, s>>>(v, (const T *)v.Q);
}

template <typename T> void composite(const View &v, int lvl, int64_t ncell, hipStream_t s)
{
    const int nblk = clamp_grid((ncell + 255) / 256, 8192);
    if (v.dim == 2) k_composite<T, 2><<<nblk, 256, 0, s>>>(v, lvl);
    else k_composite<T, 3><<<nblk, 256, 0, s>>>(v, lvl);
}

template <typename T> void details(const View &v, int64_t ncell, hipStream_t s)
{
    const int nblk = clamp_grid((ncell + 255) / 256, 8192);
    if (v.dim == 2) k_details<T, 2><<<nblk, 256, 0, s>>>(v, (const T *)v.Q, ncell);
    else k_details<T, 3><<<nblk, 256, 0, s>>>(v, (const T *)v.Q, ncell);
}

template <typename T> void gradient(const View &v, int64_t ncell, hipStream_t s)
{
    const int nblk = clamp_grid((ncell + 255) / 256, 8192);
    if (v.dim == 2) k_gradient<T, 2><<<nblk, 256, 0, s>>>(v, (const T *)v.Q, ncell);
    else k_gradient<T, 3><<<nblk, 256, 0, s>>>(v, (const T *)v.Q, ncell);
}

template <typename T> KSet make()
{
    KSet k;
    k.elem = sizeof(T);
    k.init = init<T>;
    k.restrict_full = restrict_full<T>;
    k.restrict_cov = restrict_cov<T>;
    k.restrict2 = restrict2<T>;
    k.composite = composite<T>;
    k.predict = predict<T>;
    k.fv_stage = fv_stage<T>;
    k.fv_strip = fv_strip<T>;
    k.hancock_strip = hancock_strip<T>;
    k.hancock_tile = hancock_tile<T>;
    k.fv_strip3 = fv_strip3<T>;
    k.copy_level = copy_level<T>;
    k.reflux = reflux<T>;
    k.cfl_slots = cfl_slots<T>;
    k.totals = totals<T>;
    k.details = details<T>;
    k.gradient = gradient<T>;
    return k;
}

}  // namespace impl
}  // namespace eu
