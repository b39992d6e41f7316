// eu_kernels.hpp -- gfx950 kernels of the finite-volume / multiresolution
// path, templated on the state type T (double | float) and the dimension D.
// Included by eu_fp64.hip (built without FMA contraction, so FP64 results
// follow the reference expression trees operation for operation) and by
// eu_fp32.hip (contraction allowed, hardware reciprocal and square root).
#pragma once

#include "eu_internal.hpp"
#include "eu_kset.hpp"

namespace eu {

// ----------------------------------------------------------------------------
// arithmetic per precision
// ----------------------------------------------------------------------------
template <typename T> struct Ar;
template <> struct Ar<double> {
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double sqrt(double a) { return __builtin_sqrt(a); }
    static __device__ __forceinline__ double abs(double a) { return __builtin_fabs(a); }
};
template <> struct Ar<float> {
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float sqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
    static __device__ __forceinline__ float abs(float a) { return __builtin_fabsf(a); }
};

// Boundary index map: outflow (zero-order extrapolation) clamps to the
// nearest interior cell; periodic wraps.  |i| stays within one period.
__device__ __forceinline__ int bcmap(int i, int n, int bc)
{
    if (bc == 1) return i < 0 ? i + n : (i >= n ? i - n : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ int64_t gidx(int n, int x, int y, int z)
{
    return x + (int64_t)n * (y + (int64_t)n * z);
}

// The same index in 32 bits (every grid has fewer than 2^31 cells; the
// library checks this at creation): with a per-field base pointer held in
// scalar registers the address is one 32-bit offset.
__device__ __forceinline__ uint32_t gidx32(int n, int x, int y, int z)
{
    return (uint32_t)x + (uint32_t)n * ((uint32_t)y + (uint32_t)n * (uint32_t)z);
}

// XCD-aware assignment of list items to workgroups.  Workgroups are
// dispatched to the 8 XCDs round robin (blockIdx % 8), each XCD with its own
// L2; XCD x walks the contiguous x-th eighth of the list, its workgroups
// taking consecutive items, so tiles processed together on one XCD are
// neighbours and share their halo cells in that L2.  The grid is a multiple
// of 8 (launchers round it up) or 1..7 workgroups (one region).
struct XcdWalk {
    int nx, per, x, R, j;
    __device__ XcdWalk(int count)
    {
        nx = (gridDim.x % 8 == 0) ? 8 : 1;
        per = gridDim.x / nx;
        x = blockIdx.x % nx;
        j = blockIdx.x / nx;
        R = (count + nx - 1) / nx;
    }
    __device__ bool next(int count, int &t)
    {
        if (j >= R) return false;
        t = x * R + j;
        j += per;
        return t < count;
    }
};

// Virtual index of workgroup b of a grid of G: a permutation of 0 .. G-1
// under which each XCD (b mod 8) takes runs of consecutive indices, 32 long
// when G is a multiple of 256, 8 long when it is a multiple of 64.  A
// workgroup's first work item, index xcd_run(b) (then + G, + 2G, ...), does
// not depend on any count, and neighbouring items share an L2.
__device__ __forceinline__ int xcd_run(int b, int G)
{
    const int x = b & 7, j = b >> 3;
    if (G % 256 == 0) return (j >> 5) * 256 + x * 32 + (j & 31);
    if (G % 64 == 0) return (j >> 3) * 64 + x * 8 + (j & 7);
    return b;
}

// issued(a, b, ...): the values are needed at this point.  The compiler
// would otherwise sink a load whose result is only used under a later
// branch into that branch, after the loads that decide it, and pay two
// round trips to memory instead of one.  (An empty statement with the values
// as inputs; it emits no instruction.)
__device__ __forceinline__ void issued() {}
template <typename A, typename... R>
__device__ __forceinline__ void issued(A a, R... r)
{
    asm volatile("" ::"v"(a));
    issued(r...);
}

// Grid table of a hierarchy in LDS, for kernels that look a grid up by the
// level of a tile they have just loaded: reading the table (at most MAXLEV
// grids, grid index = level) into LDS at kernel start, alongside the first
// reads of the device counters, keeps those lookups off the chain of
// dependent memory reads (an argument-block read at a tile-dependent offset
// is one more such read).  A workgroup barrier must separate grid_tab_load
// and grid_tab.
struct GridTab {
    static constexpr int W = (int)(sizeof(Grid) / 4);
    int w[MAXLEV][W];
};
__device__ __forceinline__ void grid_tab_load(const View &v, GridTab &s)
{
    const int n = (v.ngrid < MAXLEV ? v.ngrid : MAXLEV) * GridTab::W;
    const int *src = reinterpret_cast<const int *>(v.grids);
    for (int i = threadIdx.x; i < n; i += blockDim.x) s.w[i / GridTab::W][i % GridTab::W] = src[i];
}
// Grid i (workgroup-uniform) from the table, in scalar registers.
__device__ __forceinline__ Grid grid_tab(const GridTab &s, int i)
{
    int w[GridTab::W];
#pragma unroll
    for (int k = 0; k < GridTab::W; ++k) w[k] = __builtin_amdgcn_readfirstlane(s.w[i][k]);
    Grid G;
    __builtin_memcpy(&G, w, sizeof(Grid));
    return G;
}

// Grid `lvl` of a hierarchy when lvl may differ between lanes: a select over
// the grids passed by value (no dynamic indexing of the argument block).
__device__ __forceinline__ Grid grid_lane(const View &v, int lvl)
{
    Grid G = v.gt[0];
    for (int k = 1; k < MAXLEV && k < v.L; ++k)
        if (lvl == k) G = v.gt[k];
    return G;
}

// ----------------------------------------------------------------------------
// physics (Sec. 2): conserved <-> primitive, van Albada slope, AUSM+
// ----------------------------------------------------------------------------
template <typename T, int D>
__device__ __forceinline__ void cons2prim(const T *q, T *w, T g)
{
    T rho = q[0], K = T(0);
    w[0] = rho;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        T v = Ar<T>::div(q[1 + d], rho);
        w[1 + d] = v;
        K = K + v * v;
    }
    w[D + 1] = (g - T(1)) * (q[D + 1] - (T(0.5) * rho) * K);
}

template <typename T>
__device__ __forceinline__ T slope_va(T wm, T w0, T wp)
{
    T a = w0 - wm, b = wp - w0, ab = a * b;
    if constexpr (sizeof(T) == 4) {
        // FP32: with differences below ~1e-19 the denominator underflows and
        // the hardware reciprocal returns inf (0 * inf = NaN); such a slope
        // is below FP32 resolution of the state, so it is taken as zero.
        const T den = a * a + b * b;
        return (ab > T(0) && den >= T(1.1754944e-38f)) ? Ar<T>::div(ab * (a + b), den) : T(0);
    } else {
        return ab > T(0) ? Ar<T>::div(ab * (a + b), a * a + b * b) : T(0);
    }
}

// velocity component along axis dn of a primitive state (selects, so a
// runtime axis stays in registers)
template <typename T, int D>
__device__ __forceinline__ T vel_along(const T *w, int dn)
{
    T u = w[1];
    if (D >= 2) u = dn == 1 ? w[2] : u;
    if (D >= 3) u = dn == 2 ? w[3] : u;
    return u;
}

// AUSM+ (Liou 1996) across a face with normal along axis dn; wL, wR are the
// primitive face states; gi = 1 / (gamma - 1).
// cs selects the interface sound speed: 0 the mean of the two sound speeds,
// 1 Liou's critical speed min(c*_L^2 / max(c*_L, u_L), c*_R^2 / max(c*_R,
// -u_R)), c*^2 = 2 (gamma - 1) / (gamma + 1) H with H the total enthalpy.
template <typename T, int D>
__device__ __forceinline__ void ausm_plus(T g, T gi, int dn, const T *wL, const T *wR, T *F, int cs = 0)
{
    const T rL = wL[0], pL = wL[D + 1], uL = vel_along<T, D>(wL, dn);
    const T rR = wR[0], pR = wR[D + 1], uR = vel_along<T, D>(wR, dn);
    T ch;
    if (cs) {
        T KL = T(0), KR = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            KL = KL + wL[1 + k] * wL[1 + k];
            KR = KR + wR[1 + k] * wR[1 + k];
        }
        const T HL = Ar<T>::div((pL * gi + (T(0.5) * rL) * KL) + pL, rL);
        const T HR = Ar<T>::div((pR * gi + (T(0.5) * rR) * KR) + pR, rR);
        const T kc = (T)((2.0 * ((double)g - 1.0)) / ((double)g + 1.0));
        const T sL = kc * HL, sR = kc * HR;
        const T csL = Ar<T>::sqrt(sL), csR = Ar<T>::sqrt(sR);
        const T tL = Ar<T>::div(sL, csL >= uL ? csL : uL);
        const T tR = Ar<T>::div(sR, csR >= -uR ? csR : -uR);
        ch = tL <= tR ? tL : tR;
    } else {
        const T cL = Ar<T>::sqrt(Ar<T>::div(g * pL, rL));
        const T cR = Ar<T>::sqrt(Ar<T>::div(g * pR, rR));
        ch = T(0.5) * (cL + cR);
    }
    const T ML = Ar<T>::div(uL, ch), MR = Ar<T>::div(uR, ch);
    T Mp, Pp, Mm, Pm;
    if (Ar<T>::abs(ML) >= T(1)) {
        Mp = T(0.5) * (ML + Ar<T>::abs(ML));
        Pp = ML > T(0) ? T(1) : T(0);
    } else {
        const T a = ML + T(1), b = ML - T(1);
        const T m2p = T(0.25) * (a * a), m2m = T(-0.25) * (b * b);
        Mp = m2p * (T(1) - T(2) * m2m);
        Pp = m2p * ((T(2) - ML) - (T(3) * ML) * m2m);
    }
    if (Ar<T>::abs(MR) >= T(1)) {
        Mm = T(0.5) * (MR - Ar<T>::abs(MR));
        Pm = MR < T(0) ? T(1) : T(0);
    } else {
        const T a = MR + T(1), b = MR - T(1);
        const T m2p = T(0.25) * (a * a), m2m = T(-0.25) * (b * b);
        Mm = m2m * (T(1) + T(2) * m2p);
        Pm = m2m * ((T(-2) - MR) + (T(3) * MR) * m2p);
    }
    const T mh = Mp + Mm;
    const T ph = Pp * pL + Pm * pR;
    const T mf = ch * mh;
    const bool up = mh >= T(0);
    T wu[D + 2];
#pragma unroll
    for (int f = 0; f < D + 2; ++f) {
        const T l = wL[f], r = wR[f];   // select values, not addresses (keeps the arrays in registers)
        wu[f] = up ? l : r;
    }
    const T ru = wu[0], pu = wu[D + 1];
    T K = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) K = K + wu[1 + k] * wu[1 + k];
    const T rH = (pu * gi + (T(0.5) * ru) * K) + pu;
    F[0] = mf * ru;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T fk = mf * (ru * wu[1 + k]);
        F[1 + k] = k == dn ? fk + ph : fk;
    }
    F[D + 1] = mf * rH;
}

// Face flux from the primitive states of the 4 cells i-1, i, i+1, i+2 along dn.
template <typename T, int D>
__device__ __forceinline__ void face_flux4(T g, T gi, int dn, const T *wa, const T *wb, const T *wc,
                                           const T *wd, T *F, int cs = 0)
{
    T wL[D + 2], wR[D + 2];
#pragma unroll
    for (int f = 0; f < D + 2; ++f) {
        wL[f] = wb[f] + T(0.5) * slope_va<T>(wa[f], wb[f], wc[f]);
        wR[f] = wc[f] - T(0.5) * slope_va<T>(wb[f], wc[f], wd[f]);
    }
    ausm_plus<T, D>(g, gi, dn, wL, wR, F, cs);
}

// Mean of the 2^(D-1) fine fluxes on the face between coarse cell p (global
// coordinates on its grid) and its covered neighbour on side s of axis dn,
// computed from the next finer grid gf of the stencil source (virtual
// leaves, Sec. 2.1).  Transverse offsets: first along the lower transverse axis.
template <typename T, int D>
__device__ void fine_mean(const View &v, const Grid &gf, const T *src, int px, int py, int pz, int s,
                          int dn, T g, T gi, T *F)
{
    const T *S = src + gf.off;
    const int nf = gf.n;
    const int64_t Nf = gf.ncell;
    const int along = dn == 0 ? px : dn == 1 ? py : pz;
    const int bd = s > 0 ? 2 * along + 1 : 2 * along - 1;
    const int t1 = dn == 0 ? 1 : 0;   // lower transverse axis
    const int t2 = dn == 2 ? 1 : 2;   // upper transverse axis (3D)
    constexpr int NS = D == 2 ? 2 : 4;
    T Fs[NS][D + 2];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int o1 = k & 1, o2 = D == 3 ? (k >> 1) & 1 : 0;
        int c[3] = {2 * px, 2 * py, 2 * pz};
#pragma unroll
        for (int a = 0; a < 3; ++a) c[a] += (a == t1 ? o1 : 0) + (a == t2 ? o2 : 0);
        T w[4][D + 2];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int e = bcmap(bd + j - 1, nf, v.bc);
            const int ex = dn == 0 ? e : c[0], ey = dn == 1 ? e : c[1], ez = dn == 2 ? e : c[2];
            const int64_t id = gidx(nf, ex, ey, D == 3 ? ez : 0);
            T q[D + 2];
#pragma unroll
            for (int f = 0; f < D + 2; ++f) q[f] = S[f * Nf + id];
            cons2prim<T, D>(q, w[j], g);
        }
        face_flux4<T, D>(g, gi, dn, w[0], w[1], w[2], w[3], Fs[k], v.ausm_cs);
    }
#pragma unroll
    for (int f = 0; f < D + 2; ++f) {
        if (D == 2) F[f] = T(0.5) * (Fs[0][f] + Fs[1][f]);
        else F[f] = T(0.25) * ((Fs[0][f] + Fs[1][f]) + (Fs[2][f] + Fs[3][f]));
    }
}

// ----------------------------------------------------------------------------
// MR operators (Sec. 2.1)
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T pred1(T qm, T q0, T qp, int upper)
{
    const T s8 = upper ? T(-0.125) : T(0.125);
    return q0 + s8 * (qm - qp);
}

// Third-order prediction of child ch of coarse cell p for one field (array A
// is the coarse field, n its side), separable x, then y, then z.
template <typename T, int D, typename TA>
__device__ __forceinline__ T predict_child(const TA *A, int n, int bc, int px, int py, int pz,
                                           int cx, int cy, int cz)
{
    int xs[3], ys[3], zs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xs[k] = bcmap(px + k - 1, n, bc);
        ys[k] = bcmap(py + k - 1, n, bc);
        zs[k] = D == 3 ? bcmap(pz + k - 1, n, bc) : 0;
    }
    if (D == 2) {
        T r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] = pred1<T>((T)A[gidx(n, xs[0], ys[j], 0)], (T)A[gidx(n, xs[1], ys[j], 0)],
                            (T)A[gidx(n, xs[2], ys[j], 0)], cx);
        return pred1<T>(r[0], r[1], r[2], cy);
    }
    T s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] = pred1<T>((T)A[gidx(n, xs[0], ys[j], zs[k])], (T)A[gidx(n, xs[1], ys[j], zs[k])],
                            (T)A[gidx(n, xs[2], ys[j], zs[k])], cx);
        s[k] = pred1<T>(r[0], r[1], r[2], cy);
    }
    return pred1<T>(s[0], s[1], s[2], cz);
}

// Projection: mean of the 2^D children (pairwise order).
template <typename T, int D>
__device__ __forceinline__ T restrict_cell(const T *Af, int nf, int px, int py, int pz)
{
    const int x = 2 * px, y = 2 * py, z = 2 * pz;
    if (D == 2)
        return T(0.25) * ((Af[gidx(nf, x, y, 0)] + Af[gidx(nf, x + 1, y, 0)]) +
                          (Af[gidx(nf, x, y + 1, 0)] + Af[gidx(nf, x + 1, y + 1, 0)]));
    return T(0.125) * (((Af[gidx(nf, x, y, z)] + Af[gidx(nf, x + 1, y, z)]) +
                        (Af[gidx(nf, x, y + 1, z)] + Af[gidx(nf, x + 1, y + 1, z)])) +
                       ((Af[gidx(nf, x, y, z + 1)] + Af[gidx(nf, x + 1, y, z + 1)]) +
                        (Af[gidx(nf, x, y + 1, z + 1)] + Af[gidx(nf, x + 1, y + 1, z + 1)])));
}

__device__ __forceinline__ bool block_active(const View &v, const uint8_t *mask, const Grid &G,
                                             int x, int y, int z)
{
    return mask[G.boff + (int64_t)gidx32(G.nb, x >> 3, y >> 3, z >> 3)] != 0;
}

// covered: the children of cell (x, y, z) belong to a patch of the finer
// grid F (the caller checks that the cell's grid has one).
__device__ __forceinline__ bool covered(const uint8_t *mask, const Grid &F, int x, int y, int z)
{
    return mask[F.boff + (int64_t)gidx32(F.nb, x >> 2, y >> 2, z >> 2)] != 0;
}

// ----------------------------------------------------------------------------
// finite-volume stage on every leaf of the tiles of the leaf list
// ----------------------------------------------------------------------------
// Tile geometry of the stage kernel: one BS^D block with a 2-cell halo,
// NT threads.
template <int D, int NT_> struct FV {
    static constexpr int B = BS, H = 2, E = BS + 4;
    static constexpr int NT = NT_;
    static constexpr int NE = D == 2 ? E * E : E * E * E;
    static constexpr int NV = D + 2;
    static constexpr int TC = D == 2 ? B * B : B * B * B;
    static constexpr int CPT = (TC + NT - 1) / NT;
    static constexpr int NF = (B + 1) * (D == 2 ? B : B * B);   // faces per axis
    static constexpr int NS = (B + 2) * (D == 2 ? B : B * B);   // cells -1 .. B of the lines of an axis
};

// Face layout of axis dn: face a (0..B) between local cells a-1 and a along
// dn, on the line given by the other coordinates; x varies fastest in every
// axis' layout, so consecutive lanes read consecutive LDS words for every
// axis (a layout with the axis coordinate fastest puts y and z faces on a
// few LDS banks).  Returns a and the left cell's local coordinates.
template <int D, int B>
__device__ __forceinline__ void face_coords(int dn, int fi, int &a, int &lx, int &ly, int &lz)
{
    if (dn == 0) {
        a = fi % (B + 1);
        const int r = fi / (B + 1);
        lx = a - 1;
        ly = r % B;
        lz = D == 3 ? r / B : 0;
    } else if (dn == 1) {
        lx = fi % B;
        const int q = fi / B;
        a = q % (B + 1);
        ly = a - 1;
        lz = D == 3 ? q / (B + 1) : 0;
    } else {
        lx = fi % B;
        ly = (fi / B) % B;
        a = fi / (B * B);
        lz = a - 1;
    }
}
// Index of the per-cell face states of axis dn for the cell at position
// p - 1 (p = 0..B+1) along dn on the line of cell (lx, ly, lz); x fastest.
template <int B>
__device__ __forceinline__ int cell_state_idx(int dn, int lx, int ly, int lz, int p)
{
    return dn == 0 ? p + (B + 2) * (ly + B * lz) : dn == 1 ? lx + B * (p + (B + 2) * lz) : lx + B * (ly + B * p);
}

// Flux of face fi of axis dn of the tile (fi = a + (B+1) r: a-th face along
// the axis, r-th line across it), written to F.
// With sFm/sFp given (per-cell face states of axis dn, see k_fv_stage), the
// face states of a face between two cells of the tile's level are read from
// them instead of being reconstructed here.
template <typename T, int D, int NT>
__device__ __forceinline__ void fv_face(const View &v, const Grid &G, const Grid &GF, const T *src, int ox, int oy, int oz,
                                        const T (*sW)[FV<D, NT>::NE], const uint8_t *sCov,
                                        const uint8_t *sAct, T g, T gi, bool lts, bool record, int sub,
                                        int dn, int fi, T *F, const T (*sFm)[FV<D, NT>::NS] = nullptr,
                                        const T (*sFp)[FV<D, NT>::NS] = nullptr)
{
    using C = FV<D, NT>;
    constexpr int E = C::E, H = C::H, B = C::B;
    const int SD = dn == 0 ? 1 : dn == 1 ? E : E * E;
    // face a (0..B) along axis dn; local coordinates of its left cell
    int a, lx, ly, lz;
    face_coords<D, B>(dn, fi, a, lx, ly, lz);
    const int hl = (lx + H) + E * ((ly + H) + (D == 3 ? E * (lz + H) : 0));
    const int hr = hl + SD;
    const bool lin = a >= 1, rin = a <= B - 1;
    const bool lcov = sCov[hl] != 0, rcov = sCov[hr] != 0;
    // global mode: fluxes of faces next to a leaf of the tile; local time
    // stepping: every face of the tile (whole patches are updated)
    const bool need = lts ? (lin || rin) : ((lin && !lcov) || (rin && !rcov));
    if (!need) {
#pragma unroll
        for (int f = 0; f < D + 2; ++f) F[f] = T(0);
        return;
    }
    if (!lts && (lcov || rcov)) {
        int px = ox + lx, py = oy + ly, pz = oz + lz, s = +1;
        if (lcov) {
            s = -1;
            px += dn == 0 ? 1 : 0;
            py += dn == 1 ? 1 : 0;
            pz += dn == 2 ? 1 : 0;
        }
        fine_mean<T, D>(v, GF, src, px, py, D == 3 ? pz : 0, s, dn, g, gi, F);
        return;
    }
    if (sFp) {
        // left cell a-1 and right cell a of line r: entries a and a+1
        T wL[D + 2], wR[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) {
            wL[f] = sFp[f][cell_state_idx<B>(dn, lx, ly, lz, a)];
            wR[f] = sFm[f][cell_state_idx<B>(dn, lx, ly, lz, a + 1)];
        }
        ausm_plus<T, D>(g, gi, dn, wL, wR, F, v.ausm_cs);
    } else {
        T wa[D + 2], wb[D + 2], wc[D + 2], wd[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) {
            wa[f] = sW[f][hl - SD];
            wb[f] = sW[f][hl];
            wc[f] = sW[f][hr];
            wd[f] = sW[f][hr + SD];
        }
        face_flux4<T, D>(g, gi, dn, wa, wb, wc, wd, F, v.ausm_cs);
    }
    if (record) {
        // registers are indexed by the cell on the low side of the face
        int qx = ox + lx, qy = oy + ly, qz = oz + lz;
        if (dn == 0) qx = bcmap(qx, G.n, v.bc);
        else if (dn == 1) qy = bcmap(qy, G.n, v.bc);
        else qz = bcmap(qz, G.n, v.bc);
        const int64_t iq = gidx(G.n, qx, qy, D == 3 ? qz : 0);
        const bool lact = sAct[hl] != 0, ract = sAct[hr] != 0;
        const bool lleaf = lact && !lcov, rleaf = ract && !rcov;
        T *reg = (T *)v.reg;
        if (G.rcoff >= 0 && ((lleaf && rcov) || (rleaf && lcov)))
#pragma unroll
            for (int f = 0; f < D + 2; ++f) reg[G.rcoff + ((int64_t)dn * (D + 2) + f) * G.ncell + iq] = F[f];
        if (G.rfoff >= 0 && lact != ract)
#pragma unroll
            for (int f = 0; f < D + 2; ++f)
                reg[G.rfoff + (((int64_t)sub * D + dn) * (D + 2) + f) * G.ncell + iq] = F[f];
    }
}

// Residual of the thread's cells along axis dn, accumulated axis by axis in
// the order ((dF_1 + dF_2) + dF_3), dF = F_{+1/2} - F_{-1/2}.
template <typename T, int D, int NT>
__device__ __forceinline__ void fv_collect(const T (*sF)[FV<D, NT>::NF], T (*R)[D + 2], int dn)
{
    using C = FV<D, NT>;
    constexpr int B = C::B;
#pragma unroll
    for (int k = 0; k < C::CPT; ++k) {
        const int c = threadIdx.x + k * C::NT;
        if (c >= C::TC) break;
        const int x = c % B, y = (c / B) % B, z = c / (B * B);
        // faces x and x+1 of the cell along axis dn (x-fastest face layout)
        const int lo = dn == 0 ? x + (B + 1) * (y + B * z) : dn == 1 ? x + B * (y + (B + 1) * z) : x + B * (y + B * z);
        const int hi = lo + (dn == 0 ? 1 : dn == 1 ? B : B * B);
#pragma unroll
        for (int f = 0; f < D + 2; ++f) {
            const T d = sF[f][hi] - sF[f][lo];
            R[k][f] = dn == 0 ? d : R[k][f] + d;
        }
    }
}

// One explicit stage: out = base - lam ((dF_1 + dF_2) + dF_3), lam = (dt *
// fac) / dx (FP64, then cast), fluxes from src.  Global time step (lvl < 0):
// every leaf of every level (leaf list), faces next to a covered cell take
// the fine-flux mean.  Local time stepping (lvl >= 0): every cell in a patch
// of level lvl with the level's own fluxes; with record set, fluxes across
// refinement boundaries go to the flux registers (substep sub).
// blend (Heun's second stage): out = (base + src) / 2 - lam R.
// Schedules (bit-identical FP64 results): SCHED 0 computes the faces axis
// by axis (one LDS flux array reused per axis); SCHED 2 does the same but
// first reconstructs the two face states of every cell of the axis' lines
// once (slope, then W -/+ slope/2) instead of twice per cell, once for each
// of its faces; SCHED 1 computes the
// faces of all axes in one pass over all threads (one array per axis).
// fineproj (2D hierarchy, global step): a tile of the finest level L-1
// also writes the projection of its cells (the values it has just written)
// onto its 4x4 parent cells of level L-2, all of them covered: every cell of
// a finest block is a leaf, and no other workgroup of the launch reads those
// cells of out.
template <typename T, int D, int NT, int SCHED>
__global__ void __launch_bounds__(NT)
k_fv_stage(View v, const T *__restrict__ src, const T *base, T *out, double fac, int lvl, int sub,
           int record, int fineproj, int blend)
{
    using C = FV<D, NT>;
    constexpr int E = C::E, H = C::H, B = C::B, NV = C::NV;
    constexpr bool MERGED = SCHED == 1;
    constexpr bool CELLS = SCHED == 2;
    constexpr int NA = MERGED ? D : 1;   // flux arrays held at once
    __shared__ T sW[NV][C::NE];
    __shared__ T sF[NA][NV][C::NF];
    __shared__ T sFm[CELLS ? NV : 1][CELLS ? C::NS : 1], sFp[CELLS ? NV : 1][CELLS ? C::NS : 1];
    __shared__ uint8_t sCov[C::NE];
    __shared__ uint8_t sAct[C::NE];
    __shared__ GridTab tab;
    // first reads, independent of each other: counters, grid table, dt
    const bool lts = lvl >= 0;
    const bool hier = v.mode == MODE_HIER;
    const int done = v.meta->done;
    const Tile *list = lts ? v.actv + v.meta->loff[LST_ACT][lvl] : v.leaf;
    const int count = lts ? v.meta->loff[LST_ACT][lvl + 1] - v.meta->loff[LST_ACT][lvl] : v.meta->nleaf;
    const double dt0 = v.dt[lts ? lvl : 0];
    // One pass over an adaptive hierarchy's leaf list (a few thousand tiles
    // at most, latency-bound) gives workgroup b a tile that does not depend
    // on the count, tf, then tf + gridDim.x, ...: the first entry is read
    // with the count, one round trip less before the halo loads.  Workgroup
    // b runs on XCD b mod 8; with a grid of a multiple of 256 workgroups
    // each XCD takes runs of 32 consecutive tiles (list neighbours share its
    // L2; runs of 4, 8 and 16 measured slower).
    // Other passes (uniform grids, batches, a level of local time stepping)
    // walk their tiles XCD by XCD.
    const bool inter = hier && !lts && v.L > 1;
    const int tf = xcd_run(blockIdx.x, gridDim.x);
    const int t0 = tf < v.max_tiles ? tf : v.max_tiles - 1;
    const Tile first = inter ? v.leaf[t0] : Tile{0, 0};
    if (hier) grid_tab_load(v, tab);
    issued(list, count, dt0, first.grid, first.block);
    if (done) return;
    __syncthreads();
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    XcdWalk walk(count);
    int t = inter ? tf - (int)gridDim.x : 0;
    while (inter ? (t += gridDim.x) < count : walk.next(count, t)) {
        Tile tl;
        if (inter && t == tf) tl = first;
        else tl = list[t];
        const Grid G = hier ? grid_tab(tab, tl.grid) : v.grids[tl.grid];
        const bool hasf = G.fine >= 0;
        const Grid GF = hasf ? grid_tab(tab, G.fine) : G;
        const int n = G.n, nb = G.nb;
        const int ox = (tl.block % nb) * B;
        const int oy = ((tl.block / nb) % nb) * B;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * B : 0;
        const T *S = src + G.off;
        const int64_t N = G.ncell;
        // the tile with its halo.  2D: every read of the thread's cells
        // (states and masks, from valid addresses) issued before any is used;
        // 3D: cell by cell (the registers of all of them would cost occupancy)
        if constexpr (D == 2) {
            constexpr int IE = (C::NE + NT - 1) / NT;
            T qh[IE][NV];
            uint8_t cvb[IE], acb[IE];
#pragma unroll
            for (int u = 0; u < IE; ++u) {
                const int c0 = threadIdx.x + u * NT, c = c0 < C::NE ? c0 : C::NE - 1;
                const int lx = c % E, ly = c / E;
                const int x = bcmap(ox + lx - H, n, v.bc), y = bcmap(oy + ly - H, n, v.bc);
                const int64_t id = gidx32(n, x, y, 0);
#pragma unroll
                for (int f = 0; f < NV; ++f) qh[u][f] = S[f * N + id];
                // children's block on the finer grid (block 0 of the own grid
                // when there is none: a valid address, the value unused)
                const int64_t cb = hasf ? GF.boff + (int64_t)gidx32(GF.nb, x >> 2, y >> 2, 0) : G.boff;
                cvb[u] = v.act[cb];
                acb[u] = v.act[G.boff + (int64_t)gidx32(G.nb, x >> 3, y >> 3, 0)];
            }
#pragma unroll
            for (int u = 0; u < IE; ++u) {
                const int c = threadIdx.x + u * NT;
                if (c >= C::NE) break;
                T w[NV];
                cons2prim<T, D>(qh[u], w, g);
#pragma unroll
                for (int f = 0; f < NV; ++f) sW[f][c] = w[f];
                sCov[c] = hasf && cvb[u] != 0 ? 1 : 0;
                if (record) sAct[c] = acb[u] != 0 ? 1 : 0;
            }
        } else {
            for (int c = threadIdx.x; c < C::NE; c += NT) {
                const int lx = c % E, ly = (c / E) % E, lz = c / (E * E);
                const int x = bcmap(ox + lx - H, n, v.bc);
                const int y = bcmap(oy + ly - H, n, v.bc);
                const int z = bcmap(oz + lz - H, n, v.bc);
                const int64_t id = gidx32(n, x, y, z);
                T q[NV], w[NV];
#pragma unroll
                for (int f = 0; f < NV; ++f) q[f] = S[f * N + id];
                const bool cv = hasf && covered(v.act, GF, x, y, z);
                const bool ac = record && block_active(v, v.act, G, x, y, z);
                cons2prim<T, D>(q, w, g);
#pragma unroll
                for (int f = 0; f < NV; ++f) sW[f][c] = w[f];
                sCov[c] = cv ? 1 : 0;
                if (record) sAct[c] = ac ? 1 : 0;
            }
        }
        // base state of the thread's cells, read while the fluxes are computed
        // (blend: Heun's second stage, the base is (base + src) / 2)
        T qb[C::CPT][NV];
#pragma unroll
        for (int k = 0; k < C::CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= C::TC) break;
            const int x = c % B, y = (c / B) % B, z = c / (B * B);
            const int64_t id = G.off + (int64_t)gidx32(n, ox + x, oy + y, oz + z);
#pragma unroll
            for (int f = 0; f < NV; ++f) qb[k][f] = base[f * N + id];
            if (blend)
#pragma unroll
                for (int f = 0; f < NV; ++f) qb[k][f] = T(0.5) * (qb[k][f] + src[f * N + id]);
        }
        __syncthreads();
        T R[C::CPT][NV];
        if constexpr (MERGED) {
            for (int j = threadIdx.x; j < D * C::NF; j += NT) {
                const int dn = j / C::NF, fi = j - dn * C::NF;
                T F[NV];
                fv_face<T, D, NT>(v, G, GF, src, ox, oy, oz, sW, sCov, sAct, g, gi, lts, record, sub, dn, fi, F);
#pragma unroll
                for (int f = 0; f < NV; ++f) sF[dn][f][fi] = F[f];
            }
            __syncthreads();
#pragma unroll
            for (int dn = 0; dn < D; ++dn) fv_collect<T, D, NT>(sF[dn], R, dn);
        } else {
#pragma unroll
            for (int dn = 0; dn < D; ++dn) {
                if constexpr (CELLS) {
                    // face states of cells -1 .. B of every line of axis dn
                    const int SD = dn == 0 ? 1 : dn == 1 ? E : E * E;
                    for (int c = threadIdx.x; c < C::NS; c += NT) {
                        // cell p - 1 along dn (p = 0..B+1), x fastest as in cell_state_idx
                        int lx, ly, lz;
                        if (dn == 0) {
                            lx = c % (B + 2) - 1;
                            ly = (c / (B + 2)) % B;
                            lz = D == 3 ? c / ((B + 2) * B) : 0;
                        } else if (dn == 1) {
                            lx = c % B;
                            ly = (c / B) % (B + 2) - 1;
                            lz = D == 3 ? c / (B * (B + 2)) : 0;
                        } else {
                            lx = c % B;
                            ly = (c / B) % B;
                            lz = c / (B * B) - 1;
                        }
                        const int h = (lx + H) + E * ((ly + H) + (D == 3 ? E * (lz + H) : 0));
#pragma unroll
                        for (int f = 0; f < NV; ++f) {
                            const T w0 = sW[f][h];
                            const T sl = slope_va<T>(sW[f][h - SD], w0, sW[f][h + SD]);
                            sFm[f][c] = w0 - T(0.5) * sl;
                            sFp[f][c] = w0 + T(0.5) * sl;
                        }
                    }
                    __syncthreads();
                }
                for (int fi = threadIdx.x; fi < C::NF; fi += NT) {
                    T F[NV];
                    if constexpr (CELLS)
                        fv_face<T, D, NT>(v, G, GF, src, ox, oy, oz, sW, sCov, sAct, g, gi, lts, record, sub, dn, fi, F,
                                          sFm, sFp);
                    else
                        fv_face<T, D, NT>(v, G, GF, src, ox, oy, oz, sW, sCov, sAct, g, gi, lts, record, sub, dn, fi, F);
#pragma unroll
                    for (int f = 0; f < NV; ++f) sF[0][f][fi] = F[f];
                }
                __syncthreads();
                fv_collect<T, D, NT>(sF[0], R, dn);
                __syncthreads();
            }
        }
        const double dt = v.mode == MODE_BATCH ? v.dt[tl.grid] : dt0;
        const T lam = (T)((dt * fac) / G.dx);
        const bool fp = D == 2 && fineproj && tl.grid == v.L - 1;
#pragma unroll
        for (int k = 0; k < C::CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= C::TC) break;
            const int x = c % B, y = (c / B) % B, z = c / (B * B);
            const int h = (x + H) + E * ((y + H) + (D == 3 ? E * (z + H) : 0));
            if (!lts && sCov[h]) continue;
            const int64_t id = G.off + (int64_t)gidx32(n, ox + x, oy + y, oz + z);
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                const T q = qb[k][f] - lam * R[k][f];
                out[f * N + id] = q;
                if (fp) sW[f][c] = q;   // the flux phase no longer reads sW
            }
        }
        if (D == 2 && fp) {
            __syncthreads();
            if (threadIdx.x < (B / 2) * (B / 2)) {
                // parent (px, py): the mean of its children in the pairwise
                // order of the projection kernels
                const int px = threadIdx.x % (B / 2), py = threadIdx.x / (B / 2);
                const Grid P = grid_tab(tab, G.coarse);
                const int64_t ip = P.off + gidx(P.n, (ox >> 1) + px, (oy >> 1) + py, 0);
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    const int c0 = (2 * py) * B + 2 * px;
                    out[ip + f * P.ncell] =
                        T(0.25) * ((sW[f][c0] + sW[f][c0 + 1]) + (sW[f][c0 + B] + sW[f][c0 + B + 1]));
                }
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// CFL reduction over leaves (FP64): per-grid max of the signal speed, then
// dt (second kernel)
// ----------------------------------------------------------------------------
// Hierarchy: workgroup b writes its per-level maxima and its count of leaf
// cells advanced to column b of the level-major partials (plain stores; the
// kernel boundary publishes them).  Batch: one atomic max per tile on its
// instance.

// Signal speed of a cell from its conserved state (FP64): sum_d (|v_d| + c),
// or with mx the largest |v_d| + c; bad when its density or pressure is not
// positive.
template <int D>
__device__ __forceinline__ double cell_speed(const double *q, double g, int mx, bool &bad)
{
#pragma clang fp contract(off)
    double w[D + 2];
    cons2prim<double, D>(q, w, g);
    bad = !(w[0] > 0.0) || !(w[D + 1] > 0.0);
    const double cs = __builtin_sqrt((g * w[D + 1]) / w[0]);
    double S = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double sd = __builtin_fabs(w[1 + d]) + cs;
        S = mx ? (sd > S ? sd : S) : S + sd;
    }
    return S;
}

// Per-level maxima and leaf count of one workgroup (the wave's row; lane 0
// adds the wave's share of a tile of level lv)
__device__ __forceinline__ void cfl_tile_done(double (*lmax)[MAXLEV], unsigned long long *lcnt, const View &v,
                                              int lv, double m, int nl)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int o = 32; o > 0; o >>= 1) {
        const double r = __shfl_xor(m, o);
        m = r > m ? r : m;
        nl += __shfl_xor(nl, o);
    }
    if (lane == 0) {
        // leaf cells advanced this step (a level-l leaf 2^l times with local
        // time stepping)
        lcnt[wave] += (unsigned long long)nl << (v.lts ? lv : 0);
        if (m > lmax[wave][lv]) lmax[wave][lv] = m;
    }
}

// The workgroup's maxima over its waves and its leaf count, added into CFL
// slot blockIdx.x mod CFL_NSLOT (vector atomics; zeros add nothing).
template <int NW>
__device__ __forceinline__ void cfl_publish(const double (*lmax)[MAXLEV], const unsigned long long *lcnt,
                                            const View &v)
{
    const int l = threadIdx.x, slot = blockIdx.x % CFL_NSLOT;
    if (l < MAXLEV && l < v.L) {
        double mm = lmax[0][l];
        for (int w = 1; w < NW; ++w) mm = lmax[w][l] > mm ? lmax[w][l] : mm;
        if (mm > 0.0) atomicMax(v.cfls + cfl_slot(l, slot), (unsigned long long)__double_as_longlong(mm));
    } else if (l == MAXLEV) {
        unsigned long long c = lcnt[0];
        if (NW == 4) c = (lcnt[0] + lcnt[1]) + (lcnt[2] + lcnt[3]);
        if (c) atomicAdd(v.cfls + cfl_slot(MAXLEV, slot), c);
    }
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_cfl(View v, const T *__restrict__ Q)
{
#pragma clang fp contract(off)
    __shared__ double lmax[4][MAXLEV];
    __shared__ unsigned long long lcnt[4];
    __shared__ GridTab tab;
    const bool hier = v.mode == MODE_HIER;
    const int count = v.meta->nleaf;
    if (hier) grid_tab_load(v, tab);
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS;
    const double g = v.gamma;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane < MAXLEV) lmax[wave][lane] = 0.0;
    if (lane == 0) lcnt[wave] = 0ull;
    __syncthreads();
    bool bad = false;
    for (int t = blockIdx.x * 4 + wave; t < count; t += gridDim.x * 4) {
        const Tile tl = v.leaf[t];
        const Grid G = hier ? grid_tab(tab, tl.grid) : v.grids[tl.grid];
        const bool hasf = G.fine >= 0;
        const Grid GF = hasf ? grid_tab(tab, G.fine) : G;
        const int n = G.n, nb = G.nb;
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
        double m = 0.0;
        int nl = 0;   // leaf cells of the tile
        for (int c = lane; c < TC; c += 64) {
            const int x = ox + c % BS, y = oy + (c / BS) % BS, z = oz + (D == 3 ? c / (BS * BS) : 0);
            const int64_t id = G.off + gidx(n, x, y, z);
            // the state is read whether or not the cell is covered (a
            // covered cell holds its children's mean); it only counts for
            // leaves
            double q[D + 2];
#pragma unroll
            for (int f = 0; f < D + 2; ++f) q[f] = (double)Q[f * G.ncell + id];
            const bool leaf = !(hasf && covered(v.act, GF, x, y, z));
            bool b;
            const double S = cell_speed<D>(q, g, v.cfl_max, b);
            if (leaf && b) bad = true;
            if (leaf && S > m) m = S;
            nl += leaf ? 1 : 0;
        }
        if (hier) {
            cfl_tile_done(lmax, lcnt, v, tl.grid, m, nl);
        } else {
            for (int o = 32; o > 0; o >>= 1) {
                const double r = __shfl_xor(m, o);
                m = r > m ? r : m;
            }
            if (lane == 0 && m > 0.0) atomicMax(&v.smax[tl.grid], (unsigned long long)__double_as_longlong(m));
        }
    }
    if (__any(bad) && lane == 0) atomicOr(&v.meta->status, 1);
    __syncthreads();
    if (hier) cfl_publish<4>(lmax, lcnt, v);
}

// ----------------------------------------------------------------------------
// conserved totals: per-tile partial sums in a fixed order (FP64)
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_totals(View v, const T *__restrict__ Q)
{
#pragma clang fp contract(off)
    __shared__ double sm[D + 2][256];
    const int count = v.meta->nleaf;
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const Tile tl = v.leaf[t];
        const Grid G = v.grids[tl.grid];
        const bool hasf = G.fine >= 0;
        const Grid GF = hasf ? v.grids[G.fine] : G;
        const int n = G.n, nb = G.nb;
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
        const double vol = D == 2 ? G.dx * G.dx : G.dx * G.dx * G.dx;
        double acc[D + 2];
#pragma unroll
        for (int f = 0; f < D + 2; ++f) acc[f] = 0.0;
        for (int c = threadIdx.x; c < TC; c += blockDim.x) {
            const int x = ox + c % BS, y = oy + (c / BS) % BS, z = oz + (D == 3 ? c / (BS * BS) : 0);
            if (hasf && covered(v.act, GF, x, y, z)) continue;
            const int64_t id = G.off + gidx(n, x, y, z);
#pragma unroll
            for (int f = 0; f < D + 2; ++f) acc[f] = acc[f] + (double)Q[f * G.ncell + id] * vol;
        }
#pragma unroll
        for (int f = 0; f < D + 2; ++f) sm[f][threadIdx.x] = acc[f];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s)
#pragma unroll
                for (int f = 0; f < D + 2; ++f) sm[f][threadIdx.x] += sm[f][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x < D + 2) v.partial[(int64_t)t * (D + 2) + threadIdx.x] = sm[threadIdx.x][0];
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// initial data (cell-centre sampling, FP64 arithmetic, then cast)
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_init(View v, InitArgs a, int grid, T *Q)
{
#pragma clang fp contract(off)
    const Grid G = v.grids[grid];
    const int n = G.n;
    const double g = v.gamma, gi = 1.0 / (g - 1.0);
    const double lo = a.lo, dx = (a.hi - a.lo) / (double)n;
    const int64_t N = G.ncell;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = D == 3 ? (int)(i / ((int64_t)n * n)) : 0;
        const double xc = lo + ((double)x + 0.5) * dx;
        const double yc = lo + ((double)y + 0.5) * dx;
        const double zc = lo + ((double)z + 0.5) * dx;
        double w[5] = {0, 0, 0, 0, 0};
        if (a.kind == 0) {  // four quadrants (2D)
            const int qd = xc > a.x0 ? (yc > a.y0 ? 0 : 3) : (yc > a.y0 ? 1 : 2);
            w[0] = a.quad[qd][0]; w[1] = a.quad[qd][1]; w[2] = a.quad[qd][2];
            w[D + 1] = a.quad[qd][3];
        } else if (a.kind == 1) {  // rotated ellipsoid (3D)
            const double x1 = xc * a.ell[3] - yc * a.ell[4];
            const double s = xc * a.ell[4] + yc * a.ell[3];
            const double x2 = s * a.ell[5] - zc * a.ell[6];
            const double x3 = s * a.ell[6] + zc * a.ell[5];
            const double r2 = ((x1 / a.ell[0]) * (x1 / a.ell[0]) + (x2 / a.ell[1]) * (x2 / a.ell[1])) +
                              (x3 / a.ell[2]) * (x3 / a.ell[2]);
            const bool in = r2 < a.ell[7] * a.ell[7];
            w[0] = in ? a.es[0] : a.es[2];
            w[D + 1] = in ? a.es[1] : a.es[3];
        } else if (a.kind == 2) {  // 1D Riemann problem along an axis
            const double xa = a.axis == 0 ? xc : a.axis == 1 ? yc : zc;
            const int s = xa < a.split ? 0 : 3;
            w[0] = a.lr[s];
            w[1 + a.axis] = a.lr[s + 1];
            w[D + 1] = a.lr[s + 2];
        } else {  // uniform state
            for (int f = 0; f < D + 2; ++f) w[f] = a.uni[f];
        }
        double K = 0.0;
        Q[G.off + i] = (T)w[0];
        for (int d = 0; d < D; ++d) {
            Q[G.off + (1 + d) * N + i] = (T)(w[0] * w[1 + d]);
            K = K + w[1 + d] * w[1 + d];
        }
        Q[G.off + (D + 1) * N + i] = (T)(w[D + 1] * gi + (0.5 * w[0]) * K);
    }
}

// ----------------------------------------------------------------------------
// projection / prediction / ghost cells
// ----------------------------------------------------------------------------
// Projection of every cell of coarse grid gc from its finer grid (set-up).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_restrict_full(View v, T *A, int gc)
{
    const Grid G = v.grids[gc];
    const Grid F = v.grids[G.fine];
    const int n = G.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = D == 3 ? (int)(i / ((int64_t)n * n)) : 0;
#pragma unroll
        for (int f = 0; f < D + 2; ++f)
            A[G.off + f * G.ncell + i] = restrict_cell<T, D>(A + F.off + f * F.ncell, F.n, x, y, z);
    }
}

// Projection onto the covered cells of the blocks of level lvl's covered list.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_restrict_cov(View v, T *A, int lvl)
{
    // first reads, independent of each other (grid index = level)
    const int done = v.meta->done;
    const int off = v.meta->loff[LST_COV][lvl], count = v.meta->loff[LST_COV][lvl + 1] - off;
    const Grid G = v.grids[lvl];
    const Grid F = v.grids[lvl + 1];
    issued(off, count, G.n, G.off, G.ncell, F.n, F.off, F.ncell, F.boff, F.nb);
    if (done) return;
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS;
    const int nb = G.nb;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const Tile tl = v.cov[off + t];
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
        for (int c = threadIdx.x; c < TC; c += blockDim.x) {
            const int x = ox + c % BS, y = oy + (c / BS) % BS, z = oz + (D == 3 ? c / (BS * BS) : 0);
            // children read whether or not the cell is covered (they exist
            // on the dense finer grid); every load before the first store
            T val[D + 2];
#pragma unroll
            for (int f = 0; f < D + 2; ++f) val[f] = restrict_cell<T, D>(A + F.off + f * F.ncell, F.n, x, y, z);
            const bool cv = covered(v.act, F, x, y, z);
#pragma unroll
            for (int f = 0; f < D + 2; ++f) issued(val[f]);
            if (!cv) continue;
            const int64_t id = gidx(G.n, x, y, z);
#pragma unroll
            for (int f = 0; f < D + 2; ++f) A[G.off + f * G.ncell + id] = val[f];
        }
    }
}

// Projection of the covered cells of levels lvl .. lvl+nlev-1 (nlev = 1 or
// 2; level lvl+nlev final) in one launch (Sec. 2.1: a covered cell is
// the mean of its children), 2D; with ghosts set, in the same launch, the
// ghost fill of every level, with ndet the MR details (used when lvl = 0,
// projected last).  Every block of the projected levels is a work item;
// those whose code has the covered bit project their covered cells.  A cell
// is the mean of its four children, each of which is final or, on a level
// projected in the same pass, itself the mean of its own children (and so
// on, proj_field): the arithmetic of successive one-level projections, every
// read issued before any result is stored.
// ghost cell of a ghost block (a block outside every patch of its level):
// a cell within two cells of a patch.  Cells x-2 .. x+2 reach the lower
// neighbour block along an axis when x mod 8 < 2 and the upper one when
// x mod 8 > 5 (the boundary map is applied to blocks as to cells), so the
// test reads the block's neighbour mask only.
template <int D>
__device__ __forceinline__ bool ghost_cell(uint32_t gm, int x, int y, int z)
{
    const int c[3] = {x & 7, y & 7, z & 7};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = d < D && c[d] < 2 ? -1 : 0;
        hi[d] = d < D && c[d] > 5 ? 1 : 0;
    }
    bool hit = false;
    for (int dz = lo[2]; dz <= hi[2]; ++dz)
        for (int dy = lo[1]; dy <= hi[1]; ++dy)
            for (int dx = lo[0]; dx <= hi[0]; ++dx)
                hit |= ((gm >> ((dx + 1) + 3 * (dy + 1) + (D == 3 ? 9 * (dz + 1) : 0))) & 1u) != 0;
    return hit;
}

// Third-order prediction of child (cx, cy, cz) of the coarse cell at local
// position (px, py, pz) (1..4) of a staged 6^D region of one field (the
// coarse cells around a block's parents, boundary map already applied);
// the same separable x, y, z order as predict_child.
template <typename T, int D>
__device__ __forceinline__ T predict_child_lds(const T *S, int px, int py, int pz, int cx, int cy, int cz)
{
    constexpr int W = BS / 2 + 2;
    auto at = [&](int x, int y, int z) { return S[x + W * (y + W * z)]; };
    if (D == 2) {
        T r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] = pred1<T>(at(px - 1, py + j - 1, 0), at(px, py + j - 1, 0), at(px + 1, py + j - 1, 0), cx);
        return pred1<T>(r[0], r[1], r[2], cy);
    }
    T sz[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] = pred1<T>(at(px - 1, py + j - 1, pz + k - 1), at(px, py + j - 1, pz + k - 1),
                            at(px + 1, py + j - 1, pz + k - 1), cx);
        sz[k] = pred1<T>(r[0], r[1], r[2], cy);
    }
    return pred1<T>(sz[0], sz[1], sz[2], cz);
}

// Field f of level-k cell (x, y) of a 2D hierarchy when the DEPTH levels
// k .. k+DEPTH-1 are projected in the same pass and level k+DEPTH is final:
// a covered cell is the mean of its four children in pairwise order, each
// child taken the same way one level down (DEPTH 0: the stored value).  The
// arithmetic of successive one-level projections; every read is issued and
// the value selected.
template <typename T, int DEPTH>
__device__ __forceinline__ T proj_field(const View &v, const T *A, const GridTab &tab, int k, int x, int y, int f)
{
    const Grid G = grid_tab(tab, k);
    const T own = A[G.off + f * G.ncell + gidx(G.n, x, y, 0)];
    if constexpr (DEPTH == 0) {
        return own;
    } else {
        const bool cov = covered(v.act, grid_tab(tab, k + 1), x, y, 0);
        T c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            c[j] = proj_field<T, DEPTH - 1>(v, A, tab, k + 1, 2 * x + (j & 1), 2 * y + (j >> 1), f);
        const T m = T(0.25) * ((c[0] + c[1]) + (c[2] + c[3]));
        return cov ? m : own;
    }
}

// Value of level-k cell (x, y) of a 2D hierarchy after the projection of
// levels k .. hi-1 in one pass (hi - k = 1 or 2 levels below it), the first
// NV fields (all four, or the density alone).
template <typename T, int NV = 4>
__device__ __forceinline__ void projected_value(const View &v, const T *A, const GridTab &tab, int k, int hi,
                                                int x, int y, T *out)
{
    const int depth = hi - k;
    if (depth >= 2) {
#pragma unroll
        for (int f = 0; f < NV; ++f) out[f] = proj_field<T, 2>(v, A, tab, k, x, y, f);
    } else {
#pragma unroll
        for (int f = 0; f < NV; ++f) out[f] = proj_field<T, 1>(v, A, tab, k, x, y, f);
    }
}

// MR detail (Sec. 2.1) of cell (x, y) of an 8x8 block at (ox, oy) from its
// densities staged in LDS: S the 10x10 stencil region of the block's level
// (periodic or mirrored at the domain edge), C the 16x16 children.  The same
// FP64 expression as k_details.
template <typename T>
__device__ __forceinline__ double detail_lds(const T *S, const T *C, int lx, int ly)
{
#pragma clang fp contract(off)
    double s[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) s[j][i] = (double)S[(ly + j) * (BS + 2) + lx + i];
    double Dm = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int cx = c & 1, cy = c >> 1;
        const double rho = (double)C[(2 * ly + cy) * (2 * BS) + 2 * lx + cx];
        double r[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) r[j] = pred1<double>(s[j][0], s[j][1], s[j][2], cx);
        const double pr = pred1<double>(r[0], r[1], r[2], cy);
        const double dd = __builtin_fabs(rho - pr);
        if (dd > Dm) Dm = dd;
    }
    return Dm;
}

template <typename T>
__global__ void __launch_bounds__(64) k_restrict2(View v, T *A, int lvl, int nlev, int ghosts, int64_t ndet)
{
    constexpr int NV = 4;
    constexpr int W = BS / 2 + 2, NS = W * W;
    constexpr int SW = BS + 2, NSD = SW * SW, CW = 2 * BS;
    __shared__ GridTab tab;
    __shared__ T sA[NV][NS];
    __shared__ T sS[NSD], sC[CW * CW];
    // Work items: MR details, then every block of the projected levels lvl ..
    // hi-1 (walked directly: its code says whether it holds covered cells),
    // then the ghost list.  Level hi is final.  No item waits for the done
    // flag before its first reads: the flag is tested with them.
    const int done = v.meta->done;
    const int ngh = ghosts ? v.meta->nghost : 0;
    const int hi = lvl + nlev;
    grid_tab_load(v, tab);
    __syncthreads();
    int nbl[3];   // blocks of the projected levels (nlev <= 2: the last is zero)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int nb = i < nlev ? grid_tab(tab, lvl + i).nb : 0;
        nbl[i] = nb * nb;
    }
    const int ncov = nbl[0] + nbl[1] + nbl[2];
    // projection items: with two levels, each block of level lvl (two levels
    // deep, 21 reads a field) is four items, one per field
    const int nsplit = nlev == 2 ? 4 : 1;
    const int nproj = nsplit * nbl[0] + nbl[1] + nbl[2];
    // MR details of levels 0 .. L-2 (ndet cells in all, only with lvl = 0):
    // 8x8 blocks of the levels projected here, then chunks of 64 cells of
    // the finer levels, from the first cell after those levels
    const Grid Gt = grid_tab(tab, hi - 1);
    const int64_t dfirst = Gt.coff + Gt.ncell;
    const int nin = ndet ? ncov : 0;
    const int nch = ndet ? nin + (int)((ndet - dfirst + 63) / 64) : 0;
    const int nitem = nch + nproj + (ghosts ? v.nbt : 0);   // ghost entries: at most one per block
    // block r of the projected levels: its level and index within the level
    auto level_block = [&](int r, int &k, int &b) {
        const int i = (r >= nbl[0] ? 1 : 0) + (r >= nbl[0] + nbl[1] ? 1 : 0);
        k = lvl + i;
        b = r - (i >= 1 ? nbl[0] : 0) - (i >= 2 ? nbl[1] : 0);
    };
    for (int t = xcd_run(blockIdx.x, gridDim.x); t < nitem; t += gridDim.x) {
        if (t < nch) {
            const int r = t;
            if (r < nin) {
                // 8x8 block of a projected level: the projected densities of
                // its stencil region and of its children staged in LDS
                int k, b;
                level_block(r, k, b);
                const Grid G = grid_tab(tab, k), F = grid_tab(tab, k + 1);
                const bool fin = k + 1 < hi;   // children projected here too
                const int ox = (b % G.nb) * BS, oy = (b / G.nb) * BS;
                const int lx = threadIdx.x % BS, ly = threadIdx.x / BS;
                const bool act = block_active(v, v.act, G, ox, oy, 0);
                const bool cov = covered(v.act, F, ox + lx, oy + ly, 0);
                if (done) break;
                // every staging read in flight at once (64 threads)
                T vs[2], vc[4];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int i = threadIdx.x + 64 * u < NSD ? threadIdx.x + 64 * u : NSD - 1;
                    const int ax = bcmap(ox - 1 + i % SW, G.n, v.bc), ay = bcmap(oy - 1 + i / SW, G.n, v.bc);
                    projected_value<T, 1>(v, A, tab, k, hi, ax, ay, &vs[u]);
                }
                if (fin) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = threadIdx.x + 64 * u;
                        projected_value<T, 1>(v, A, tab, k + 1, hi, 2 * ox + i % CW, 2 * oy + i / CW, &vc[u]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = threadIdx.x + 64 * u;
                        vc[u] = A[F.off + gidx(F.n, 2 * ox + i % CW, 2 * oy + i / CW, 0)];
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (threadIdx.x + 64 * u < NSD) sS[threadIdx.x + 64 * u] = vs[u];
#pragma unroll
                for (int u = 0; u < 4; ++u) sC[threadIdx.x + 64 * u] = vc[u];
                __syncthreads();
                const double Dm = act && cov ? detail_lds<T>(sS, sC, lx, ly) : 0.0;
                const int64_t j = G.coff + gidx(G.n, ox + lx, oy + ly, 0);
                v.D[j] = Dm;
                v.sig[j] = Dm >= v.eps_lv[k] ? 1 : 0;
                __syncthreads();
                continue;
            }
            // one cell of a finer level per thread, its values final
            const int64_t j = dfirst + (int64_t)(r - nin) * 64 + threadIdx.x;
            if (j < ndet) {
                int k = 0;
                for (int q = 1; q < MAXLEV && q < v.L - 1; ++q) k += j >= v.gt[q].coff ? 1 : 0;
                const Grid G = grid_lane(v, k), F = grid_lane(v, k + 1);
                const int64_t i = j - G.coff;
                const int x = (int)(i % G.n), y = (int)(i / G.n);
                const bool act = block_active(v, v.act, G, x, y, 0);
                const bool cov = covered(v.act, F, x, y, 0);
                if (done) break;
                double Dm = 0.0;
                if (act && cov) {
#pragma clang fp contract(off)
                    for (int c = 0; c < 4; ++c) {
                        const int cx = c & 1, cy = c >> 1;
                        const double rho = (double)A[F.off + gidx(F.n, 2 * x + cx, 2 * y + cy, 0)];
                        const double pr = predict_child<double, 2, T>(A + G.off, G.n, v.bc, x, y, 0, cx, cy, 0);
                        const double dd = __builtin_fabs(rho - pr);
                        if (dd > Dm) Dm = dd;
                    }
                }
                v.D[j] = Dm;
                v.sig[j] = Dm >= v.eps_lv[k] ? 1 : 0;
            }
            continue;
        }
        if (t >= nch + nproj) {
            // ghost block of any level: predicted from the level below, whose
            // values are final or, for the levels projected in this pass,
            // projected here (the entry is read with the count)
            const int g = t - nch - nproj;
            const Tile tl = v.ghost[g];
            if (done || g >= ngh) break;   // so are the later items of this workgroup
            const int lv = tl.grid & ((1 << Tile::GRID_BITS) - 1);
            const uint32_t gm = (uint32_t)tl.grid >> Tile::GRID_BITS;
            const Grid G = grid_tab(tab, lv), Cg = grid_tab(tab, lv - 1);
            const bool otf = lv - 1 >= lvl && lv - 1 < hi;
            const int nb = G.nb;
            const int ox = (tl.block % nb) * BS, oy = ((tl.block / nb) % nb) * BS;
            const int qx0 = (ox >> 1) - 1, qy0 = (oy >> 1) - 1;
            for (int i = threadIdx.x; i < NS; i += blockDim.x) {
                const int ax = bcmap(qx0 + i % W, Cg.n, v.bc), ay = bcmap(qy0 + i / W, Cg.n, v.bc);
                T val[NV];
                if (otf) {
                    projected_value<T>(v, A, tab, lv - 1, hi, ax, ay, val);
                } else {
#pragma unroll
                    for (int f = 0; f < NV; ++f) val[f] = A[Cg.off + f * Cg.ncell + gidx(Cg.n, ax, ay, 0)];
                }
#pragma unroll
                for (int f = 0; f < NV; ++f) sA[f][i] = val[f];
            }
            __syncthreads();
            for (int c = threadIdx.x; c < BS * BS; c += blockDim.x) {
                const int x = ox + c % BS, y = oy + c / BS;
                if (!ghost_cell<2>(gm, x, y, 0)) continue;
                const int64_t id = gidx(G.n, x, y, 0);
#pragma unroll
                for (int f = 0; f < NV; ++f)
                    A[G.off + f * G.ncell + id] =
                        predict_child_lds<T, 2>(sA[f], (x >> 1) - qx0, (y >> 1) - qy0, 0, x & 1, y & 1, 0);
            }
            __syncthreads();
            continue;
        }
        // block of a projected level, when it holds covered cells: each
        // covered cell the mean of its children, projected through the
        // levels below it in this pass (a block two levels deep: one field)
        const int r = t - nch;
        const bool split = r < nsplit * nbl[0] && nsplit > 1;
        int k, block;
        level_block(split ? r / nsplit : r - (nsplit - 1) * nbl[0], k, block);
        const Grid G = grid_tab(tab, k);
        const int code = v.code[G.boff + block];
        if (done) break;
        if (!(code & 2)) continue;
        const int nb = G.nb;
        const int x = (block % nb) * BS + threadIdx.x % BS;
        const int y = ((block / nb) % nb) * BS + threadIdx.x / BS;
        const bool cov = covered(v.act, grid_tab(tab, k + 1), x, y, 0);
        const int64_t id = G.off + gidx(G.n, x, y, 0);
        if (split) {
            const int f = r % nsplit;
            const T val = proj_field<T, 2>(v, A, tab, k, x, y, f);
            if (cov) A[id + f * G.ncell] = val;
            continue;
        }
        T val[NV];
        projected_value<T>(v, A, tab, k, hi, x, y, val);
        if (!cov) continue;
#pragma unroll
        for (int f = 0; f < NV; ++f) A[id + f * G.ncell] = val[f];
    }
}

// Prediction from the next coarser level into array A:
//   mode 0: every cell of the blocks created at level lvl (new list);
//   mode 1: every ghost cell of every level (ghost list);
//   mode 2: the ghost cells of level lvl, from the coarse level's state
//           interpolated in time between Qo (theta = 0) and Q (theta = 1);
//   mode 3: mode 0, then the ghost cells of level lvl, in one launch (both
//           read level lvl-1 only, which is final by then); with nlev = 2
//           the same for levels lvl and lvl+1 in one launch: a level-(lvl+1)
//           block recomputes the new level-lvl cells its stencils read from
//           level lvl-1 (the same prediction, so the same bits) instead of
//           waiting for them.
// CFL speeds of the leaf cells of leaf blocks ta and (two) tb, their reads
// issued together; a new block of levels lvl .. lvl+nlev-1 counts nothing
// (its prediction counts its cells).
template <typename T, int D>
__device__ __forceinline__ void leaf_speeds(const View &v, const T *A, const GridTab &tab, const Tile &ta, int lvl,
                                            int nlev, double g, double (*lmax)[MAXLEV], unsigned long long *lcnt,
                                            bool &bad, bool two, const Tile &tb)
{
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS, NV = D + 2;
    constexpr int CPT = TC / (D == 2 ? 64 : 256);   // cells per thread (64 or 256 threads)
    double q[2][CPT][NV];
    bool leaf[2][CPT];
    int lv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const Tile &tl = k ? tb : ta;
        lv[k] = tl.grid;
        const Grid G = grid_tab(tab, tl.grid);
        const bool hasf = G.fine >= 0;
        const Grid GF = hasf ? grid_tab(tab, G.fine) : G;
        const bool mine = tl.grid >= lvl && tl.grid < lvl + nlev && (v.code[G.boff + tl.block] & 8) != 0;
        const int nb = G.nb;
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int c = threadIdx.x + i * (TC / CPT);
            const int x = ox + c % BS, y = oy + (c / BS) % BS, z = oz + (D == 3 ? c / (BS * BS) : 0);
            const int64_t id = G.off + gidx(G.n, x, y, z);
#pragma unroll
            for (int f = 0; f < NV; ++f) q[k][i][f] = (double)A[f * G.ncell + id];
            leaf[k][i] = !mine && !(hasf && covered(v.act, GF, x, y, z));
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && !two) break;
        double m = 0.0;
        int nl = 0;
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            bool b;
            const double S = cell_speed<D>(q[k][i], g, v.cfl_max, b);
            if (leaf[k][i] && b) bad = true;
            if (leaf[k][i] && S > m) m = S;
            nl += leaf[k][i] ? 1 : 0;
        }
        cfl_tile_done(lmax, lcnt, v, lv[k], m, nl);
    }
}

// Gl, Cl and Gh are the grids of levels lvl, lvl-1 and lvl+1 (modes 0, 2, 3),
// passed at fixed argument offsets.
// cfl (mode 3, the launch of the finest levels, A the state): the launch
// also leaves the CFL partials of the new hierarchy, as k_cfl would compute
// them from the state it leaves: the new blocks of its levels take the speeds
// of the leaf cells they predict, the leaf tiles every other leaf block.
// direct (mode 3 without cfl): the work items are the blocks of the levels
// themselves, each taken when its code marks it new or ghost (no list read
// at a device offset).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_predict(View v, T *A, int lvl, int mode, double theta, int nlev, Grid Gl,
                                                 Grid Cl, Grid Gh, int cfl, int direct)
{
    constexpr int W = BS / 2 + 2, NS = D == 2 ? W * W : W * W * W;
    constexpr int NW = D == 2 ? 1 : 4;   // waves per workgroup
    __shared__ GridTab tab;
    __shared__ T sA[D + 2][NS];
    __shared__ double lmax[NW][MAXLEV];
    __shared__ unsigned long long lcnt[NW];
    // first reads, independent of each other (grid index = level)
    const int done = v.meta->done;
    int off0 = 0, cnt0 = 0, off1 = 0, cnt1 = 0;   // ranges in the new and ghost lists
    if (!direct && (mode == 0 || mode == 3)) {
        off0 = v.meta->loff[LST_NEW][lvl];
        cnt0 = v.meta->loff[LST_NEW][lvl + nlev] - off0;
    }
    if (mode == 1) cnt1 = v.meta->nghost;
    if (!direct && mode >= 2) {
        off1 = v.meta->loff[LST_GHOST][lvl];
        cnt1 = v.meta->loff[LST_GHOST][lvl + nlev] - off1;
    }
    const int nleaf = cfl ? v.meta->nleaf : 0;
    const bool all = mode == 1;
    if (all || cfl) grid_tab_load(v, tab);
    if (!direct) {
        issued(off0, cnt0, off1, cnt1, nleaf);
        if (done) return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (cfl) {
        if (lane < MAXLEV) lmax[wave][lane] = 0.0;
        if (lane == 0) lcnt[wave] = 0ull;
    }
    if (all || cfl) __syncthreads();
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS;
    constexpr int NV = D + 2;
    const double g = v.gamma;
    bool bad = false;
    const int nb0 = D == 2 ? Gl.nb * Gl.nb : Gl.nb * Gl.nb * Gl.nb;
    const int nbh = nlev == 2 ? (D == 2 ? Gh.nb * Gh.nb : Gh.nb * Gh.nb * Gh.nb) : 0;
    const int count = direct ? nb0 + nbh : cnt0 + cnt1;
    const int bv = xcd_run(blockIdx.x, gridDim.x);   // this workgroup's virtual index
    for (int t = bv; t < count; t += gridDim.x) {
        bool fresh;
        Tile tl;
        if (direct) {
            // block t of level lvl, then of lvl+1: its code and neighbour
            // mask, read with the done flag
            const bool lo = t < nb0;
            const int b = lo ? t : t - nb0;
            const int64_t gb = (lo ? Gl.boff : Gh.boff) + b;
            const int code = v.code[gb];
            const uint32_t gmk = v.gmask[gb];
            if (done) break;
            if (!(code & 12)) continue;
            fresh = (code & 8) != 0;
            tl = Tile{(lo ? lvl : lvl + 1) | (fresh ? 0 : (int)(gmk << Tile::GRID_BITS)), b};
        } else {
            fresh = t < cnt0;
            tl = fresh ? v.fresh[off0 + t] : v.ghost[off1 + t - cnt0];
        }
        const int lv = fresh ? tl.grid : tl.grid & ((1 << Tile::GRID_BITS) - 1);
        const uint32_t gm = fresh ? 0u : (uint32_t)tl.grid >> Tile::GRID_BITS;
        const bool up = !all && lv != lvl;   // a level-(lvl+1) block of a two-level launch
        const Grid G = all ? grid_tab(tab, lv) : up ? Gh : Gl;
        const Grid Cg = all ? grid_tab(tab, G.coarse) : up ? Gl : Cl;
        const int nb = G.nb;
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
        // the coarse cells the block's predictions read (parents +-1 per
        // axis), staged once per block; with time interpolation the staged
        // value is the interpolated state
        const int qx0 = (ox >> 1) - 1, qy0 = (oy >> 1) - 1, qz0 = D == 3 ? (oz >> 1) - 1 : 0;
        for (int i = threadIdx.x; i < NS; i += blockDim.x) {
            const int sx = i % W, sy = (i / W) % W, sz = D == 3 ? i / (W * W) : 0;
            const int ax = bcmap(qx0 + sx, Cg.n, v.bc), ay = bcmap(qy0 + sy, Cg.n, v.bc);
            const int az = D == 3 ? bcmap(qz0 + sz, Cg.n, v.bc) : 0;
            const int64_t ic = Cg.off + gidx(Cg.n, ax, ay, az);
            if (up) {
                // a cell of a new block of level lvl is predicted here from
                // level lvl-1: both candidates read with the block's code, in
                // one round trip, and the value selected
                const int code = v.code[Cg.boff + gidx(Cg.nb, ax >> 3, ay >> 3, az >> 3)];
                T pv[NV], sv[NV];
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    pv[f] = predict_child<T, D, T>(A + Cl.off + f * Cl.ncell, Cl.n, v.bc, ax >> 1, ay >> 1, az >> 1,
                                                   ax & 1, ay & 1, az & 1);
                    sv[f] = A[ic + f * Cg.ncell];
                }
                const bool pre = (code & 8) != 0;
#pragma unroll
                for (int f = 0; f < NV; ++f) sA[f][i] = pre ? pv[f] : sv[f];
                continue;
            }
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                if (mode == 2) {
                    const T om = T(1) - (T)theta;
                    sA[f][i] = om * ((const T *)v.Qo)[ic + f * Cg.ncell] + (T)theta * ((const T *)v.Q)[ic + f * Cg.ncell];
                } else {
                    sA[f][i] = A[ic + f * Cg.ncell];
                }
            }
        }
        __syncthreads();
        const bool speeds = cfl && fresh;   // the leaf cells of a new block
        const bool hasf = lv + 1 < v.L;
        const Grid GF = speeds && hasf ? grid_tab(tab, lv + 1) : G;
        double m = 0.0;
        int nl = 0;
        for (int c = threadIdx.x; c < TC; c += blockDim.x) {
            const int x = ox + c % BS, y = oy + (c / BS) % BS, z = oz + (D == 3 ? c / (BS * BS) : 0);
            // every cell of a new block is predicted; in a ghost block only
            // the ghost cells
            if (!fresh && !ghost_cell<D>(gm, x, y, z)) continue;
            const bool leaf = speeds && !(hasf && covered(v.act, GF, x, y, z));
            const int px = (x >> 1) - qx0, py = (y >> 1) - qy0, pz = D == 3 ? (z >> 1) - qz0 : 0;
            const int64_t id = gidx(G.n, x, y, z);
            double q[NV];
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                const T val = predict_child_lds<T, D>(sA[f], px, py, pz, x & 1, y & 1, z & 1);
                A[G.off + f * G.ncell + id] = val;
                q[f] = (double)val;
            }
            if (speeds) {
                bool b;
                const double S = cell_speed<D>(q, g, v.cfl_max, b);
                if (leaf && b) bad = true;
                if (leaf && S > m) m = S;
                nl += leaf ? 1 : 0;
            }
        }
        if (speeds) cfl_tile_done(lmax, lcnt, v, lv, m, nl);
        __syncthreads();
    }
    if (cfl) {
        // the leaf blocks, on the workgroups without a prediction when there
        // are such, two blocks at a time
        const int G = gridDim.x, b = bv;
        const int nw = count < G ? G - count : G;
        const int w = count < G ? b - count : b;
        for (int u = w; w >= 0 && u < nleaf; u += 2 * nw) {
            const bool two = u + nw < nleaf;
            const Tile ta = v.leaf[u], tb = v.leaf[two ? u + nw : u];
            leaf_speeds<T, D>(v, A, tab, ta, lvl, nlev, g, lmax, lcnt, bad, two, tb);
        }
        if (__any(bad) && lane == 0) atomicOr(&v.meta->status, 1);
        __syncthreads();
        cfl_publish<NW>(lmax, lcnt, v);
    }
}

// Composite solution on level lvl, in the stage array (error assessment,
// Sec. 3): level 0 is copied; on a finer level a cell in a patch keeps its
// value and every other cell is predicted from the composite of the level
// below.  Called for lvl = 0, 1, .., L-1 in order.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_composite(View v, int lvl)
{
    const Grid G = v.grids[lvl];
    const T *Q = (const T *)v.Q;
    T *U = (T *)v.Qs;
    const int n = G.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = D == 3 ? (int)(i / ((int64_t)n * n)) : 0;
        const bool keep = lvl == 0 || block_active(v, v.act, G, x, y, z);
        if (keep) {
#pragma unroll
            for (int f = 0; f < D + 2; ++f) U[G.off + f * G.ncell + i] = Q[G.off + f * G.ncell + i];
        } else {
            const Grid Cg = v.grids[lvl - 1];
#pragma unroll
            for (int f = 0; f < D + 2; ++f)
                U[G.off + f * G.ncell + i] = predict_child<T, D, T>(U + Cg.off + f * Cg.ncell, Cg.n, v.bc, x >> 1,
                                                                    y >> 1, z >> 1, x & 1, y & 1, z & 1);
        }
    }
}

// Local time stepping: copy the cells of level lvl's patches from Q to Qo:
// the level's state at the start of its step, kept for the time
// interpolation of finer ghost cells (Q -> Qo), or the AMR scheme's new
// state from the stage array (Qs -> Q).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_copy_level(View v, int lvl, const T *__restrict__ Q, T *Qo)
{
    if (v.meta->done) return;
    const int off = v.meta->loff[LST_ACT][lvl], count = v.meta->loff[LST_ACT][lvl + 1] - off;
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const Tile tl = v.actv[off + t];
        const Grid G = v.grids[tl.grid];
        const int nb = G.nb;
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
        for (int c = threadIdx.x; c < TC; c += blockDim.x) {
            const int64_t id = G.off + gidx(G.n, ox + c % BS, oy + (c / BS) % BS, oz + (D == 3 ? c / (BS * BS) : 0));
#pragma unroll
            for (int f = 0; f < D + 2; ++f) Qo[f * G.ncell + id] = Q[f * G.ncell + id];
        }
    }
}

// Flux correction of level lvl after the two substeps of level lvl+1
// (Berger-Colella): at every face between a leaf and a covered cell,
// Q += s lam (F_c - Fbar), Fbar = (A_0 + A_1) / 2 with A_k the area mean of
// the fine fluxes of substep k; axes in order, low face first.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_reflux(View v, int lvl)
{
    if (v.meta->done) return;
    const int off = v.meta->loff[LST_LEAF][lvl], count = v.meta->loff[LST_LEAF][lvl + 1] - off;
    constexpr int TC = D == 2 ? BS * BS : BS * BS * BS;
    T *Q = (T *)v.Q;
    const T *reg = (const T *)v.reg;
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const Tile tl = v.leaf[off + t];
        const Grid G = v.grids[tl.grid];
        const Grid F = v.grids[G.fine];
        const int n = G.n, nb = G.nb, nf = F.n;
        const int ox = (tl.block % nb) * BS;
        const int oy = ((tl.block / nb) % nb) * BS;
        const int oz = D == 3 ? (tl.block / (nb * nb)) * BS : 0;
        const T lam = (T)(v.dt[lvl] / G.dx);
        for (int c = threadIdx.x; c < TC; c += blockDim.x) {
            const int p[3] = {ox + c % BS, oy + (c / BS) % BS, oz + (D == 3 ? c / (BS * BS) : 0)};
            if (covered(v.act, F, p[0], p[1], p[2])) continue;
            const int64_t ip = gidx(n, p[0], p[1], p[2]);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                for (int s = -1; s <= 1; s += 2) {
                    int nbc[3] = {p[0], p[1], p[2]};
                    nbc[d] = bcmap(p[d] + s, n, v.bc);
                    if (!covered(v.act, F, nbc[0], nbc[1], nbc[2])) continue;
                    const int64_t ic = s > 0 ? ip : gidx(n, nbc[0], nbc[1], nbc[2]);
                    int fb[3] = {2 * p[0], 2 * p[1], D == 3 ? 2 * p[2] : 0};
                    fb[d] = bcmap(s > 0 ? 2 * p[d] + 1 : 2 * p[d] - 1, nf, v.bc);
                    int c10[3] = {fb[0], fb[1], fb[2]}, c01[3] = {fb[0], fb[1], fb[2]}, c11[3] = {fb[0], fb[1], fb[2]};
                    c10[t1] += 1;
                    c01[t2] += 1;
                    c11[t1] += 1;
                    c11[t2] += 1;
                    for (int f = 0; f < D + 2; ++f) {
                        T A[2];
                        for (int k = 0; k < 2; ++k) {
                            const T *Rg = reg + F.rfoff + (((int64_t)k * D + d) * (D + 2) + f) * F.ncell;
                            if (D == 2)
                                A[k] = T(0.5) * (Rg[gidx(nf, fb[0], fb[1], 0)] + Rg[gidx(nf, c10[0], c10[1], 0)]);
                            else
                                A[k] = T(0.25) * ((Rg[gidx(nf, fb[0], fb[1], fb[2])] + Rg[gidx(nf, c10[0], c10[1], c10[2])]) +
                                                  (Rg[gidx(nf, c01[0], c01[1], c01[2])] + Rg[gidx(nf, c11[0], c11[1], c11[2])]));
                        }
                        const T Fbar = T(0.5) * (A[0] + A[1]);
                        const T Fc = reg[G.rcoff + ((int64_t)d * (D + 2) + f) * G.ncell + ic];
                        T &q = Q[G.off + f * G.ncell + ip];
                        if (s > 0) q = q + lam * (Fc - Fbar);
                        else q = q - lam * (Fc - Fbar);
                    }
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// MR details (FP64) of every refined cell of levels 0 .. L-2, one launch over
// the concatenated cells of those levels
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_details(View v, const T *__restrict__ Q, int64_t ntot)
{
#pragma clang fp contract(off)
    const int done = v.meta->done;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ntot;
         j += (int64_t)gridDim.x * blockDim.x) {
        int lvl = 0;
        for (int k = 1; k < MAXLEV && k < v.L - 1; ++k) lvl += j >= v.gt[k].coff ? 1 : 0;
        const Grid G = grid_lane(v, lvl);
        const Grid F = grid_lane(v, lvl + 1);
        const int n = G.n;
        const int64_t i = j - G.coff;
        const int x = (int)(i % n), y = (int)((i / n) % n), z = D == 3 ? (int)(i / ((int64_t)n * n)) : 0;
        double Dm = 0.0;
        const bool act = block_active(v, v.act, G, x, y, z);
        const bool cov = covered(v.act, F, x, y, z);
        issued((int)act, (int)cov);
        if (done) return;   // read with the masks above: one round trip for both
        if (act && cov) {
            const T *Ac = Q + G.off;  // density field of the coarse level
            const T *Af = Q + F.off;
            for (int k = 0; k < (1 << D); ++k) {
                const int cx = k & 1, cy = (k >> 1) & 1, cz = (k >> 2) & 1;
                const double rho = (double)Af[gidx(F.n, 2 * x + cx, 2 * y + cy, D == 3 ? 2 * z + cz : 0)];
                const double pr = predict_child<double, D, T>(Ac, n, v.bc, x, y, z, cx, cy, cz);
                const double dd = __builtin_fabs(rho - pr);
                if (dd > Dm) Dm = dd;
            }
        }
        v.D[j] = Dm;
        v.sig[j] = Dm >= v.eps_lv[lvl] ? 1 : 0;
    }
}

// ----------------------------------------------------------------------------
// the AMR method's refinement indicators (Sec. 2.2): scaled gradients of
// density and pressure, every cell of levels 0 .. L-2 in a patch of its
// level, one launch over the concatenated cells of those levels; ghost cells
// must be filled.  D receives the largest density difference.
// ----------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(256) k_gradient(View v, const T *__restrict__ Q, int64_t ntot)
{
#pragma clang fp contract(off)
    const int done = v.meta->done;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ntot;
         j += (int64_t)gridDim.x * blockDim.x) {
        int lvl = 0;
        for (int k = 1; k < MAXLEV && k < v.L - 1; ++k) lvl += j >= v.gt[k].coff ? 1 : 0;
        const Grid G = grid_lane(v, lvl);
        const int n = G.n;
        const int64_t i = j - G.coff;
        const int x = (int)(i % n), y = (int)((i / n) % n), z = D == 3 ? (int)(i / ((int64_t)n * n)) : 0;
        const bool act = block_active(v, v.act, G, x, y, z);
        issued((int)act);
        if (done) return;
        double dr = 0.0, dpm = 0.0;
        if (act) {
            const T *A = Q + G.off;
            double q[D + 2], w0[D + 2];
#pragma unroll
            for (int f = 0; f < D + 2; ++f) q[f] = (double)A[f * G.ncell + i];
            cons2prim<double, D>(q, w0, v.gamma);
            for (int a = 1; a < (1 << D); ++a) {
                const int64_t ja = gidx(n, bcmap(x + (a & 1), n, v.bc), bcmap(y + ((a >> 1) & 1), n, v.bc),
                                        D == 3 ? bcmap(z + ((a >> 2) & 1), n, v.bc) : 0);
                double qa[D + 2], wa[D + 2];
#pragma unroll
                for (int f = 0; f < D + 2; ++f) qa[f] = (double)A[f * G.ncell + ja];
                cons2prim<double, D>(qa, wa, v.gamma);
                const double er = __builtin_fabs(wa[0] - w0[0]), ep = __builtin_fabs(wa[D + 1] - w0[D + 1]);
                if (er > dr) dr = er;
                if (ep > dpm) dpm = ep;
            }
        }
        v.D[j] = dr;
        v.sig[j] = act && (dr > v.eps || (v.eps_p > 0.0 && dpm > v.eps_p)) ? 1 : 0;
    }
}

}  // namespace eu

#include "eu_strip.hpp"
#include "eu_strip3.hpp"
#include "eu_hancock.hpp"
