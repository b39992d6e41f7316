// eu_hancock.hpp -- the AMR scheme (Sec. 2: unsplit MUSCL-Hancock with the
// Minmod limiter in primitive variables, AUSMDV at the faces, one corrector
// stage) on the leaves of a 2D or 3D adaptive hierarchy (or uniform grid),
// with a global time step or in the recursive level cycle.
// A face between a leaf and a covered cell takes the mean of the finer
// level's fluxes along it, each from the finer level's own evolved face
// values (Sec. 2.2: the fine fluxes replace the coarse one, which keeps the
// update conservative across refinement boundaries).
#pragma once

namespace eu {

// Evolved face values of one cell from its primitive state w0 and its
// neighbours along x (xl, xr) and y (yl, yr): Minmod slopes, face values
// W -/+ slope/2, advanced half a step in conservative form with the exact
// flux, dQ = hl ((f_x(W^-_x) - f_x(W^+_x)) + (f_y(W^-_y) - f_y(W^+_y))),
// the same increment for all four.  Ev[0..3]: lower x, upper x, lower y,
// upper y face value (primitive).  The arithmetic of hancock_row.
template <typename T>
__device__ __forceinline__ void hancock_cell2(T g, T gi, T hl, const T *w0, const T *xl, const T *xr, const T *yl,
                                              const T *yr, T (*Ev)[4])
{
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const T sx = slope_minmod<T>(xl[f], w0[f], xr[f]);
        Ev[0][f] = w0[f] - T(0.5) * sx;
        Ev[1][f] = w0[f] + T(0.5) * sx;
        const T sy = slope_minmod<T>(yl[f], w0[f], yr[f]);
        Ev[2][f] = w0[f] - T(0.5) * sy;
        Ev[3][f] = w0[f] + T(0.5) * sy;
    }
    T fl[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) phys_flux2<T>(gi, k >> 1, Ev[k], fl[k]);
    T dQ[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) dQ[f] = hl * ((fl[0][f] - fl[1][f]) + (fl[2][f] - fl[3][f]));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T q[4];
        prim2cons2<T>(gi, Ev[k], q);
#pragma unroll
        for (int f = 0; f < 4; ++f) q[f] = q[f] + dQ[f];
        cons2prim<T, 2>(q, Ev[k], g);
    }
}

// Primitive state of cell (x, y) of grid gf (coordinates through the
// boundary map).
template <typename T>
__device__ __forceinline__ void prim_at2(const View &v, const Grid &gf, const T *S, int x, int y, T g, T *w)
{
    const int64_t id = gidx(gf.n, bcmap(x, gf.n, v.bc), bcmap(y, gf.n, v.bc), 0);
    T q[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) q[f] = S[f * gf.ncell + id];
    cons2prim<T, 2>(q, w, g);
}

// Evolved face value of cell (x, y) of grid gf on the upper (upper = 1) or
// lower side of axis dn.
template <typename T>
__device__ void hancock_face_at(const View &v, const Grid &gf, const T *S, int x, int y, int dn, int upper, T g,
                                T gi, T hl, T *w)
{
    T w0[4], xl[4], xr[4], yl[4], yr[4], Ev[4][4];
    prim_at2<T>(v, gf, S, x, y, g, w0);
    prim_at2<T>(v, gf, S, x - 1, y, g, xl);
    prim_at2<T>(v, gf, S, x + 1, y, g, xr);
    prim_at2<T>(v, gf, S, x, y - 1, g, yl);
    prim_at2<T>(v, gf, S, x, y + 1, g, yr);
    hancock_cell2<T>(g, gi, hl, w0, xl, xr, yl, yr, Ev);
#pragma unroll
    for (int f = 0; f < 4; ++f) w[f] = Ev[2 * dn + upper][f];
}

// Mean of the two fine AMR-scheme fluxes on the face between coarse cell
// (px, py) and its covered neighbour on side s of axis dn, from grid gf
// (the next finer level; hl its (dt / 2) / dx): the fine faces at transverse
// offsets 0 and 1, each AUSMDV of the evolved face values of the fine cells
// on either side.
template <typename T>
__device__ void fine_mean_hancock(const View &v, const Grid &gf, const T *src, int px, int py, int s, int dn, T g,
                                  T gi, T hl, T *F)
{
    const T *S = src + gf.off;
    const int along = dn == 0 ? px : py;
    const int bd = s > 0 ? 2 * along + 1 : 2 * along - 1;   // fine cell on the low side of the face
    T Fs[2][4];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int cx = dn == 0 ? bd : 2 * px + k;
        const int cy = dn == 0 ? 2 * py + k : bd;
        T wl[4], wr[4];
        hancock_face_at<T>(v, gf, S, cx, cy, dn, 1, g, gi, hl, wl);
        hancock_face_at<T>(v, gf, S, cx + (dn == 0 ? 1 : 0), cy + (dn == 1 ? 1 : 0), dn, 0, g, gi, hl, wr);
        ausmdv2<T>(g, gi, dn, wl, wr, Fs[k]);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) F[f] = T(0.5) * (Fs[0][f] + Fs[1][f]);
}

// One MUSCL-Hancock step, out = src - (dt / dx) ((dF_1 + dF_2)), into the
// other state array.  Global time step (lvl < 0): the leaf cells of every
// tile of the leaf list of a 2D hierarchy (or uniform grid); a face next to
// a covered cell takes the fine-flux mean.  Local time stepping (lvl >= 0):
// every cell of the patches of level lvl with the level's own fluxes and
// step dt_lvl; with record set, the fluxes across refinement boundaries go
// to the flux registers (substep sub), as k_fv_stage records them.  Per
// tile: the tile with a 2-cell halo converted to primitive variables in
// LDS; the evolved face values of cells -1 .. B of both axes; the fluxes of
// the faces the tile needs; the update.  fineproj (global step): a tile of
// the finest level also writes the projection of its new values onto its
// 4x4 parent cells (as k_fv_stage).  Past t_end a global step copies the
// whole state (nstate elements), so that the step leaves it as it was; a
// local step writes nothing.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_hancock_tile(View v, const T *__restrict__ src, T *out, int fineproj,
                                                     int64_t nstate, int lvl, int sub, int record)
{
    constexpr int B = BS, H = 2, E = BS + 4, NE = E * E, NV = 4;
    constexpr int HW = B + 2, NH = HW * HW;   // cells -1 .. B of both axes
    constexpr int NF = (B + 1) * B;           // faces per axis
    constexpr int TC = B * B, CPT = (TC + NT - 1) / NT;
    __shared__ T sW[NV][NE];
    __shared__ T sE[4][NV][NH];
    __shared__ T sF[2][NV][NF];
    __shared__ uint8_t sCov[NE];
    __shared__ uint8_t sAct[NE];
    __shared__ GridTab tab;
    const bool lts = lvl >= 0;
    const int done = v.meta->done;
    const Tile *list = lts ? v.actv + v.meta->loff[LST_ACT][lvl] : v.leaf;
    const int count = lts ? v.meta->loff[LST_ACT][lvl + 1] - v.meta->loff[LST_ACT][lvl] : v.meta->nleaf;
    const double dt = v.dt[lts ? lvl : 0];
    // workgroup b's first leaf tile read with the count (as k_fv_stage)
    const int tf = xcd_run(blockIdx.x, gridDim.x);
    const int t0 = tf < v.max_tiles ? tf : v.max_tiles - 1;
    const Tile first = lts ? Tile{0, 0} : v.leaf[t0];
    grid_tab_load(v, tab);
    issued(list, count, dt, first.grid, first.block);
    if (done) {
        if (!lts)
            for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nstate; i += (int64_t)gridDim.x * NT)
                out[i] = src[i];
        return;
    }
    __syncthreads();
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    for (int t = tf; t < count; t += gridDim.x) {
        const Tile tl = t == tf && !lts ? first : list[t];
        const Grid G = grid_tab(tab, tl.grid);
        const bool hasf = G.fine >= 0;
        const Grid GF = hasf ? grid_tab(tab, G.fine) : G;
        const int n = G.n, nb = G.nb;
        const int ox = (tl.block % nb) * B, oy = (tl.block / nb) * B;
        const T *S = src + G.off;
        const int64_t N = G.ncell;
        // the tile with its halo: every read of the thread's cells issued
        // before any is used
        constexpr int IE = (NE + NT - 1) / NT;
        T qh[IE][NV];
        uint8_t cvb[IE], acb[IE];
#pragma unroll
        for (int u = 0; u < IE; ++u) {
            const int c0 = threadIdx.x + u * NT, c = c0 < NE ? c0 : NE - 1;
            const int x = bcmap(ox + c % E - H, n, v.bc), y = bcmap(oy + c / E - H, n, v.bc);
            const int64_t id = gidx32(n, x, y, 0);
#pragma unroll
            for (int f = 0; f < NV; ++f) qh[u][f] = S[f * N + id];
            const int64_t cb = hasf ? GF.boff + (int64_t)gidx32(GF.nb, x >> 2, y >> 2, 0) : G.boff;
            cvb[u] = v.act[cb];
            acb[u] = record ? v.act[G.boff + (int64_t)gidx32(G.nb, x >> 3, y >> 3, 0)] : 0;
        }
        T qb[CPT][NV];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= TC) break;
            const int64_t id = gidx32(n, ox + c % B, oy + c / B, 0);
#pragma unroll
            for (int f = 0; f < NV; ++f) qb[k][f] = S[f * N + id];
        }
#pragma unroll
        for (int u = 0; u < IE; ++u) {
            const int c = threadIdx.x + u * NT;
            if (c >= NE) break;
            T w[NV];
            cons2prim<T, 2>(qh[u], w, g);
#pragma unroll
            for (int f = 0; f < NV; ++f) sW[f][c] = w[f];
            sCov[c] = hasf && cvb[u] != 0 ? 1 : 0;
            sAct[c] = acb[u] != 0 ? 1 : 0;
        }
        __syncthreads();
        // evolved face values of cells (-1 .. B)^2 (entry c: cell (c % HW - 1, c / HW - 1))
        const T hl = (T)((dt * 0.5) / G.dx);
        for (int c = threadIdx.x; c < NH; c += NT) {
            const int h = (c % HW + 1) + E * (c / HW + 1);
            T w0[NV], xl[NV], xr[NV], yl[NV], yr[NV], Ev[4][NV];
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                w0[f] = sW[f][h];
                xl[f] = sW[f][h - 1];
                xr[f] = sW[f][h + 1];
                yl[f] = sW[f][h - E];
                yr[f] = sW[f][h + E];
            }
            hancock_cell2<T>(g, gi, hl, w0, xl, xr, yl, yr, Ev);
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int f = 0; f < NV; ++f) sE[k][f][c] = Ev[k][f];
        }
        __syncthreads();
        // faces of both axes; face a (0 .. B) of a line lies between local
        // cells a-1 and a along the axis (x-fastest layout in both axes)
        const T hlf = hasf ? (T)((dt * 0.5) / GF.dx) : T(0);
        for (int j = threadIdx.x; j < 2 * NF; j += NT) {
            const int dn = j >= NF ? 1 : 0, fi = j - dn * NF;
            int a, lx, ly;
            if (dn == 0) {
                a = fi % (B + 1);
                lx = a - 1;
                ly = fi / (B + 1);
            } else {
                lx = fi % B;
                a = fi / B;
                ly = a - 1;
            }
            const int hl_ = (lx + H) + E * (ly + H), hr_ = hl_ + (dn == 0 ? 1 : E);
            const bool lin = a >= 1, rin = a <= B - 1;
            const bool lcov = sCov[hl_] != 0, rcov = sCov[hr_] != 0;
            // global step: faces next to a leaf of the tile; local step:
            // every face of the tile (whole patches are updated)
            const bool need = lts ? (lin || rin) : ((lin && !lcov) || (rin && !rcov));
            T F[NV];
            if (!need) {
#pragma unroll
                for (int f = 0; f < NV; ++f) F[f] = T(0);
            } else if (!lts && (lcov || rcov)) {
                int px = ox + lx, py = oy + ly, s = +1;
                if (lcov) {
                    s = -1;
                    px += dn == 0 ? 1 : 0;
                    py += dn == 1 ? 1 : 0;
                }
                fine_mean_hancock<T>(v, GF, src, px, py, s, dn, g, gi, hlf, F);
            } else {
                const int el = (lx + 1) + HW * (ly + 1), er = el + (dn == 0 ? 1 : HW);
                T wl[NV], wr[NV];
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    wl[f] = sE[2 * dn + 1][f][el];
                    wr[f] = sE[2 * dn][f][er];
                }
                ausmdv2<T>(g, gi, dn, wl, wr, F);
                if (record) {
                    // registers are indexed by the cell on the low side of the face
                    const int qx = dn == 0 ? bcmap(ox + lx, n, v.bc) : ox + lx;
                    const int qy = dn == 1 ? bcmap(oy + ly, n, v.bc) : oy + ly;
                    const int64_t iq = gidx(n, qx, qy, 0);
                    const bool lact = sAct[hl_] != 0, ract = sAct[hr_] != 0;
                    const bool lleaf = lact && !lcov, rleaf = ract && !rcov;
                    T *reg = (T *)v.reg;
                    if (G.rcoff >= 0 && ((lleaf && rcov) || (rleaf && lcov)))
#pragma unroll
                        for (int f = 0; f < NV; ++f) reg[G.rcoff + ((int64_t)dn * NV + f) * N + iq] = F[f];
                    if (G.rfoff >= 0 && lact != ract)
#pragma unroll
                        for (int f = 0; f < NV; ++f)
                            reg[G.rfoff + (((int64_t)sub * 2 + dn) * NV + f) * N + iq] = F[f];
                }
            }
#pragma unroll
            for (int f = 0; f < NV; ++f) sF[dn][f][fi] = F[f];
        }
        __syncthreads();
        const T lam = (T)(dt / G.dx);
        const bool fp = !lts && fineproj && tl.grid == v.L - 1;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= TC) break;
            const int x = c % B, y = c / B;
            if (!lts && sCov[(x + H) + E * (y + H)]) continue;
            const int fx = x + (B + 1) * y, fy = x + B * y;
            const int64_t id = G.off + (int64_t)gidx32(n, ox + x, oy + y, 0);
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                const T R = (sF[0][f][fx + 1] - sF[0][f][fx]) + (sF[1][f][fy + B] - sF[1][f][fy]);
                const T q = qb[k][f] - lam * R;
                out[f * N + id] = q;
                if (fp) sW[f][c] = q;   // the face phase no longer reads sW
            }
        }
        if (fp) {
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
// 3D: the same scheme with D-generic physics (the arithmetic of the oracle's
// dimension-generic routines; for D = 2 it equals the 2D functions above)
// ----------------------------------------------------------------------------

// Physical flux f_dn at a primitive state: (rho u, rho u v + p e_dn,
// u (rho e + p)), |v|^2 summed ((v1 v1 + v2 v2) + v3 v3).
template <typename T, int D>
__device__ __forceinline__ void phys_flux_d(T gi, int dn, const T *w, T *F)
{
    const T r = w[0], u = w[1 + dn], p = w[D + 1];
    T K = w[1] * w[1];
#pragma unroll
    for (int k = 1; k < D; ++k) K = K + w[1 + k] * w[1 + k];
    const T E = p * gi + (T(0.5) * r) * K;
    const T m = r * u;
    F[0] = m;
#pragma unroll
    for (int k = 0; k < D; ++k) F[1 + k] = k == dn ? m * w[1 + k] + p : m * w[1 + k];
    F[D + 1] = u * (E + p);
}

template <typename T, int D>
__device__ __forceinline__ void prim2cons_d(T gi, const T *w, T *q)
{
    const T r = w[0];
    q[0] = r;
    T K = w[1] * w[1];
#pragma unroll
    for (int k = 0; k < D; ++k) q[1 + k] = r * w[1 + k];
#pragma unroll
    for (int k = 1; k < D; ++k) K = K + w[1 + k] * w[1 + k];
    q[D + 1] = w[D + 1] * gi + (T(0.5) * r) * K;
}

// AUSMDV across a face with normal along axis dn (as ausmdv2, every
// tangential momentum upwinded with the mass flux).
template <typename T, int D>
__device__ __forceinline__ void ausmdv_d(T g, T gi, int dn, const T *wL, const T *wR, T *F)
{
    const T rL = wL[0], pL = wL[D + 1], uL = wL[1 + dn];
    const T rR = wR[0], pR = wR[D + 1], uR = wR[1 + dn];
    const T cL = Ar<T>::sqrt(Ar<T>::div(g * pL, rL));
    const T cR = Ar<T>::sqrt(Ar<T>::div(g * pR, rR));
    const T cm = cL >= cR ? cL : cR;
    const T sL = Ar<T>::div(pL, rL), sR = Ar<T>::div(pR, rR);
    const T aL = Ar<T>::div(T(2) * sL, sL + sR), aR = Ar<T>::div(T(2) * sR, sL + sR);
    const T upL = T(0.5) * (uL + Ar<T>::abs(uL)), umR = T(0.5) * (uR - Ar<T>::abs(uR));
    T Up, Um, Pp, Pm;
    if (Ar<T>::abs(uL) <= cm) {
        const T a = uL + cm, M = Ar<T>::div(uL, cm), b = M + T(1);
        Up = aL * (Ar<T>::div(a * a, T(4) * cm) - upL) + upL;
        Pp = pL * (((b * b) * (T(2) - M)) * T(0.25));
    } else {
        Up = upL;
        Pp = uL > T(0) ? pL : T(0);
    }
    if (Ar<T>::abs(uR) <= cm) {
        const T a = uR - cm, M = Ar<T>::div(uR, cm), b = M - T(1);
        Um = aR * (-Ar<T>::div(a * a, T(4) * cm) - umR) + umR;
        Pm = pR * (((b * b) * (T(2) + M)) * T(0.25));
    } else {
        Um = umR;
        Pm = uR < T(0) ? pR : T(0);
    }
    const T mh = Up * rL + Um * rR;
    const T am = Ar<T>::abs(mh);
    const T ph = Pp + Pm;
    const T dp = Ar<T>::abs(pR - pL), pmin = pL <= pR ? pL : pR;
    const T sw = Ar<T>::div(T(10) * dp, pmin);
    const T s = T(0.5) * (sw < T(1) ? sw : T(1));
    const T fV = Up * (rL * uL) + Um * (rR * uR);
    const T fD = T(0.5) * (mh * (uL + uR) - am * (uR - uL));
    T KL = wL[1] * wL[1], KR = wR[1] * wR[1];
#pragma unroll
    for (int k = 1; k < D; ++k) {
        KL = KL + wL[1 + k] * wL[1 + k];
        KR = KR + wR[1 + k] * wR[1 + k];
    }
    const T HL = Ar<T>::div((pL * gi + (T(0.5) * rL) * KL) + pL, rL);
    const T HR = Ar<T>::div((pR * gi + (T(0.5) * rR) * KR) + pR, rR);
    F[0] = mh;
#pragma unroll
    for (int k = 0; k < D; ++k)
        F[1 + k] = k == dn ? ((T(0.5) + s) * fV + (T(0.5) - s) * fD) + ph
                           : T(0.5) * (mh * (wL[1 + k] + wR[1 + k]) - am * (wR[1 + k] - wL[1 + k]));
    F[D + 1] = T(0.5) * (mh * (HL + HR) - am * (HR - HL));
}

// Half-step increment dQ = hl ((D_1 + D_2) + D_3), D_d = f_d(W - s_d/2) -
// f_d(W + s_d/2), of a cell with primitive state w0 and neighbours wn[d][0]
// (below along axis d) and wn[d][1] (above).
template <typename T>
__device__ __forceinline__ void hancock_dq3(T gi, T hl, const T *w0, const T (*wn)[2][5], T *dQ)
{
    T Dd[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T wm[5], wp[5], Fm[5], Fp[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const T sl = slope_minmod<T>(wn[d][0][f], w0[f], wn[d][1][f]);
            wm[f] = w0[f] - T(0.5) * sl;
            wp[f] = w0[f] + T(0.5) * sl;
        }
        phys_flux_d<T, 3>(gi, d, wm, Fm);
        phys_flux_d<T, 3>(gi, d, wp, Fp);
#pragma unroll
        for (int f = 0; f < 5; ++f) Dd[d][f] = Fm[f] - Fp[f];
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) dQ[f] = hl * ((Dd[0][f] + Dd[1][f]) + Dd[2][f]);
}

// Evolved face value W +/- s_dn/2 (upper / lower) advanced by dQ.
template <typename T>
__device__ __forceinline__ void hancock_evolve3(T g, T gi, const T *w0, const T *wm, const T *wp, const T *dQ,
                                                int upper, T *w)
{
    T e[5], q[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const T sl = slope_minmod<T>(wm[f], w0[f], wp[f]);
        e[f] = upper ? w0[f] + T(0.5) * sl : w0[f] - T(0.5) * sl;
    }
    prim2cons_d<T, 3>(gi, e, q);
#pragma unroll
    for (int f = 0; f < 5; ++f) q[f] = q[f] + dQ[f];
    cons2prim<T, 3>(q, w, g);
}

// Evolved face value of cell (x, y, z) of grid gf on side upper of axis dn,
// from its seven-cell stencil in HBM.
template <typename T>
__device__ void hancock_face_at3(const View &v, const Grid &gf, const T *S, int x, int y, int z, int dn, int upper,
                                 T g, T gi, T hl, T *w)
{
    const int nf = gf.n;
    auto prim = [&](int px, int py, int pz, T *out) {
        const int64_t id = gidx(nf, bcmap(px, nf, v.bc), bcmap(py, nf, v.bc), bcmap(pz, nf, v.bc));
        T q[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) q[f] = S[f * gf.ncell + id];
        cons2prim<T, 3>(q, out, g);
    };
    T w0[5], wn[3][2][5], dQ[5];
    prim(x, y, z, w0);
    prim(x - 1, y, z, wn[0][0]);
    prim(x + 1, y, z, wn[0][1]);
    prim(x, y - 1, z, wn[1][0]);
    prim(x, y + 1, z, wn[1][1]);
    prim(x, y, z - 1, wn[2][0]);
    prim(x, y, z + 1, wn[2][1]);
    hancock_dq3<T>(gi, hl, w0, wn, dQ);
    // the neighbours along dn, by selects (no indexing of the private
    // array by a run-time axis)
    T wm[5], wp[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        wm[f] = dn == 0 ? wn[0][0][f] : dn == 1 ? wn[1][0][f] : wn[2][0][f];
        wp[f] = dn == 0 ? wn[0][1][f] : dn == 1 ? wn[1][1][f] : wn[2][1][f];
    }
    hancock_evolve3<T>(g, gi, w0, wm, wp, dQ, upper, w);
}

// Mean of the four fine AMR-scheme fluxes on the face between coarse cell p
// and its covered neighbour on side s of axis dn (grid gf the next finer
// level): transverse offsets first along the lower transverse axis,
// ((F00 + F10) + (F01 + F11)) / 4.
template <typename T>
__device__ void fine_mean_hancock3(const View &v, const Grid &gf, const T *src, int px, int py, int pz, int s,
                                   int dn, T g, T gi, T hl, T *F)
{
    const T *S = src + gf.off;
    const int along = dn == 0 ? px : dn == 1 ? py : pz;
    const int bd = s > 0 ? 2 * along + 1 : 2 * along - 1;
    // one fine face at a time (register pressure): A = F00 + F10, C = F01 + F11
    T A[5], C[5];
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
        // offset k & 1 along the lower transverse axis, k >> 1 along the upper
        const int o1 = k & 1, o2 = k >> 1;
        const int cx = dn == 0 ? bd : 2 * px + o1;
        const int cy = dn == 1 ? bd : 2 * py + (dn == 0 ? o1 : o2);
        const int cz = dn == 2 ? bd : 2 * pz + o2;
        T wl[5], wr[5], Fk[5];
        hancock_face_at3<T>(v, gf, S, cx, cy, cz, dn, 1, g, gi, hl, wl);
        hancock_face_at3<T>(v, gf, S, cx + (dn == 0), cy + (dn == 1), cz + (dn == 2), dn, 0, g, gi, hl, wr);
        ausmdv_d<T, 3>(g, gi, dn, wl, wr, Fk);
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            if (k == 0) A[f] = Fk[f];
            else if (k == 1) A[f] = A[f] + Fk[f];
            else if (k == 2) C[f] = Fk[f];
            else C[f] = C[f] + Fk[f];
        }
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) F[f] = T(0.25) * (A[f] + C[f]);
}

// The 3D form of k_hancock_tile (global step over the leaf list, or local
// time stepping over the patches of level lvl): per 8^3 tile, the tile with
// a 2-cell halo as primitive variables in LDS, the half-step increments of
// the (-1 .. B)^3 cells around its faces, then axis by axis the face fluxes
// (each evolved face value from its cell's slope along the axis and the
// increment; the fine-flux mean next to a covered cell) and their
// differences, accumulated ((dF_1 + dF_2) + dF_3); the update.
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_hancock_tile3(View v, const T *__restrict__ src, T *out, int64_t nstate,
                                                      int lvl, int sub, int record)
{
    constexpr int B = BS, H = 2, E = BS + 4, NE = E * E * E, NV = 5;
    constexpr int HW = B + 2, NH = HW * HW * HW;
    constexpr int NF = (B + 1) * B * B;
    constexpr int TC = B * B * B, CPT = (TC + NT - 1) / NT;
    __shared__ T sW[NV][NE];
    __shared__ T sD[NV][NH];
    __shared__ T sF[NV][NF];
    __shared__ uint8_t sCov[NE];
    __shared__ uint8_t sAct[NE];
    const bool lts = lvl >= 0;
    const int done = v.meta->done;
    const Tile *list = lts ? v.actv + v.meta->loff[LST_ACT][lvl] : v.leaf;
    const int count = lts ? v.meta->loff[LST_ACT][lvl + 1] - v.meta->loff[LST_ACT][lvl] : v.meta->nleaf;
    const double dt = v.dt[lts ? lvl : 0];
    if (done) {
        if (!lts)
            for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < nstate; i += (int64_t)gridDim.x * NT)
                out[i] = src[i];
        return;
    }
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    XcdWalk walk(count);
    int t;
    while (walk.next(count, t)) {
        const Tile tl = list[t];
        const Grid G = v.grids[tl.grid];
        const bool hasf = G.fine >= 0;
        const Grid GF = hasf ? v.grids[G.fine] : G;
        const int n = G.n, nb = G.nb;
        const int ox = (tl.block % nb) * B, oy = ((tl.block / nb) % nb) * B, oz = (tl.block / (nb * nb)) * B;
        const T *S = src + G.off;
        const int64_t N = G.ncell;
        for (int c = threadIdx.x; c < NE; c += NT) {
            const int x = bcmap(ox + c % E - H, n, v.bc);
            const int y = bcmap(oy + (c / E) % E - H, n, v.bc);
            const int z = bcmap(oz + c / (E * E) - H, n, v.bc);
            const int64_t id = gidx32(n, x, y, z);
            T q[NV], w[NV];
#pragma unroll
            for (int f = 0; f < NV; ++f) q[f] = S[f * N + id];
            const bool cv = hasf && covered(v.act, GF, x, y, z);
            const bool ac = record && block_active(v, v.act, G, x, y, z);
            cons2prim<T, 3>(q, w, g);
#pragma unroll
            for (int f = 0; f < NV; ++f) sW[f][c] = w[f];
            sCov[c] = cv ? 1 : 0;
            sAct[c] = ac ? 1 : 0;
        }
        T qb[CPT][NV];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= TC) break;
            const int64_t id = gidx32(n, ox + c % B, oy + (c / B) % B, oz + c / (B * B));
#pragma unroll
            for (int f = 0; f < NV; ++f) qb[k][f] = S[f * N + id];
        }
        __syncthreads();
        // half-step increments of cells (-1 .. B)^3
        const T hl = (T)((dt * 0.5) / G.dx);
        for (int c = threadIdx.x; c < NH; c += NT) {
            const int h = (c % HW + 1) + E * ((c / HW) % HW + 1) + E * E * (c / (HW * HW) + 1);
            T w0[NV], wn[3][2][NV], dQ[NV];
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                w0[f] = sW[f][h];
                wn[0][0][f] = sW[f][h - 1];
                wn[0][1][f] = sW[f][h + 1];
                wn[1][0][f] = sW[f][h - E];
                wn[1][1][f] = sW[f][h + E];
                wn[2][0][f] = sW[f][h - E * E];
                wn[2][1][f] = sW[f][h + E * E];
            }
            hancock_dq3<T>(gi, hl, w0, wn, dQ);
#pragma unroll
            for (int f = 0; f < NV; ++f) sD[f][c] = dQ[f];
        }
        __syncthreads();
        const T hlf = hasf ? (T)((dt * 0.5) / GF.dx) : T(0);
        T R[CPT][NV];
        // one axis at a time, not unrolled (register pressure)
#pragma unroll 1
        for (int dn = 0; dn < 3; ++dn) {
            const int SD = dn == 0 ? 1 : dn == 1 ? E : E * E;
            const int SB = dn == 0 ? 1 : dn == 1 ? HW : HW * HW;
            for (int fi = threadIdx.x; fi < NF; fi += NT) {
                int a, lx, ly, lz;
                face_coords<3, B>(dn, fi, a, lx, ly, lz);
                const int hl_ = (lx + H) + E * ((ly + H) + E * (lz + H)), hr_ = hl_ + SD;
                const bool lin = a >= 1, rin = a <= B - 1;
                const bool lcov = sCov[hl_] != 0, rcov = sCov[hr_] != 0;
                const bool need = lts ? (lin || rin) : ((lin && !lcov) || (rin && !rcov));
                T F[NV];
                if (!need) {
#pragma unroll
                    for (int f = 0; f < NV; ++f) F[f] = T(0);
                } else if (!lts && (lcov || rcov)) {
                    int px = ox + lx, py = oy + ly, pz = oz + lz, s = +1;
                    if (lcov) {
                        s = -1;
                        px += dn == 0 ? 1 : 0;
                        py += dn == 1 ? 1 : 0;
                        pz += dn == 2 ? 1 : 0;
                    }
                    fine_mean_hancock3<T>(v, GF, src, px, py, pz, s, dn, g, gi, hlf, F);
                } else {
                    const int el = (lx + 1) + HW * ((ly + 1) + HW * (lz + 1)), er = el + SB;
                    T w0[NV], wm[NV], wp[NV], dQ[NV], wl[NV], wr[NV];
#pragma unroll
                    for (int f = 0; f < NV; ++f) {
                        w0[f] = sW[f][hl_];
                        wm[f] = sW[f][hl_ - SD];
                        wp[f] = sW[f][hl_ + SD];
                        dQ[f] = sD[f][el];
                    }
                    hancock_evolve3<T>(g, gi, w0, wm, wp, dQ, 1, wl);
#pragma unroll
                    for (int f = 0; f < NV; ++f) {
                        w0[f] = sW[f][hr_];
                        wm[f] = sW[f][hr_ - SD];
                        wp[f] = sW[f][hr_ + SD];
                        dQ[f] = sD[f][er];
                    }
                    hancock_evolve3<T>(g, gi, w0, wm, wp, dQ, 0, wr);
                    ausmdv_d<T, 3>(g, gi, dn, wl, wr, F);
                    if (record) {
                        int qx = ox + lx, qy = oy + ly, qz = oz + lz;
                        if (dn == 0) qx = bcmap(qx, n, v.bc);
                        else if (dn == 1) qy = bcmap(qy, n, v.bc);
                        else qz = bcmap(qz, n, v.bc);
                        const int64_t iq = gidx(n, qx, qy, qz);
                        const bool lact = sAct[hl_] != 0, ract = sAct[hr_] != 0;
                        const bool lleaf = lact && !lcov, rleaf = ract && !rcov;
                        T *reg = (T *)v.reg;
                        if (G.rcoff >= 0 && ((lleaf && rcov) || (rleaf && lcov)))
#pragma unroll
                            for (int f = 0; f < NV; ++f) reg[G.rcoff + ((int64_t)dn * NV + f) * N + iq] = F[f];
                        if (G.rfoff >= 0 && lact != ract)
#pragma unroll
                            for (int f = 0; f < NV; ++f)
                                reg[G.rfoff + (((int64_t)sub * 3 + dn) * NV + f) * N + iq] = F[f];
                    }
                }
#pragma unroll
                for (int f = 0; f < NV; ++f) sF[f][fi] = F[f];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int c = threadIdx.x + k * NT;
                if (c >= TC) break;
                const int x = c % B, y = (c / B) % B, z = c / (B * B);
                const int lo = dn == 0 ? x + (B + 1) * (y + B * z) : dn == 1 ? x + B * (y + (B + 1) * z)
                                                                              : x + B * (y + B * z);
                const int hi = lo + (dn == 0 ? 1 : dn == 1 ? B : B * B);
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    const T d = sF[f][hi] - sF[f][lo];
                    R[k][f] = dn == 0 ? d : R[k][f] + d;
                }
            }
            __syncthreads();
        }
        const T lam = (T)(dt / G.dx);
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c >= TC) break;
            const int x = c % B, y = (c / B) % B, z = c / (B * B);
            if (!lts && sCov[(x + H) + E * ((y + H) + E * (z + H))]) continue;
            const int64_t id = G.off + (int64_t)gidx32(n, ox + x, oy + y, oz + z);
#pragma unroll
            for (int f = 0; f < NV; ++f) out[f * N + id] = qb[k][f] - lam * R[k][f];
        }
        __syncthreads();
    }
}

}  // namespace eu
