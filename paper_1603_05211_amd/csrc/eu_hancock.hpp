// eu_hancock.hpp -- the AMR scheme (Sec. 2: unsplit MUSCL-Hancock with the
// Minmod limiter in primitive variables, AUSMDV at the faces, one corrector
// stage) on the leaves of a 2D adaptive hierarchy with a global time step.
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

}  // namespace eu
