// eu_strip.hpp -- finite-volume update of uniform 2D grids and batches of
// them (one level, no refinement boundaries), one wave per strip.
//
// A strip is 64 consecutive columns of one grid (lane l holds column
// xb + l) and a run of rows.  The wave marches up the rows: each new row is
// converted to primitive variables once; the y slopes, the face states and
// the flux of the face below the row before are computed from a window of
// three rows held in registers, and the x slopes and fluxes of a row from
// the neighbouring lanes (DPP wave shifts).  Every lane does the whole work
// of its column, so no pass of the wave runs with idle lanes; the two (one
// stage) or four (both stages fused) lanes at each end only provide the
// halo.  The arithmetic is the stage kernel's expression tree operation for
// operation (slope, face states, AUSM+, ((dF_1 + dF_2)), q - lam R), so FP64
// results are identical to it bit for bit.
//
// Fused form (both stages of the midpoint rule in one pass): the stage-1
// state of each row is produced two rows ahead of the stage-2 pipeline that
// consumes it and never leaves registers; its ghost cells are the clamped
// cells' stage values (outflow boundaries), taken from their lanes.  It
// reads Q^n and writes Q^{n+1} to the other state array.
//
// CFL partials of the new state: with cfl set, the launch that writes the
// step's new state also takes, in FP64 from the values it writes, the
// largest signal speed of its cells (the CFL reduction's: the sum or the
// largest over axes of |v_d| + c) and adds it into the grid's maximum (a batch)
// or a CFL slot with the count of cells advanced (a uniform grid), and
// raises the non-physical status flag; cfl = 2 computes them without
// publishing (timing passes).
#pragma once

namespace eu {

// Lane exchange within the wave: the value of lane i-1 (lane_from_left) or
// lane i+1 (lane_from_right); the end lanes receive 0.
__device__ __forceinline__ int dpp_shr1(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_shl1(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float lane_from_left(float x)
{
    return __builtin_bit_cast(float, dpp_shr1(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ float lane_from_right(float x)
{
    return __builtin_bit_cast(float, dpp_shl1(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double lane_from_left(double x)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)dpp_shr1((int)(unsigned)u), hi = (unsigned)dpp_shr1((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double lane_from_right(double x)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)dpp_shl1((int)(unsigned)u), hi = (unsigned)dpp_shl1((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// One stage's pipeline along y for the wave's columns.  Rows enter in
// order; after four rows, each new row r gives the residual of row r-2.
template <typename T>
struct YPipe {
    T wa[4], wb[4];   // primitive states of the two rows before the entering one
    T sp[4];          // upper face state of row wa's row (after three rows)
    T fl[4];          // flux through the lower face of wa's row (after four rows)
    int k = 0;        // rows entered
};

// x residual dF_1 of a row of primitive states w (lane = column).
template <typename T>
__device__ __forceinline__ void strip_rx(T g, T gi, const T *w, T *R)
{
    T xm[4], xp[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const T l = lane_from_left(w[f]), r = lane_from_right(w[f]);
        const T sl = slope_va<T>(l, w[f], r);
        xm[f] = w[f] - T(0.5) * sl;
        xp[f] = w[f] + T(0.5) * sl;
    }
    T rm[4], F[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) rm[f] = lane_from_right(xm[f]);
    ausm_plus<T, 2>(g, gi, 0, xp, rm, F);   // face i+1/2
#pragma unroll
    for (int f = 0; f < 4; ++f) R[f] = F[f] - lane_from_left(F[f]);
}

// Enter the primitive states wc of the next row.  Returns true when R holds
// the residual ((dF_1 + dF_2)) of the row two before wc's.
template <typename T>
__device__ __forceinline__ bool pipe_enter(YPipe<T> &P, T g, T gi, const T *wc, T *R)
{
    if (P.k < 2) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            P.wa[f] = P.wb[f];
            P.wb[f] = wc[f];
        }
        ++P.k;
        return false;
    }
    // y slope of row wb: its lower and upper face states
    T sm[4], sp[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const T sl = slope_va<T>(P.wa[f], P.wb[f], wc[f]);
        sm[f] = P.wb[f] - T(0.5) * sl;
        sp[f] = P.wb[f] + T(0.5) * sl;
    }
    bool out = false;
    if (P.k >= 3) {
        // face between rows wa and wb: the upper face of wa's row
        T F[4];
        ausm_plus<T, 2>(g, gi, 1, P.sp, sm, F);
        if (P.k >= 4) {
            T Rx[4];
            strip_rx<T>(g, gi, P.wa, Rx);
#pragma unroll
            for (int f = 0; f < 4; ++f) R[f] = Rx[f] + (F[f] - P.fl[f]);
            out = true;
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) P.fl[f] = F[f];
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        P.sp[f] = sp[f];
        P.wa[f] = P.wb[f];
        P.wb[f] = wc[f];
    }
    ++P.k;
    return out;
}

// Conserved state of the wave's columns on row y of a grid (clamped or
// wrapped column xc), and its primitive states.
template <typename T>
__device__ __forceinline__ void strip_load(const T *S, int64_t N, int n, int xc, int y, T *q)
{
    const uint32_t id = (uint32_t)xc + (uint32_t)n * (uint32_t)y;
#pragma unroll
    for (int f = 0; f < 4; ++f) q[f] = S[f * N + id];
}

// Signal speed of a written cell into the lane's running maximum (FP64
// from the stored values, the CFL reduction's expression).
template <typename T, int D = 2>
__device__ __forceinline__ void strip_speed(const T *q, double g, int mx, double &m, bool &bad)
{
    double qd[D + 2];
#pragma unroll
    for (int f = 0; f < D + 2; ++f) qd[f] = (double)q[f];
    bool b;
    const double S = cell_speed<D>(qd, g, mx, b);
    bad = bad || b;
    m = S > m ? S : m;
}

// The wave's maximum speed and cell count into the grid's CFL partials.
__device__ __forceinline__ void strip_publish(const View &v, int grid, double m, bool bad, int ncell, int wave)
{
    for (int o = 32; o > 0; o >>= 1) {
        const double r = __shfl_xor(m, o);
        m = r > m ? r : m;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&v.meta->status, 1);
    if ((threadIdx.x & 63) != 0) return;
    const unsigned long long b = (unsigned long long)__double_as_longlong(m);
    if (v.mode == MODE_BATCH) {
        if (m > 0.0) atomicMax(&v.smax[grid], b);
    } else {
        const int slot = wave % CFL_NSLOT;
        if (m > 0.0) atomicMax(v.cfls + cfl_slot(0, slot), b);
        atomicAdd(v.cfls + cfl_slot(MAXLEV, slot), (unsigned long long)ncell);
    }
}

// One stage (FUSED = 0; stage 1: src = Q, base = Q, out = Q*, own_base
// set: the base rows are the source rows already loaded; stage 2: src = Q*,
// base = Q, out = Q) or both stages (FUSED = 1: src = base = Q^n, out = the
// other state array) over the strips of the list.  Four waves per
// workgroup, each on its own strips; groups of four consecutive strips are
// walked XCD by XCD.
template <typename T, int FUSED>
__global__ void __launch_bounds__(256) k_fv_strip(View v, const Strip *__restrict__ list, int count,
                                                  const T *__restrict__ src, const T *base, T *out, double fac,
                                                  int own_base, int cfl)
{
    const int done = v.meta->done;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    constexpr int H = FUSED ? 4 : 2;   // halo lanes at each end
    const int ngroups = (count + 3) / 4;
    XcdWalk walk(ngroups);
    int t;
    while (walk.next(ngroups, t)) {
        const int si = 4 * t + wid;
        if (si >= count) continue;
        const Strip st = list[si];
        const Grid G = v.grids[st.grid];
        const int n = G.n;
        const int64_t N = G.ncell;
        const int x = st.xb + lane;
        const int xc = bcmap(x, n, v.bc);
        const bool wr = lane >= H && lane < 64 - H && x < n;   // this lane writes
        const double dt = v.mode == MODE_BATCH ? v.dt[st.grid] : v.dt[0];
        const T *S = src + G.off;
        const T *B = base + G.off;
        T *O = out + G.off;
        double smax = 0.0;   // CFL: largest speed of the lane's written cells
        bool bad = false;
        if (done) {
            // a step past t_end: the fused form still leaves the state in
            // the array it writes
            if (FUSED && wr)
                for (int y = st.y0; y < st.y0 + st.ny; ++y) {
                    T q[4];
                    strip_load<T>(S, N, n, xc, y, q);
#pragma unroll
                    for (int f = 0; f < 4; ++f) O[f * N + (uint32_t)x + (uint32_t)n * (uint32_t)y] = q[f];
                }
            continue;
        }
        if constexpr (!FUSED) {
            const T lam = (T)((dt * fac) / G.dx);
            YPipe<T> P;
            T qa[4], qb[4];   // conserved states of the rows of P.wa, P.wb (stage 1: the base)
            for (int k = 0; k < st.ny + 4; ++k) {
                const int r = st.y0 - 2 + k;
                T q[4], w[4], R[4];
                strip_load<T>(S, N, n, xc, bcmap(r, n, v.bc), q);
                T qo[4];
                const int ro = r - 2;   // the row this entry completes
                if (!own_base && k >= 4) strip_load<T>(B, N, n, xc, ro, qo);
                cons2prim<T, 2>(q, w, g);
                const bool res = pipe_enter<T>(P, g, gi, w, R);
                if (res) {
                    if (own_base)
#pragma unroll
                        for (int f = 0; f < 4; ++f) qo[f] = qa[f];
                    if (wr) {
                        T qn[4];
#pragma unroll
                        for (int f = 0; f < 4; ++f) {
                            qn[f] = qo[f] - lam * R[f];
                            O[f * N + (uint32_t)x + (uint32_t)n * (uint32_t)ro] = qn[f];
                        }
                        if (cfl) strip_speed<T>(qn, v.gamma, v.cfl_max, smax, bad);
                    }
                }
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    qa[f] = qb[f];
                    qb[f] = q[f];
                }
            }
        } else {
            // stage 1 (Q^n -> Q*) on rows ra .. rb, stage 2 on the strip's
            // rows; ghost rows and columns of Q* are the clamped cells'
            const T lam1 = (T)((dt * 0.5) / G.dx), lam2 = (T)(dt / G.dx);
            const int ra = st.y0 - 2 < 0 ? 0 : st.y0 - 2;
            const int rb = st.y0 + st.ny + 1 > n - 1 ? n - 1 : st.y0 + st.ny + 1;
            const bool edge = st.xb < 0 || st.xb + 63 >= n;   // some lanes are ghost columns
            const int srcl = xc - st.xb;                      // lane of the clamped column
            YPipe<T> P1, P2;
            T qa[4], qb[4];
            int ro2 = st.y0 - 5;   // incremented per stage-2 row entered: the row its residual belongs to
            for (int j = ra - 2; j <= rb + 2; ++j) {
                T q[4], w[4], R[4];
                strip_load<T>(S, N, n, xc, bcmap(j, n, v.bc), q);
                cons2prim<T, 2>(q, w, g);
                const bool res = pipe_enter<T>(P1, g, gi, w, R);
                if (res) {
                    // stage-1 state of row j - 2
                    T qs[4], ws[4];
#pragma unroll
                    for (int f = 0; f < 4; ++f) qs[f] = qa[f] - lam1 * R[f];
                    if (edge)
#pragma unroll
                        for (int f = 0; f < 4; ++f) qs[f] = __shfl(qs[f], srcl, 64);
                    cons2prim<T, 2>(qs, ws, g);
                    const int rs = j - 2;
                    int times = 1;
                    if (rs == ra) times += ra - (st.y0 - 2);
                    if (rs == rb) times += (st.y0 + st.ny + 1) - rb;
                    for (int m = 0; m < times; ++m) {
                        T R2[4];
                        const bool res2 = pipe_enter<T>(P2, g, gi, ws, R2);
                        ++ro2;
                        if (res2 && wr) {
                            T qo[4], qn[4];
                            strip_load<T>(B, N, n, xc, ro2, qo);
#pragma unroll
                            for (int f = 0; f < 4; ++f) {
                                qn[f] = qo[f] - lam2 * R2[f];
                                O[f * N + (uint32_t)x + (uint32_t)n * (uint32_t)ro2] = qn[f];
                            }
                            if (cfl) strip_speed<T>(qn, v.gamma, v.cfl_max, smax, bad);
                        }
                    }
                }
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    qa[f] = qb[f];
                    qb[f] = q[f];
                }
            }
        }
        if (cfl) {
            const int w = 64 - 2 * H;
            const int nx = n - (st.xb + H) < w ? n - (st.xb + H) : w;   // columns written
            const double m = cfl == 1 ? smax : -smax;   // cfl == 2: computed, not published
            if (cfl == 1) strip_publish(v, st.grid, m, bad, nx * st.ny, 4 * t + wid);
            else if (m > 1e300) atomicOr(&v.meta->status, 0);
        }
    }
}

// ----------------------------------------------------------------------------
// the AMR scheme (Sec. 2): unsplit MUSCL-Hancock, Minmod, AUSMDV
// ----------------------------------------------------------------------------

// Minmod limited slope: the difference of smaller magnitude when the
// backward and forward differences have the same sign, else 0.
template <typename T>
__device__ __forceinline__ T slope_minmod(T wm, T w0, T wp)
{
    const T a = w0 - wm, b = wp - w0;
    const T m = Ar<T>::abs(a) <= Ar<T>::abs(b) ? a : b;
    return a * b > T(0) ? m : T(0);
}

// Physical flux f_dn at a primitive state (2D).
template <typename T>
__device__ __forceinline__ void phys_flux2(T gi, int dn, const T *w, T *F)
{
    const T r = w[0], u = dn == 0 ? w[1] : w[2], p = w[3];
    const T K = w[1] * w[1] + w[2] * w[2];
    const T E = p * gi + (T(0.5) * r) * K;
    const T m = r * u;
    F[0] = m;
    F[1] = dn == 0 ? m * w[1] + p : m * w[1];
    F[2] = dn == 1 ? m * w[2] + p : m * w[2];
    F[3] = u * (E + p);
}

// primitive -> conserved (2D): rho e = p / (gamma - 1) + rho |v|^2 / 2
template <typename T>
__device__ __forceinline__ void prim2cons2(T gi, const T *w, T *q)
{
    const T r = w[0];
    q[0] = r;
    q[1] = r * w[1];
    q[2] = r * w[2];
    const T K = w[1] * w[1] + w[2] * w[2];
    q[3] = w[3] * gi + (T(0.5) * r) * K;
}

// AUSMDV (Wada and Liou 1997) across a face with normal along axis dn (2D):
// c_m = max(c_L, c_R), pressure-ratio weights, third-order pressure
// polynomials, AUSMV/AUSMD momentum blend with s = min(1, 10 |dp| / min p)/2,
// upwinded tangential momentum and total enthalpy; no entropy or shock fix.
template <typename T>
__device__ __forceinline__ void ausmdv2(T g, T gi, int dn, const T *wL, const T *wR, T *F)
{
    const T rL = wL[0], pL = wL[3], uL = dn == 0 ? wL[1] : wL[2], vL = dn == 0 ? wL[2] : wL[1];
    const T rR = wR[0], pR = wR[3], uR = dn == 0 ? wR[1] : wR[2], vR = dn == 0 ? wR[2] : wR[1];
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
    const T KL = wL[1] * wL[1] + wL[2] * wL[2], KR = wR[1] * wR[1] + wR[2] * wR[2];
    const T HL = Ar<T>::div((pL * gi + (T(0.5) * rL) * KL) + pL, rL);
    const T HR = Ar<T>::div((pR * gi + (T(0.5) * rR) * KR) + pR, rR);
    const T fn = ((T(0.5) + s) * fV + (T(0.5) - s) * fD) + ph;
    const T ft = T(0.5) * (mh * (vL + vR) - am * (vR - vL));
    F[0] = mh;
    F[1] = dn == 0 ? fn : ft;
    F[2] = dn == 0 ? ft : fn;
    F[3] = T(0.5) * (mh * (HL + HR) - am * (HR - HL));
}

// Evolved face values of a row of cells (lane = column) with primitive
// states wb, the rows below / above wa / wc: Minmod slopes along x (lanes)
// and y, face values W -/+ slope/2 advanced half a step with the exact
// flux, dQ = hl ((f_x(W^-_x) - f_x(W^+_x)) + (f_y(W^-_y) - f_y(W^+_y))).
// Outputs (primitive): xm, xp (lower / upper x face), ym, yp.
template <typename T>
__device__ __forceinline__ void hancock_row(T gi, T g, T hl, const T *wa, const T *wb, const T *wc, T *xm, T *xp,
                                            T *ym, T *yp)
{
    T fxm[4], fxp[4], fym[4], fyp[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const T sx = slope_minmod<T>(lane_from_left(wb[f]), wb[f], lane_from_right(wb[f]));
        xm[f] = wb[f] - T(0.5) * sx;
        xp[f] = wb[f] + T(0.5) * sx;
        const T sy = slope_minmod<T>(wa[f], wb[f], wc[f]);
        ym[f] = wb[f] - T(0.5) * sy;
        yp[f] = wb[f] + T(0.5) * sy;
    }
    phys_flux2<T>(gi, 0, xm, fxm);
    phys_flux2<T>(gi, 0, xp, fxp);
    phys_flux2<T>(gi, 1, ym, fym);
    phys_flux2<T>(gi, 1, yp, fyp);
    T dQ[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) dQ[f] = hl * ((fxm[f] - fxp[f]) + (fym[f] - fyp[f]));
    T *st[4] = {xm, xp, ym, yp};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        T q[4];
        prim2cons2<T>(gi, st[k], q);
#pragma unroll
        for (int f = 0; f < 4; ++f) q[f] = q[f] + dQ[f];
        cons2prim<T, 2>(q, st[k], g);
    }
}

// The Hancock pipeline along y: rows enter in order; row r completes the
// evolved face values of row r-1, the face between rows r-2 and r-1, the
// x residual of row r-1, and (from the fifth row on) the residual
// ((dF_1 + dF_2)) of row r-2.
template <typename T>
struct HPipe {
    T wa[4], wb[4];   // primitive states of the two rows before the entering one
    T sp[4];          // evolved upper y face value of wa's row
    T fl[4];          // flux through the lower face of wa's row
    T rx[4];          // x residual of wa's row
    int k = 0;
};

template <typename T>
__device__ __forceinline__ bool hpipe_enter(HPipe<T> &P, T g, T gi, T hl, const T *wc, T *R)
{
    if (P.k < 2) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            P.wa[f] = P.wb[f];
            P.wb[f] = wc[f];
        }
        ++P.k;
        return false;
    }
    T xm[4], xp[4], ym[4], yp[4];
    hancock_row<T>(gi, g, hl, P.wa, P.wb, wc, xm, xp, ym, yp);
    bool out = false;
    if (P.k >= 3) {
        // y face between rows wa and wb; x residual of row wb
        T F[4], Fx[4], rm[4], Rx[4];
        ausmdv2<T>(g, gi, 1, P.sp, ym, F);
#pragma unroll
        for (int f = 0; f < 4; ++f) rm[f] = lane_from_right(xm[f]);
        ausmdv2<T>(g, gi, 0, xp, rm, Fx);
#pragma unroll
        for (int f = 0; f < 4; ++f) Rx[f] = Fx[f] - lane_from_left(Fx[f]);
        if (P.k >= 4) {
#pragma unroll
            for (int f = 0; f < 4; ++f) R[f] = P.rx[f] + (F[f] - P.fl[f]);
            out = true;
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            P.fl[f] = F[f];
            P.rx[f] = Rx[f];
        }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        P.sp[f] = yp[f];
        P.wa[f] = P.wb[f];
        P.wb[f] = wc[f];
    }
    ++P.k;
    return out;
}

// One MUSCL-Hancock step (the AMR scheme, a single corrector stage) over
// the strips of the list: out = src - (dt/dx) ((dF_1 + dF_2)), out the other
// state array; with cfl set the CFL partials of the state it writes (as
// k_fv_strip).  Past t_end the state is copied.
template <typename T>
__global__ void __launch_bounds__(256) k_hancock_strip(View v, const Strip *__restrict__ list, int count,
                                                       const T *__restrict__ src, T *out, int cfl)
{
    const int done = v.meta->done;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    constexpr int H = 2;
    const int ngroups = (count + 3) / 4;
    XcdWalk walk(ngroups);
    int t;
    while (walk.next(ngroups, t)) {
        const int si = 4 * t + wid;
        if (si >= count) continue;
        const Strip st = list[si];
        const Grid G = v.grids[st.grid];
        const int n = G.n;
        const int64_t N = G.ncell;
        const int x = st.xb + lane;
        const int xc = bcmap(x, n, v.bc);
        const bool wr = lane >= H && lane < 64 - H && x < n;
        const double dt = v.mode == MODE_BATCH ? v.dt[st.grid] : v.dt[0];
        const T *S = src + G.off;
        T *O = out + G.off;
        double smax = 0.0;
        bool bad = false;
        if (done) {
            if (wr)
                for (int y = st.y0; y < st.y0 + st.ny; ++y) {
                    T q[4];
                    strip_load<T>(S, N, n, xc, y, q);
#pragma unroll
                    for (int f = 0; f < 4; ++f) O[f * N + (uint32_t)x + (uint32_t)n * (uint32_t)y] = q[f];
                }
            continue;
        }
        const T lam = (T)(dt / G.dx), hl = (T)((dt * 0.5) / G.dx);
        HPipe<T> P;
        T qa[4], qb[4];
        for (int k = 0; k < st.ny + 4; ++k) {
            const int r = st.y0 - 2 + k;
            T q[4], w[4], R[4];
            strip_load<T>(S, N, n, xc, bcmap(r, n, v.bc), q);
            cons2prim<T, 2>(q, w, g);
            const bool res = hpipe_enter<T>(P, g, gi, hl, w, R);
            if (res && wr) {
                const int ro = r - 2;
                T qn[4];
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    qn[f] = qa[f] - lam * R[f];
                    O[f * N + (uint32_t)x + (uint32_t)n * (uint32_t)ro] = qn[f];
                }
                if (cfl) strip_speed<T>(qn, v.gamma, v.cfl_max, smax, bad);
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                qa[f] = qb[f];
                qb[f] = q[f];
            }
        }
        if (cfl == 1) strip_publish(v, st.grid, smax, bad, (n - (st.xb + H) < 60 ? n - (st.xb + H) : 60) * st.ny,
                                    4 * t + wid);
        else if (cfl == 2 && smax > 1e300) atomicOr(&v.meta->status, 0);
    }
}

}  // namespace eu
