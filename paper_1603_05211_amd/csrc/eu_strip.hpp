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
// largest signal speed sum_d (|v_d| + c) of its cells (as the CFL reduction
// kernel would on that state) and adds it into the grid's maximum (a batch)
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
template <typename T>
__device__ __forceinline__ void strip_speed(const T *q, double g, double &m, bool &bad)
{
    double qd[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) qd[f] = (double)q[f];
    bool b;
    const double S = cell_speed<2>(qd, g, b);
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
                        if (cfl) strip_speed<T>(qn, v.gamma, smax, bad);
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
                            if (cfl) strip_speed<T>(qn, v.gamma, smax, bad);
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

}  // namespace eu
