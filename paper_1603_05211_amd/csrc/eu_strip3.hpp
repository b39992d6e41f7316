// eu_strip3.hpp -- finite-volume stage on uniform 3D grids (one level), one
// workgroup per strip.
//
// A strip is 64 consecutive columns (lane l holds column xb + l) of W
// consecutive rows (wave w holds row y0 - 2 + w: two halo rows at each
// end) and a run of planes.  The workgroup marches through the planes: each
// wave converts its row of the entering plane to primitive variables once
// and keeps a window of three planes in registers for the z slopes, face
// states and fluxes; the x slopes and fluxes of a row come from the
// neighbouring lanes (DPP wave shifts), the y ones from the neighbouring
// rows through LDS (three workgroup barriers per plane: rows published,
// upper face states published, face fluxes published).  Halo rows only load
// (and, next to the output rows, provide y face states and fluxes), so
// their waves cost little issue time.  The arithmetic is the stage kernel's
// expression tree operation for operation (slope, face states, AUSM+,
// ((dF_1 + dF_2) + dF_3), q - lam R): FP64 results are identical to it.
#pragma once

namespace eu {

// x residual dF_1 of a row of primitive states w (3D; lane = column).
template <typename T>
__device__ __forceinline__ void strip_rx3(T g, T gi, const T *w, T *R)
{
    T xm[5], xp[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const T l = lane_from_left(w[f]), r = lane_from_right(w[f]);
        const T sl = slope_va<T>(l, w[f], r);
        xm[f] = w[f] - T(0.5) * sl;
        xp[f] = w[f] + T(0.5) * sl;
    }
    T rm[5], F[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) rm[f] = lane_from_right(xm[f]);
    ausm_plus<T, 3>(g, gi, 0, xp, rm, F);   // face i+1/2
#pragma unroll
    for (int f = 0; f < 5; ++f) R[f] = F[f] - lane_from_left(F[f]);
}

// One stage (stage 1: src = Q, base = Q, out = Q*, own_base set; stage 2:
// src = Q*, base = Q, out = Q) over the strips of the list; with cfl set the
// CFL partials of the state it writes (as k_fv_strip).  W waves per
// workgroup (W - 4 output rows per strip); strips walked XCD by XCD.
template <typename T, int W>
__global__ void __launch_bounds__(W * 64) k_fv_strip3(View v, const Strip *__restrict__ list, int count,
                                                      const T *__restrict__ src, const T *base, T *out, double fac,
                                                      int own_base, int cfl)
{
    constexpr int NV = 5, H = 2;
    // per row: the primitive states of the plane being finished, then the
    // flux through its lower y face (two planes in flight, by parity)
    __shared__ T sW[2][W][NV][64];
    // per row: the upper y face state of the plane being finished
    __shared__ T sP[W][NV][64];
    if (v.meta->done) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    XcdWalk walk(count);
    int si;
    while (walk.next(count, si)) {
        const Strip st = list[si];
        const Grid G = v.grids[st.grid];
        const int n = G.n;
        const int64_t N = G.ncell;
        const int x = st.xb + lane;
        const int xc = bcmap(x, n, v.bc);
        const int j = w - 2;   // this wave's row relative to the first output row
        const int yc = bcmap(st.y0 + j, n, v.bc);
        const bool live = j <= st.ny + 1;            // row loaded
        const bool slope = j >= -1 && j <= st.ny;    // y face states needed
        const bool face = j >= 0 && j <= st.ny;      // its lower y face flux needed
        const bool outr = j >= 0 && j < st.ny;       // output row
        const bool wr = outr && lane >= H && lane < 64 - H && x < n;
        const double dt = v.mode == MODE_BATCH ? v.dt[st.grid] : v.dt[0];
        const T lam = (T)((dt * fac) / G.dx);
        const T *S = src + G.off;
        const T *B = base + G.off;
        T *O = out + G.off;
        const uint32_t rowoff = (uint32_t)xc + (uint32_t)n * (uint32_t)yc;
        const uint32_t nn = (uint32_t)n * (uint32_t)n;
        T wa[NV], wb[NV], sp[NV], fl[NV], qa[NV], qb[NV];
        double smax = 0.0;
        bool bad = false;
        for (int k = 0; k < st.nz + 4; ++k) {
            const int z = st.z0 - 2 + k;
            T q[NV], wc[NV];
            if (live) {
                const uint32_t id = rowoff + nn * (uint32_t)bcmap(z, n, v.bc);
#pragma unroll
                for (int f = 0; f < NV; ++f) q[f] = S[f * N + id];
                cons2prim<T, 3>(q, wc, g);
            }
            // z slope of plane wb; the z face between planes wa and wb
            T spn[NV], Fz[NV];
            if (outr && k >= 2) {
                T sm[NV];
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    const T sl = slope_va<T>(wa[f], wb[f], wc[f]);
                    sm[f] = wb[f] - T(0.5) * sl;
                    spn[f] = wb[f] + T(0.5) * sl;
                }
                if (k >= 3) ausm_plus<T, 3>(g, gi, 2, sp, sm, Fz);
            }
            if (k >= 4) {
                // plane wa (z - 2) is finished: y faces through LDS, x faces
                // by lane shifts, the update
                const int par = k & 1;
                if (live)
#pragma unroll
                    for (int f = 0; f < NV; ++f) sW[par][w][f][lane] = wa[f];
                __syncthreads();
                T ym[NV];
                if (slope) {
#pragma unroll
                    for (int f = 0; f < NV; ++f) {
                        const T sl = slope_va<T>(sW[par][w - 1][f][lane], wa[f], sW[par][w + 1][f][lane]);
                        ym[f] = wa[f] - T(0.5) * sl;
                        sP[w][f][lane] = wa[f] + T(0.5) * sl;
                    }
                }
                __syncthreads();
                T Fy[NV];
                if (face) {
                    T yl[NV];
#pragma unroll
                    for (int f = 0; f < NV; ++f) yl[f] = sP[w - 1][f][lane];
                    ausm_plus<T, 3>(g, gi, 1, yl, ym, Fy);
#pragma unroll
                    for (int f = 0; f < NV; ++f) sW[par][w][f][lane] = Fy[f];
                }
                __syncthreads();
                if (outr) {
                    T Rx[NV], qo[NV];
                    strip_rx3<T>(g, gi, wa, Rx);
                    const uint32_t ido = rowoff + nn * (uint32_t)(z - 2);
                    if (own_base) {
#pragma unroll
                        for (int f = 0; f < NV; ++f) qo[f] = qa[f];
                    } else {
#pragma unroll
                        for (int f = 0; f < NV; ++f) qo[f] = B[f * N + ido];
                    }
                    if (wr) {
                        T qn[NV];
#pragma unroll
                        for (int f = 0; f < NV; ++f) {
                            const T R = (Rx[f] + (sW[par][w + 1][f][lane] - Fy[f])) + (Fz[f] - fl[f]);
                            qn[f] = qo[f] - lam * R;
                            O[f * N + ido] = qn[f];
                        }
                        if (cfl) strip_speed<T, 3>(qn, v.gamma, smax, bad);
                    }
                }
            }
            if (outr && k >= 3)
#pragma unroll
                for (int f = 0; f < NV; ++f) fl[f] = Fz[f];
            if (outr && k >= 2)
#pragma unroll
                for (int f = 0; f < NV; ++f) sp[f] = spn[f];
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                wa[f] = wb[f];
                wb[f] = wc[f];
                qa[f] = qb[f];
                qb[f] = q[f];
            }
        }
        if (outr) {
            const int nx = n - (st.xb + H) < 64 - 2 * H ? n - (st.xb + H) : 64 - 2 * H;
            if (cfl == 1) strip_publish(v, st.grid, smax, bad, nx * st.nz, W * blockIdx.x + w);
            else if (cfl == 2 && smax > 1e300) atomicOr(&v.meta->status, 0);
        }
        // the next strip writes the row buffers again
        __syncthreads();
    }
}

}  // namespace eu
