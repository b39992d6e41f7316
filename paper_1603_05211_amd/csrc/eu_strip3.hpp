// eu_strip3.hpp -- finite-volume stage on uniform 3D grids (one level), one
// workgroup per strip.
//
// A strip is 64 consecutive columns (lane l holds column xb + l) of W
// consecutive output rows (wave w holds row y0 + w; waves 0, 1, W-2 and W-1
// also hold one of the two halo rows at each end) and a run of planes.  The
// workgroup marches through the planes: each wave converts its row of the entering plane to primitive variables once
// and keeps a window of three planes in registers for the z slopes, face
// states and fluxes; the x slopes and fluxes of a row come from the
// neighbouring lanes (DPP wave shifts), the y ones from the neighbouring
// rows through LDS (three workgroup barriers per plane: rows published,
// upper face states published, face fluxes published).  Halo rows only load
// and, next to the output rows, provide y face states and fluxes.  Four
// waves per SIMD are asked for (two workgroups of 8 rows, or one of 16, per
// CU).  The arithmetic is the stage kernel's expression tree operation for
// operation (slope, face states, AUSM+, ((dF_1 + dF_2) + dF_3), q - lam R):
// FP64 results are identical to it.
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

// One row of a 3D strip: its z window of primitive states (wa, wb) and,
// for an output row, the base window (qa, qb) and the z faces (sp, fl).
template <typename T>
struct Row3 {
    T wa[5], wb[5], qa[5], qb[5], sp[5], fl[5];
};

// One stage (stage 1: src = Q, base = Q, out = Q*, own_base set; stage 2:
// src = Q*, base = Q, out = Q) over the strips of the list; with cfl set the
// CFL partials of the state it writes (as k_fv_strip).  W waves per
// workgroup, wave w on output row y0 + w; the two halo rows below the first
// output row go to waves 0 and 1, the two above the last to waves W-2 and
// W-1 (a second row each: loads, and the y face values or fluxes the
// output rows need), so every wave has an output row.  Strips walked XCD
// by XCD.
template <typename T, int W>
__global__ void __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4))) k_fv_strip3(View v, const Strip *__restrict__ list, int count,
                                                      const T *__restrict__ src, const T *base, T *out, double fac,
                                                      int own_base, int cfl)
{
    constexpr int NV = 5, H = 2, NR = W + 4;
    // per row (row index j + 2): the primitive states of the plane being
    // finished, then the flux through its lower y face (two planes in
    // flight, by parity)
    __shared__ T sW[2][NR][NV][64];
    // per row: the upper y face state of the plane being finished
    __shared__ T sP[NR][NV][64];
    if (v.meta->done) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const T g = (T)v.gamma;
    const T gi = (T)(1.0 / (v.gamma - 1.0));
    // the wave's second row: halo rows -2, -1 (waves 0, 1) and W, W+1
    // (waves W-2, W-1)
    const bool has2 = w < 2 || w >= W - 2;
    const int j2 = w < 2 ? w - 2 : w + 2;
    XcdWalk walk(count);
    int si;
    while (walk.next(count, si)) {
        const Strip st = list[si];
        const Grid G = v.grids[st.grid];
        const int n = G.n;
        const int64_t N = G.ncell;
        const int x = st.xb + lane;
        const int xc = bcmap(x, n, v.bc);
        const int ny = st.ny;
        // roles of a row j (relative to the first output row): loaded, its y
        // face values needed, its lower y face flux needed, output
        const int j1 = w;
        const bool live1 = j1 <= ny + 1, slope1 = j1 <= ny, face1 = j1 <= ny, outr = j1 < ny;
        const bool live2 = has2 && j2 <= ny + 1, slope2 = has2 && j2 >= -1 && j2 <= ny;
        const bool face2 = has2 && j2 >= 0 && j2 <= ny;
        const bool wr = outr && lane >= H && lane < 64 - H && x < n;
        const double dt = v.mode == MODE_BATCH ? v.dt[st.grid] : v.dt[0];
        const T lam = (T)((dt * fac) / G.dx);
        const T *S = src + G.off;
        const T *B = base + G.off;
        T *O = out + G.off;
        const uint32_t nn = (uint32_t)n * (uint32_t)n;
        const uint32_t off1 = (uint32_t)xc + (uint32_t)n * (uint32_t)bcmap(st.y0 + j1, n, v.bc);
        const uint32_t off2 = (uint32_t)xc + (uint32_t)n * (uint32_t)bcmap(st.y0 + j2, n, v.bc);
        Row3<T> A;                 // primary row
        T wa2[NV], wb2[NV];        // second row's window
        double smax = 0.0;
        bool bad = false;
        for (int k = 0; k < st.nz + 4; ++k) {
            const int z = st.z0 - 2 + k;
            const uint32_t zo = nn * (uint32_t)bcmap(z, n, v.bc);
            T q[NV], wc[NV], q2[NV], wc2[NV];
            if (live1) {
#pragma unroll
                for (int f = 0; f < NV; ++f) q[f] = S[f * N + off1 + zo];
            }
            if (live2) {
#pragma unroll
                for (int f = 0; f < NV; ++f) q2[f] = S[f * N + off2 + zo];
            }
            if (live1) cons2prim<T, 3>(q, wc, g);
            if (live2) cons2prim<T, 3>(q2, wc2, g);
            // z slope of plane wb; the z face between planes wa and wb
            T spn[NV], Fz[NV];
            if (outr && k >= 2) {
                T sm[NV];
#pragma unroll
                for (int f = 0; f < NV; ++f) {
                    const T sl = slope_va<T>(A.wa[f], A.wb[f], wc[f]);
                    sm[f] = A.wb[f] - T(0.5) * sl;
                    spn[f] = A.wb[f] + T(0.5) * sl;
                }
                if (k >= 3) ausm_plus<T, 3>(g, gi, 2, A.sp, sm, Fz);
            }
            if (k >= 4) {
                // plane wa (z - 2) is finished: y faces through LDS, x faces
                // by lane shifts, the update
                const int par = k & 1;
                if (live1)
#pragma unroll
                    for (int f = 0; f < NV; ++f) sW[par][j1 + 2][f][lane] = A.wa[f];
                if (live2)
#pragma unroll
                    for (int f = 0; f < NV; ++f) sW[par][j2 + 2][f][lane] = wa2[f];
                __syncthreads();
                T ym1[NV], ym2[NV];
                if (slope1) {
#pragma unroll
                    for (int f = 0; f < NV; ++f) {
                        const T sl = slope_va<T>(sW[par][j1 + 1][f][lane], A.wa[f], sW[par][j1 + 3][f][lane]);
                        ym1[f] = A.wa[f] - T(0.5) * sl;
                        sP[j1 + 2][f][lane] = A.wa[f] + T(0.5) * sl;
                    }
                }
                if (slope2) {
#pragma unroll
                    for (int f = 0; f < NV; ++f) {
                        const T sl = slope_va<T>(sW[par][j2 + 1][f][lane], wa2[f], sW[par][j2 + 3][f][lane]);
                        ym2[f] = wa2[f] - T(0.5) * sl;
                        sP[j2 + 2][f][lane] = wa2[f] + T(0.5) * sl;
                    }
                }
                __syncthreads();
                T Fy[NV];
                if (face1) {
                    T yl[NV];
#pragma unroll
                    for (int f = 0; f < NV; ++f) yl[f] = sP[j1 + 1][f][lane];
                    ausm_plus<T, 3>(g, gi, 1, yl, ym1, Fy);
#pragma unroll
                    for (int f = 0; f < NV; ++f) sW[par][j1 + 2][f][lane] = Fy[f];
                }
                if (face2) {
                    T yl[NV], F2[NV];
#pragma unroll
                    for (int f = 0; f < NV; ++f) yl[f] = sP[j2 + 1][f][lane];
                    ausm_plus<T, 3>(g, gi, 1, yl, ym2, F2);
#pragma unroll
                    for (int f = 0; f < NV; ++f) sW[par][j2 + 2][f][lane] = F2[f];
                }
                __syncthreads();
                if (outr) {
                    T Rx[NV], qo[NV];
                    strip_rx3<T>(g, gi, A.wa, Rx);
                    const uint32_t ido = off1 + nn * (uint32_t)(z - 2);
                    if (own_base) {
#pragma unroll
                        for (int f = 0; f < NV; ++f) qo[f] = A.qa[f];
                    } else {
#pragma unroll
                        for (int f = 0; f < NV; ++f) qo[f] = B[f * N + ido];
                    }
                    if (wr) {
                        T qn[NV];
#pragma unroll
                        for (int f = 0; f < NV; ++f) {
                            const T R = (Rx[f] + (sW[par][j1 + 3][f][lane] - Fy[f])) + (Fz[f] - A.fl[f]);
                            qn[f] = qo[f] - lam * R;
                            O[f * N + ido] = qn[f];
                        }
                        if (cfl) strip_speed<T, 3>(qn, v.gamma, v.cfl_max, smax, bad);
                    }
                }
            }
            if (outr && k >= 3)
#pragma unroll
                for (int f = 0; f < NV; ++f) A.fl[f] = Fz[f];
            if (outr && k >= 2)
#pragma unroll
                for (int f = 0; f < NV; ++f) A.sp[f] = spn[f];
#pragma unroll
            for (int f = 0; f < NV; ++f) {
                A.wa[f] = A.wb[f];
                A.wb[f] = wc[f];
                A.qa[f] = A.qb[f];
                A.qb[f] = q[f];
                wa2[f] = wb2[f];
                wb2[f] = wc2[f];
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
