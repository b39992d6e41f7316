// eu_mesh.hip -- precision-independent kernels: CFL time-step finalisation,
// time advance, refinement flags with buffer and nesting closure, patch
// tiling with the efficiency rule, work-list construction, totals.
// Built with -ffp-contract=off.
#include "eu_kernels.hpp"

namespace eu {

// ----------------------------------------------------------------------------
// dt = min over levels of cfl dx_l / smax_l (hierarchy) or per instance
// (batch), clipped to reach t_end; a step starting at t >= t_end is skipped
// by every later kernel of the step (meta->done).
// ----------------------------------------------------------------------------
__global__ void k_cfl_finalize(View v)
{
    if (v.mode == MODE_HIER) {
        if (threadIdx.x != 0 || blockIdx.x != 0) return;
        double dt = __builtin_inf();
        for (int g = 0; g < v.ngrid; ++g) {
            const unsigned long long b = v.smax[g];
            if (b) {
                const double s = __longlong_as_double((long long)b);
                const double dtl = (v.cfl * v.grids[g].dx) / s;
                if (dtl < dt) dt = dtl;
            }
            v.smax[g] = 0ull;
        }
        const double t = v.t[0];
        v.meta->done = t < v.t_end ? 0 : 1;
        if (dt > v.t_end - t) dt = v.t_end - t;
        v.dt[0] = dt;
        return;
    }
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < v.ngrid; g += gridDim.x * blockDim.x) {
        const unsigned long long b = v.smax[g];
        const double s = __longlong_as_double((long long)b);
        double dt = b ? (v.cfl * v.grids[g].dx) / s : 0.0;
        const double t = v.t[g];
        if (dt > v.t_end - t) dt = v.t_end - t;
        v.dt[g] = dt;
        v.smax[g] = 0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) v.meta->done = 0;
}

__global__ void k_time_advance(View v)
{
    if (v.meta->done) return;
    const int ng = v.mode == MODE_HIER ? 1 : v.ngrid;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x)
        v.t[g] = v.t[g] + v.dt[g];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        v.meta->steps += 1;
        if (v.mode == MODE_HIER) {
            long long s = 0;
            for (int l = 0; l < v.L; ++l) s += v.meta->leaf_cells[l];
            v.meta->leaf_updates += s;
        }
    }
}

__global__ void k_zero_nflag(View v)
{
    if (v.meta->done) return;
    if (threadIdx.x < MAXLEV) v.meta->nflag[threadIdx.x] = 0;
}

// ----------------------------------------------------------------------------
// refinement flags of level lvl (decide level lvl+1 of the new hierarchy)
// ----------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_flags(View v, int lvl)
{
    if (v.meta->done) return;
    const Grid G = v.grids[lvl];
    const int n = G.n;
    const bool has2 = lvl + 2 < v.L;
    int cnt = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G.ncell;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = D == 3 ? (int)(i / ((int64_t)n * n)) : 0;
        bool fl = false;
        const int r3 = D == 3 ? 1 : 0;
        // raw flags (significant details; preventive refinement of the
        // children of significant cells), dilated by one cell
        for (int dz = -r3; dz <= r3 && !fl; ++dz)
            for (int dy = -1; dy <= 1 && !fl; ++dy)
                for (int dx = -1; dx <= 1 && !fl; ++dx) {
                    const int qx = bcmap(x + dx, n, v.bc), qy = bcmap(y + dy, n, v.bc);
                    const int qz = D == 3 ? bcmap(z + dz, n, v.bc) : 0;
                    if (v.sig[G.coff + gidx(n, qx, qy, qz)]) fl = true;
                    else if (lvl >= 1) {
                        const Grid &Cg = v.grids[G.coarse];
                        if (v.sig[Cg.coff + gidx(Cg.n, qx >> 1, qy >> 1, qz >> 1)]) fl = true;
                    }
                }
        // nesting: level-(lvl+1) cells within two cells of a level-(lvl+1)
        // cell covered by the new level lvl+2
        if (!fl && has2) {
            const Grid &F = v.grids[G.fine];
            const Grid &F2 = v.grids[F.fine];
            const int nf = F.n;
            const int z0 = D == 3 ? -2 : 0, z1 = D == 3 ? 3 : 0;
            for (int dz = z0; dz <= z1 && !fl; ++dz)
                for (int dy = -2; dy <= 3 && !fl; ++dy)
                    for (int dx = -2; dx <= 3 && !fl; ++dx) {
                        const int qx = bcmap(2 * x + dx, nf, v.bc), qy = bcmap(2 * y + dy, nf, v.bc);
                        const int qz = D == 3 ? bcmap(2 * z + dz, nf, v.bc) : 0;
                        if (v.nact[F2.boff + (qx >> 2) + (int64_t)F2.nb * ((qy >> 2) + (int64_t)F2.nb * (qz >> 2))])
                            fl = true;
                    }
        }
        v.flag[G.coff + i] = fl ? 1 : 0;
        cnt += fl ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(&v.meta->nflag[lvl], cnt);
}

// ----------------------------------------------------------------------------
// tiling of level lvl's flags into patches of level lvl+1: one 64-lane
// workgroup per aligned pmax block (Morton index = blockIdx.x); counts per
// BS-block in LDS, then the recursive split decided by lane 0 in the same
// order as a depth-first recursion over children (x fastest).
// ----------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(64) k_tile(View v, int lvl)
{
    if (v.meta->done) return;
    constexpr int MAXSUB = D == 2 ? 64 : 512;       // (pmax / BS)^D, pmax <= 64
    __shared__ int cnt8[MAXSUB];
    __shared__ uint8_t emit8[MAXSUB];
    const Grid G = v.grids[lvl];
    const Grid F = v.grids[lvl + 1];
    const int R = v.pmax / BS;                      // BS-blocks per pmax block side
    const int nsub = D == 2 ? R * R : R * R * R;
    const int m = blockIdx.x;
    int bp[3] = {0, 0, 0};
    {
        const int nbp = F.n / v.pmax;
        int bits = 0;
        while ((1 << bits) < nbp) ++bits;
        for (int k = 0; k < bits; ++k)
            for (int d = 0; d < D; ++d) bp[d] |= ((m >> (k * D + d)) & 1) << k;
    }
    // flagged parents per BS-block (coarse footprint (BS/2)^D)
    for (int s = threadIdx.x; s < nsub; s += 64) {
        const int sx = s % R, sy = (s / R) % R, sz = D == 3 ? s / (R * R) : 0;
        const int cx = (bp[0] * v.pmax + sx * BS) / 2, cy = (bp[1] * v.pmax + sy * BS) / 2;
        const int cz = D == 3 ? (bp[2] * v.pmax + sz * BS) / 2 : 0;
        int c = 0;
        const int hz = D == 3 ? BS / 2 : 1;
        for (int z = 0; z < hz; ++z)
            for (int y = 0; y < BS / 2; ++y)
                for (int x = 0; x < BS / 2; ++x) c += v.flag[G.coff + gidx(G.n, cx + x, cy + y, cz + z)];
        cnt8[s] = c;
        emit8[s] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t slot = v.pbase[lvl + 1] + m;
        int *out = v.pslot + slot * (int64_t)nsub * 5;
        int np = 0;
        short st[4 * 32];
        int sp = 0;
        st[0] = 0; st[1] = 0; st[2] = 0; st[3] = (short)R;
        sp = 1;
        while (sp) {
            --sp;
            const int ex = st[4 * sp], ey = st[4 * sp + 1], ez = st[4 * sp + 2], es = st[4 * sp + 3];
            long long c = 0;
            const int ezs = D == 3 ? es : 1;
            for (int z = 0; z < ezs; ++z)
                for (int y = 0; y < es; ++y)
                    for (int x = 0; x < es; ++x) c += cnt8[(ex + x) + R * ((ey + y) + (D == 3 ? R * (ez + z) : 0))];
            if (c == 0) continue;
            const int S = es * BS, hsz = S / 2;
            const long long cells = D == 2 ? (long long)hsz * hsz : (long long)hsz * hsz * hsz;
            if (S == v.pmin || (double)c >= v.eta * (double)cells) {
                out[5 * np + 0] = lvl + 1;
                out[5 * np + 1] = bp[0] * v.pmax + ex * BS;
                out[5 * np + 2] = bp[1] * v.pmax + ey * BS;
                out[5 * np + 3] = D == 3 ? bp[2] * v.pmax + ez * BS : 0;
                out[5 * np + 4] = S;
                ++np;
                for (int z = 0; z < ezs; ++z)
                    for (int y = 0; y < es; ++y)
                        for (int x = 0; x < es; ++x)
                            emit8[(ex + x) + R * ((ey + y) + (D == 3 ? R * (ez + z) : 0))] = 1;
                continue;
            }
            const int hs = es / 2;
            for (int k = (1 << D) - 1; k >= 0; --k) {
                st[4 * sp] = (short)(ex + hs * (k & 1));
                st[4 * sp + 1] = (short)(ey + hs * ((k >> 1) & 1));
                st[4 * sp + 2] = (short)(D == 3 ? ez + hs * ((k >> 2) & 1) : 0);
                st[4 * sp + 3] = (short)hs;
                ++sp;
            }
        }
        v.pcnt[slot] = np;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nsub; s += 64) {
        const int sx = s % R, sy = (s / R) % R, sz = D == 3 ? s / (R * R) : 0;
        const int bx = bp[0] * R + sx, by = bp[1] * R + sy, bz = D == 3 ? bp[2] * R + sz : 0;
        v.nact[F.boff + bx + (int64_t)F.nb * (by + (int64_t)F.nb * bz)] = emit8[s];
    }
}

// ----------------------------------------------------------------------------
// work lists from the new hierarchy (one workgroup; deterministic order:
// level, then block index x fastest); then current = new.
// ----------------------------------------------------------------------------
constexpr int LT = 1024;

__device__ __forceinline__ void block_coords(int b, int nb, int D, int &x, int &y, int &z)
{
    x = b % nb;
    y = (b / nb) % nb;
    z = D == 3 ? b / (nb * nb) : 0;
}

// exclusive scan over the LT threads of K counters held in sc[K][LT]
template <int K>
__device__ void scan_lt(int (*sc)[LT], int *tot)
{
    for (int off = 1; off < LT; off <<= 1) {
        int add[K];
        for (int k = 0; k < K; ++k) add[k] = threadIdx.x >= (unsigned)off ? sc[k][threadIdx.x - off] : 0;
        __syncthreads();
        for (int k = 0; k < K; ++k) sc[k][threadIdx.x] += add[k];
        __syncthreads();
    }
    // inclusive -> exclusive
    int mine[K];
    for (int k = 0; k < K; ++k) mine[k] = threadIdx.x ? sc[k][threadIdx.x - 1] : 0;
    if (threadIdx.x == LT - 1)
        for (int k = 0; k < K; ++k) tot[k] = sc[k][LT - 1];
    __syncthreads();
    for (int k = 0; k < K; ++k) sc[k][threadIdx.x] = mine[k];
    __syncthreads();
}

template <int D>
__device__ void classify(const View &v, int lvl, int b, bool &leaf, bool &cov, bool &ghost, bool &fresh,
                         int &nleafcell)
{
    const Grid &G = v.grids[lvl];
    const int nb = G.nb;
    int bx, by, bz;
    block_coords(b, nb, D, bx, by, bz);
    const bool a = v.nact[G.boff + b] != 0;
    const bool old = v.act[G.boff + b] != 0;
    int nchild = 0;
    if (a && G.fine >= 0) {
        const Grid &F = v.grids[G.fine];
        const int zs = D == 3 ? 2 : 1;
        for (int z = 0; z < zs; ++z)
            for (int y = 0; y < 2; ++y)
                for (int x = 0; x < 2; ++x)
                    nchild += v.nact[F.boff + (2 * bx + x) + (int64_t)F.nb * ((2 * by + y) + (int64_t)F.nb * (2 * bz + z))];
    }
    const int nch_all = D == 2 ? 4 : 8;
    leaf = a && nchild < nch_all;
    cov = a && nchild > 0;
    fresh = a && !old && lvl >= 1;
    const int cpb = D == 2 ? BS * BS : BS * BS * BS;
    const int cpc = D == 2 ? (BS / 2) * (BS / 2) : (BS / 2) * (BS / 2) * (BS / 2);
    nleafcell = a ? cpb - nchild * cpc : 0;
    ghost = false;
    if (!a && lvl >= 1) {
        const int r3 = D == 3 ? 1 : 0;
        for (int dz = -r3; dz <= r3 && !ghost; ++dz)
            for (int dy = -1; dy <= 1 && !ghost; ++dy)
                for (int dx = -1; dx <= 1 && !ghost; ++dx) {
                    const int qx = bcmap(bx + dx, nb, v.bc), qy = bcmap(by + dy, nb, v.bc);
                    const int qz = D == 3 ? bcmap(bz + dz, nb, v.bc) : 0;
                    if (v.nact[G.boff + qx + (int64_t)nb * (qy + (int64_t)nb * qz)]) ghost = true;
                }
    }
}

template <int D>
__global__ void __launch_bounds__(LT) k_build_lists(View v, int64_t nbt)
{
    __shared__ int sc[4][LT];
    __shared__ int tot[4];
    __shared__ int lvl_start[MAXLEV + 1];
    __shared__ int covc[MAXLEV], newc[MAXLEV];
    __shared__ long long leafcells[MAXLEV], actcells[MAXLEV];
    if (v.meta->done) return;
    if (threadIdx.x == 0) {
        int64_t s = 0;
        for (int l = 0; l < v.L; ++l) {
            lvl_start[l] = (int)s;
            const int nb = v.grids[l].nb;
            s += D == 2 ? (int64_t)nb * nb : (int64_t)nb * nb * nb;
        }
        lvl_start[v.L] = (int)s;
    }
    if (threadIdx.x < MAXLEV) {
        covc[threadIdx.x] = 0; newc[threadIdx.x] = 0;
        leafcells[threadIdx.x] = 0; actcells[threadIdx.x] = 0;
    }
    __syncthreads();
    const int64_t chunk = (nbt + LT - 1) / LT;
    const int64_t b0 = threadIdx.x * chunk, b1 = b0 + chunk < nbt ? b0 + chunk : nbt;
    int c[4] = {0, 0, 0, 0};
    long long lc[MAXLEV], ac[MAXLEV];
    int cc[MAXLEV], nc[MAXLEV];
    for (int l = 0; l < MAXLEV; ++l) { lc[l] = 0; ac[l] = 0; cc[l] = 0; nc[l] = 0; }
    int lvl = 0;
    for (int64_t gb = b0; gb < b1; ++gb) {
        while (gb >= lvl_start[lvl + 1]) ++lvl;
        bool leaf, cov, ghost, fresh;
        int nlc;
        classify<D>(v, lvl, (int)(gb - lvl_start[lvl]), leaf, cov, ghost, fresh, nlc);
        c[0] += leaf; c[1] += cov; c[2] += ghost; c[3] += fresh;
        cc[lvl] += cov; nc[lvl] += fresh;
        lc[lvl] += nlc;
        ac[lvl] += v.nact[v.grids[lvl].boff + (gb - lvl_start[lvl])] ? (D == 2 ? BS * BS : BS * BS * BS) : 0;
    }
    for (int l = 0; l < v.L; ++l) {
        if (cc[l]) atomicAdd(&covc[l], cc[l]);
        if (nc[l]) atomicAdd(&newc[l], nc[l]);
        if (lc[l]) atomicAdd((unsigned long long *)&leafcells[l], (unsigned long long)lc[l]);
        if (ac[l]) atomicAdd((unsigned long long *)&actcells[l], (unsigned long long)ac[l]);
    }
    for (int k = 0; k < 4; ++k) sc[k][threadIdx.x] = c[k];
    __syncthreads();
    scan_lt<4>(sc, tot);
    int pos[4];
    for (int k = 0; k < 4; ++k) pos[k] = sc[k][threadIdx.x];
    lvl = 0;
    for (int64_t gb = b0; gb < b1; ++gb) {
        while (gb >= lvl_start[lvl + 1]) ++lvl;
        const int b = (int)(gb - lvl_start[lvl]);
        bool leaf, cov, ghost, fresh;
        int nlc;
        classify<D>(v, lvl, b, leaf, cov, ghost, fresh, nlc);
        const Tile tl = {lvl, b};
        if (leaf) v.leaf[pos[0]++] = tl;
        if (cov) v.cov[pos[1]++] = tl;
        if (ghost) v.ghost[pos[2]++] = tl;
        if (fresh) v.fresh[pos[3]++] = tl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v.meta->nleaf = tot[0];
        v.meta->nghost = tot[2];
        int co = 0, no = 0;
        for (int l = 0; l < MAXLEV; ++l) {
            const int cl = l < v.L ? covc[l] : 0, nl = l < v.L ? newc[l] : 0;
            v.meta->cov_off[l] = co; v.meta->cov_cnt[l] = cl; co += cl;
            v.meta->new_off[l] = no; v.meta->new_cnt[l] = nl; no += nl;
            v.meta->leaf_cells[l] = l < v.L ? leafcells[l] : 0;
            v.meta->act_cells[l] = l < v.L ? actcells[l] : 0;
        }
    }
    // patch table: per level >= 1, pmax blocks in Morton order
    int64_t nslot = 0;
    for (int l = 1; l < v.L; ++l) {
        const int nbp = v.grids[l].n / v.pmax;
        nslot += D == 2 ? (int64_t)nbp * nbp : (int64_t)nbp * nbp * nbp;
    }
    const int R = v.pmax / BS;
    const int nsub = D == 2 ? R * R : R * R * R;
    const int64_t pch = (nslot + LT - 1) / LT;
    const int64_t s0 = v.L > 1 ? v.pbase[1] : 0;
    const int64_t p0 = s0 + threadIdx.x * pch;
    const int64_t p1 = p0 + pch < s0 + nslot ? p0 + pch : s0 + nslot;
    int np = 0;
    for (int64_t s = p0; s < p1; ++s) np += v.pcnt[s];
    sc[0][threadIdx.x] = np;
    __syncthreads();
    scan_lt<1>(sc, tot);
    int w = sc[0][threadIdx.x];
    for (int64_t s = p0; s < p1; ++s) {
        const int k = v.pcnt[s];
        for (int j = 0; j < k; ++j) {
            if (w < v.max_patch)
                for (int e = 0; e < 5; ++e) v.patches[5 * (int64_t)w + e] = v.pslot[(s * nsub + j) * 5 + e];
            ++w;
        }
    }
    if (threadIdx.x == 0) v.meta->npatch = tot[0];
    __syncthreads();
    // the new hierarchy becomes the current one
    for (int64_t gb = threadIdx.x; gb < nbt; gb += LT) v.act[gb] = v.nact[gb];
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t val)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// totals per group (hierarchy: all leaves; batch: one instance), fixed order
__global__ void k_totals_final(View v, int ngroups)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ngroups * v.nv) return;
    const int grp = i / v.nv, f = i % v.nv;
    int off, cnt;
    if (v.mode == MODE_HIER) { off = 0; cnt = v.meta->nleaf; }
    else { off = v.grp_off[grp]; cnt = v.grp_cnt[grp]; }
    double s = 0.0;
    for (int t = 0; t < cnt; ++t) s = s + v.partial[(int64_t)(off + t) * v.nv + f];
    v.totals[i] = s;
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
static inline int grid_for(int64_t n, int bs, int cap)
{
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    return g > cap ? cap : (int)g;
}

void launch_cfl_finalize(const View &v, hipStream_t s)
{
    k_cfl_finalize<<<v.mode == MODE_HIER ? 1 : grid_for(v.ngrid, 256, 64), v.mode == MODE_HIER ? 64 : 256, 0, s>>>(v);
}

void launch_time_advance(const View &v, hipStream_t s)
{
    k_time_advance<<<v.mode == MODE_HIER ? 1 : grid_for(v.ngrid, 256, 64), 256, 0, s>>>(v);
}

void launch_zero_meta_flags(const View &v, hipStream_t s) { k_zero_nflag<<<1, 64, 0, s>>>(v); }

void launch_flags(const View &v, int lvl, int64_t ncell, hipStream_t s)
{
    if (v.dim == 2) k_flags<2><<<grid_for(ncell, 256, 8192), 256, 0, s>>>(v, lvl);
    else k_flags<3><<<grid_for(ncell, 256, 8192), 256, 0, s>>>(v, lvl);
}

void launch_tile(const View &v, int lvl, int nblocks, hipStream_t s)
{
    if (v.dim == 2) k_tile<2><<<nblocks, 64, 0, s>>>(v, lvl);
    else k_tile<3><<<nblocks, 64, 0, s>>>(v, lvl);
}

void launch_build_lists(const View &v, int64_t nbt, hipStream_t s)
{
    if (v.dim == 2) k_build_lists<2><<<1, LT, 0, s>>>(v, nbt);
    else k_build_lists<3><<<1, LT, 0, s>>>(v, nbt);
}

void launch_fill_u8(uint8_t *p, int64_t n, uint8_t val, hipStream_t s)
{
    k_fill_u8<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, val);
}

void launch_totals_final(const View &v, int ngroups, hipStream_t s)
{
    k_totals_final<<<grid_for((int64_t)ngroups * v.nv, 64, 4096), 64, 0, s>>>(v, ngroups);
}

}  // namespace eu
