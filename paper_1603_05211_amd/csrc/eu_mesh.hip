// eu_mesh.hip -- precision-independent kernels: refinement flags with buffer
// and nesting closure fused with the patch tiling (efficiency rule), work-list
// construction (parallel classification + one-workgroup compaction), fills,
// totals.  Built with -ffp-contract=off.
#include "eu_kernels.hpp"

namespace eu {

// ----------------------------------------------------------------------------
// refinement flag of level-lvl cell (x, y, z): it decides whether the cell's
// children belong to level lvl+1 of the new hierarchy
// ----------------------------------------------------------------------------
// Distinct blocks (block side 8 at level side n) touched by cells
// c + lo .. c + hi through the boundary map; at most 3 for hi - lo <= 5 at
// half resolution, returned in out[], count returned.
__device__ __forceinline__ int distinct_blocks(int c0, int lo, int hi, int n, int bc, int shift, int *out)
{
    int k = 0;
    for (int o = lo; o <= hi; ++o) {
        const int b = bcmap(c0 + o, n, bc) >> shift;
        bool seen = false;
        for (int j = 0; j < k; ++j) seen |= out[j] == b;
        if (!seen) out[k++] = b;
    }
    return k;
}

template <int D>
__device__ __forceinline__ bool refine_flag(const View &v, const Grid &G, int lvl, int x, int y, int z)
{
    const int n = G.n;
    constexpr int R3 = D == 3 ? 1 : 0;
    constexpr int NN = D == 3 ? 27 : 9;
    // raw flags (significant details; preventive refinement of the children
    // of significant cells), dilated by one cell; all loads issued first
    uint8_t s[NN], sp[NN];
    int k = 0;
#pragma unroll
    for (int dz = -R3; dz <= R3; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int qx = bcmap(x + dx, n, v.bc), qy = bcmap(y + dy, n, v.bc);
                const int qz = D == 3 ? bcmap(z + dz, n, v.bc) : 0;
                s[k] = v.sig[G.coff + gidx(n, qx, qy, qz)];
                sp[k] = 0;
                if (lvl >= 1) {
                    const Grid &Cg = v.grids[G.coarse];
                    sp[k] = v.sig[Cg.coff + gidx(Cg.n, qx >> 1, qy >> 1, qz >> 1)];
                }
                ++k;
            }
    int any = 0;
#pragma unroll
    for (int j = 0; j < NN; ++j) any |= s[j] | sp[j];
    if (any) return true;
    // nesting: level-(lvl+1) cells within two cells of a level-(lvl+1) cell
    // covered by the new level lvl+2; cells 2x-2 .. 2x+3 of level lvl+1 lie
    // in at most three blocks of level lvl+2 per axis
    if (lvl + 2 < v.L) {
        const Grid &F = v.grids[G.fine];
        const Grid &F2 = v.grids[F.fine];
        const int nf = F.n;
        int bx[3], by[3], bz[3] = {0, 0, 0};
        const int nx = distinct_blocks(2 * x, -2, 3, nf, v.bc, 2, bx);
        const int ny = distinct_blocks(2 * y, -2, 3, nf, v.bc, 2, by);
        const int nz = D == 3 ? distinct_blocks(2 * z, -2, 3, nf, v.bc, 2, bz) : 1;
        uint8_t a[27];
        int j = 0;
        for (int kz = 0; kz < 3; ++kz)
            for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                    a[j] = (kx < nx && ky < ny && kz < nz)
                               ? v.nact[F2.boff + bx[kx] + (int64_t)F2.nb * (by[ky] + (int64_t)F2.nb * bz[kz])]
                               : 0;
                    ++j;
                }
        int hit = 0;
        for (int i = 0; i < 27; ++i) hit |= a[i];
        if (hit) return true;
    }
    return false;
}

// ----------------------------------------------------------------------------
// flags of level lvl + tiling into patches of level lvl+1: one workgroup per
// aligned pmax block of level lvl+1 (Morton index = blockIdx.x).  The
// workgroup flags the block's coarse footprint, counts flags per BS-block in
// LDS, and lane 0 takes the recursive split decisions in the order of a
// depth-first recursion over children (x fastest).
// ----------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_flag_tile(View v, int lvl)
{
    if (v.meta->done) return;
    constexpr int MAXSUB = D == 2 ? 64 : 512;       // (pmax / BS)^D, pmax <= 64
    __shared__ int cnt8[MAXSUB];
    __shared__ uint8_t emit8[MAXSUB];
    __shared__ int wsum[4];
    const Grid G = v.grids[lvl];
    const Grid F = v.grids[lvl + 1];
    const int R = v.pmax / BS;
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
    for (int s = threadIdx.x; s < nsub; s += blockDim.x) {
        cnt8[s] = 0;
        emit8[s] = 0;
    }
    __syncthreads();
    const int hp = v.pmax / 2;
    const int nfoot = D == 2 ? hp * hp : hp * hp * hp;
    int mine = 0;
    for (int k = threadIdx.x; k < nfoot; k += blockDim.x) {
        const int lx = k % hp, ly = (k / hp) % hp, lz = D == 3 ? k / (hp * hp) : 0;
        const int x = bp[0] * hp + lx, y = bp[1] * hp + ly, z = D == 3 ? bp[2] * hp + lz : 0;
        const bool fl = refine_flag<D>(v, G, lvl, x, y, z);
        v.flag[G.coff + gidx(G.n, x, y, z)] = fl ? 1 : 0;
        if (fl) {
            atomicAdd(&cnt8[(lx >> 2) + R * ((ly >> 2) + R * (lz >> 2))], 1);
            ++mine;
        }
    }
    for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wsum[w];
        const int64_t slot = v.pbase[lvl + 1] + m;
        v.fcnt[slot] = tot;
        int *out = v.pslot + slot * (int64_t)nsub * 5;
        int np = 0;
        // flagged parents inside the block of es^D BS-blocks at (ex, ey, ez)
        auto count = [&](int ex, int ey, int ez, int es) {
            int c = 0;
            const int ezs = D == 3 ? es : 1;
            for (int zz = 0; zz < ezs; ++zz)
                for (int yy = 0; yy < es; ++yy)
                    for (int xx = 0; xx < es; ++xx) c += cnt8[(ex + xx) + R * ((ey + yy) + R * (ez + zz))];
            return c;
        };
        // 0: empty, 1: emitted as a patch, 2: to be split
        auto decide = [&](int ex, int ey, int ez, int es) {
            const int c = count(ex, ey, ez, es);
            if (c == 0) return 0;
            const int S = es * BS, hsz = S / 2;
            const long long cells = D == 2 ? (long long)hsz * hsz : (long long)hsz * hsz * hsz;
            if (S == v.pmin || (double)c >= v.eta * (double)cells) {
                out[5 * np + 0] = lvl + 1;
                out[5 * np + 1] = bp[0] * v.pmax + ex * BS;
                out[5 * np + 2] = bp[1] * v.pmax + ey * BS;
                out[5 * np + 3] = D == 3 ? bp[2] * v.pmax + ez * BS : 0;
                out[5 * np + 4] = S;
                ++np;
                const int ezs = D == 3 ? es : 1;
                for (int zz = 0; zz < ezs; ++zz)
                    for (int yy = 0; yy < es; ++yy)
                        for (int xx = 0; xx < es; ++xx) emit8[(ex + xx) + R * ((ey + yy) + R * (ez + zz))] = 1;
                return 1;
            }
            return 2;
        };
        constexpr int NC = 1 << D;
        // depth-first over the split levels (R <= 8: at most four levels),
        // children in x-fastest order
        if (decide(0, 0, 0, R) == 2) {
            const int h1 = R / 2;
            for (int k1 = 0; k1 < NC; ++k1) {
                const int x1 = h1 * (k1 & 1), y1 = h1 * ((k1 >> 1) & 1), z1 = h1 * ((k1 >> 2) & 1);
                if (decide(x1, y1, z1, h1) != 2) continue;
                const int h2 = h1 / 2;
                for (int k2 = 0; k2 < NC; ++k2) {
                    const int x2 = x1 + h2 * (k2 & 1), y2 = y1 + h2 * ((k2 >> 1) & 1), z2 = z1 + h2 * ((k2 >> 2) & 1);
                    if (decide(x2, y2, z2, h2) != 2) continue;
                    const int h3 = h2 / 2;
                    for (int k3 = 0; k3 < NC; ++k3)
                        decide(x2 + h3 * (k3 & 1), y2 + h3 * ((k3 >> 1) & 1), z2 + h3 * ((k3 >> 2) & 1), h3);
                }
            }
        }
        v.pcnt[slot] = np;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nsub; s += blockDim.x) {
        const int sx = s % R, sy = (s / R) % R, sz = D == 3 ? s / (R * R) : 0;
        const int bx = bp[0] * R + sx, by = bp[1] * R + sy, bz = D == 3 ? bp[2] * R + sz : 0;
        v.nact[F.boff + bx + (int64_t)F.nb * (by + (int64_t)F.nb * bz)] = emit8[s];
    }
}

// ----------------------------------------------------------------------------
// work lists of the new hierarchy
// ----------------------------------------------------------------------------
// Per-block classification (one thread per block of every level):
//   bit 0 leaf  (in a patch, not every child block in a finer patch)
//   bit 1 cov   (in a patch, some child block in a finer patch)
//   bit 2 ghost (level >= 1, in no patch, a neighbouring block in one)
//   bit 3 fresh (level >= 1, in a patch now but not before)
//   bits 4-7    number of child blocks in finer patches
// then the block's current patch membership becomes the new one.
template <int D>
__global__ void __launch_bounds__(256) k_classify(View v, int64_t nbt)
{
    __shared__ unsigned long long part[MAXLEV][NPART];
    if (v.meta->done) return;
    if (threadIdx.x < MAXLEV * NPART) part[threadIdx.x / NPART][threadIdx.x % NPART] = 0ull;
    __syncthreads();
    constexpr int cpb = D == 2 ? BS * BS : BS * BS * BS;
    constexpr int cpc = cpb >> D;   // cells of a coarse block covered by one child block
    for (int64_t gb = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gb < nbt;
         gb += (int64_t)gridDim.x * blockDim.x) {
        int lvl = 0;
        while (lvl + 1 < v.L && gb >= v.grids[lvl + 1].boff) ++lvl;
        const Grid &G = v.grids[lvl];
        const int nb = G.nb;
        const int b = (int)(gb - G.boff);
        const int bx = b % nb, by = (b / nb) % nb, bz = D == 3 ? b / (nb * nb) : 0;
        const bool a = v.nact[gb] != 0;
        const bool old = v.act[gb] != 0;
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
        bool ghost = false;
        if (!a && lvl >= 1) {
            const int r3 = D == 3 ? 1 : 0;
            uint8_t nbv[27];
            int j = 0;
            for (int dz = -r3; dz <= r3; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int qx = bcmap(bx + dx, nb, v.bc), qy = bcmap(by + dy, nb, v.bc);
                        const int qz = D == 3 ? bcmap(bz + dz, nb, v.bc) : 0;
                        nbv[j++] = v.nact[G.boff + qx + (int64_t)nb * (qy + (int64_t)nb * qz)];
                    }
            int hit = 0;
            for (int i = 0; i < j; ++i) hit |= nbv[i];
            ghost = hit != 0;
        }
        int code = 0;
        if (a && nchild < nch_all) code |= 1;
        if (a && nchild > 0) code |= 2;
        if (ghost) code |= 4;
        if (a && !old && lvl >= 1) code |= 8;
        code |= nchild << 4;
        v.code[gb] = (uint8_t)code;
        v.act[gb] = a ? 1 : 0;
        if (a) {
            atomicAdd(&part[lvl][0], (unsigned long long)(cpb - nchild * cpc));
            atomicAdd(&part[lvl][1], (unsigned long long)cpb);
            atomicAdd(&part[lvl][6], 1ull);
        }
        if (code & 1) atomicAdd(&part[lvl][4], 1ull);
        if (code & 2) atomicAdd(&part[lvl][2], 1ull);
        if (code & 4) atomicAdd(&part[lvl][5], 1ull);
        if (code & 8) atomicAdd(&part[lvl][3], 1ull);
    }
    __syncthreads();
    if (threadIdx.x < MAXLEV * NPART)
        v.cpart[(int64_t)blockIdx.x * MAXLEV * NPART + threadIdx.x] =
            (long long)part[threadIdx.x / NPART][threadIdx.x % NPART];
}

constexpr int LT = 1024;
constexpr int NW = LT / 64;

// One workgroup: compaction of the classified blocks into the leaf, covered,
// ghost and new-block lists (order: level, then block index, x fastest),
// per-level counts, and the patch table (levels in order, pmax blocks in
// Morton order, each block's patches in split order).
template <int D>
__global__ void __launch_bounds__(LT) k_compact(View v, int64_t nbt, int64_t nslot, int nsub)
{
    constexpr int PER = 4;                 // blocks per thread per chunk
    constexpr int NL = 5;                  // leaf, covered, ghost, new, patch blocks
    __shared__ int wcnt[NL][NW];
    __shared__ int base[NL];
    __shared__ int64_t lstart[MAXLEV + 1];
    if (v.meta->done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < NL) base[tid] = 0;
    if (tid <= MAXLEV) lstart[tid] = tid < v.L ? v.grids[tid].boff : nbt;
    // per-level totals of the classification partials and of the flagged
    // cells (integer sums: the result does not depend on the order)
    __shared__ unsigned long long lsum[MAXLEV][NPART];
    __shared__ int nfl[MAXLEV];
    if (tid < MAXLEV * NPART) lsum[tid / NPART][tid % NPART] = 0ull;
    if (tid < MAXLEV) nfl[tid] = 0;
    __syncthreads();
    for (int i = tid; i < v.ncls * v.L * NPART; i += LT) {
        const int w = i / (v.L * NPART), r = i % (v.L * NPART);
        const long long p = v.cpart[((int64_t)w * MAXLEV + r / NPART) * NPART + r % NPART];
        if (p) atomicAdd(&lsum[r / NPART][r % NPART], (unsigned long long)p);
    }
    for (int64_t s = tid; s < nslot; s += LT) {
        const int f = v.fcnt[s];
        if (f) {
            int l = 1;
            while (l + 1 < v.L && s >= v.pbase[l + 1]) ++l;
            atomicAdd(&nfl[l - 1], f);
        }
    }
    __syncthreads();
    if (tid < MAXLEV) {
        const bool in = tid < v.L;
        v.meta->leaf_cells[tid] = in ? (long long)lsum[tid][0] : 0;
        v.meta->act_cells[tid] = in ? (long long)lsum[tid][1] : 0;
        v.meta->cov_cnt[tid] = in ? (int)lsum[tid][2] : 0;
        v.meta->new_cnt[tid] = in ? (int)lsum[tid][3] : 0;
        v.meta->leaf_cnt[tid] = in ? (int)lsum[tid][4] : 0;
        v.meta->ghost_cnt[tid] = in ? (int)lsum[tid][5] : 0;
        v.meta->act_cnt[tid] = in ? (int)lsum[tid][6] : 0;
        v.meta->nflag[tid] = in ? nfl[tid] : 0;
    }
    __syncthreads();
    Tile *lists[NL] = {v.leaf, v.cov, v.ghost, v.fresh, v.actv};
    for (int64_t c0 = 0; c0 < nbt; c0 += (int64_t)LT * PER) {
        const int64_t g0 = c0 + (int64_t)tid * PER;
        int codes[PER], lv[PER];
        int cnt[NL] = {0, 0, 0, 0, 0};
        for (int j = 0; j < PER; ++j) {
            const int64_t gb = g0 + j;
            codes[j] = 0;
            lv[j] = 0;
            if (gb < nbt) {
                int code = v.code[gb] & 15;
                if (code & 3) code |= 16;  // bit 4: in a patch
                int lvl = 0;
                while (gb >= lstart[lvl + 1]) ++lvl;
                codes[j] = code;
                lv[j] = lvl;
                for (int k = 0; k < NL; ++k) cnt[k] += (code >> k) & 1;
            }
        }
    // exclusive scan of the per-thread counts (wave scan + wave totals)
        int excl[NL];
        for (int k = 0; k < NL; ++k) {
            int incl = cnt[k];
            for (int o = 1; o < 64; o <<= 1) {
                const int r = __shfl_up(incl, o);
                if (lane >= o) incl += r;
            }
            excl[k] = incl - cnt[k];
            if (lane == 63) wcnt[k][wave] = incl;
        }
        __syncthreads();
        for (int k = 0; k < NL; ++k) {
            int off = base[k] + excl[k];
            for (int w = 0; w < wave; ++w) off += wcnt[k][w];
            for (int j = 0; j < PER; ++j)
                if ((codes[j] >> k) & 1) {
                    const int64_t gb = g0 + j;
                    lists[k][off++] = Tile{lv[j], (int)(gb - lstart[lv[j]])};
                }
        }
        __syncthreads();
        if (tid < NL) {
            int s = 0;
            for (int w = 0; w < NW; ++w) s += wcnt[tid][w];
            base[tid] += s;
        }
        __syncthreads();
    }
    if (tid == 0) {
        v.meta->nleaf = base[0];
        v.meta->nghost = base[2];
        int co = 0, no = 0, lo = 0, go = 0, ao = 0;
        for (int l = 0; l < MAXLEV; ++l) {
            v.meta->cov_off[l] = co; co += v.meta->cov_cnt[l];
            v.meta->new_off[l] = no; no += v.meta->new_cnt[l];
            v.meta->leaf_off[l] = lo; lo += v.meta->leaf_cnt[l];
            v.meta->ghost_off[l] = go; go += v.meta->ghost_cnt[l];
            v.meta->act_off[l] = ao; ao += v.meta->act_cnt[l];
        }
    }
    // patch table
    __syncthreads();
    if (tid == 0) base[0] = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nslot; c0 += LT) {
        const int64_t s = c0 + tid;
        const int k = s < nslot ? v.pcnt[s] : 0;
        int incl = k;
        for (int o = 1; o < 64; o <<= 1) {
            const int r = __shfl_up(incl, o);
            if (lane >= o) incl += r;
        }
        if (lane == 63) wcnt[0][wave] = incl;
        __syncthreads();
        int off = base[0] + incl - k;
        for (int w = 0; w < wave; ++w) off += wcnt[0][w];
        for (int j = 0; j < k; ++j) {
            if (off + j < v.max_patch)
                for (int e = 0; e < 5; ++e)
                    v.patches[5 * (int64_t)(off + j) + e] = v.pslot[(s * nsub + j) * 5 + e];
        }
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            for (int w = 0; w < NW; ++w) t += wcnt[0][w];
            base[0] += t;
        }
        __syncthreads();
    }
    if (tid == 0) v.meta->npatch = base[0];
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

void launch_flag_tile(const View &v, int lvl, int nblocks, hipStream_t s)
{
    if (v.dim == 2) k_flag_tile<2><<<nblocks, 256, 0, s>>>(v, lvl);
    else k_flag_tile<3><<<nblocks, 256, 0, s>>>(v, lvl);
}

void launch_build_lists(const View &v, int64_t nbt, hipStream_t s)
{
    const int R = v.pmax / BS;
    const int nsub = v.dim == 2 ? R * R : R * R * R;
    if (v.dim == 2) {
        k_classify<2><<<v.ncls, 256, 0, s>>>(v, nbt);
        k_compact<2><<<1, LT, 0, s>>>(v, nbt, v.nslot, nsub);
    } else {
        k_classify<3><<<v.ncls, 256, 0, s>>>(v, nbt);
        k_compact<3><<<1, LT, 0, s>>>(v, nbt, v.nslot, nsub);
    }
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
