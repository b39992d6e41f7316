// eu_mesh.hip -- precision-independent kernels: refinement flags with buffer
// and nesting closure fused with the patch tiling (efficiency rule), work-list
// construction (classification and compaction over contiguous block ranges),
// fills, totals.  Built with -ffp-contract=off.
#include "eu_kernels.hpp"

namespace eu {

// ----------------------------------------------------------------------------
// flags of level lvl + tiling into patches of level lvl+1: one workgroup per
// aligned pmax block of level lvl+1 (Morton index = blockIdx.x).  The
// workgroup flags the block's coarse footprint, counts flags per BS-block in
// LDS, sums them over the nodes of the split tree, and every lane decides for
// one BS-block which node of the recursive split (Sec. 2.2) holds it; patches
// come out in the order of a depth-first recursion over children (x fastest).
// ----------------------------------------------------------------------------
// The grids a flagging launch reads, at fixed offsets of its argument block
// (a read of View::gt at a level-dependent offset would be one more
// dependent read).
struct FlagArgs {
    Grid G, F, C, F2;   // levels lvl, lvl+1, lvl-1 (when lvl >= 1), lvl+2 (when lvl+2 < L)
    int64_t slot0;      // first pmax-block slot of level lvl+1
};

// Every flagged level of a regrid in one launch: the workgroups of level L-2
// come first, then those of L-3, ..., 0 (wg0[k] is the first workgroup of
// level L-2-k).  Level lvl needs the new patch masks of level lvl+2, which
// the workgroups of level lvl+1 decide: each publishes the masks of its
// pmax block (one bit per BS-block, Morton order) in a word of its slot,
// above a 16-bit epoch one higher than the previous regrid's, and the
// workgroups of level lvl read the masks from those words once they carry
// the new epoch.  Only lower-numbered workgroups are waited for, and the
// wait is bounded: past the bound the workgroup sets status flag 2 and goes
// on (it still publishes, so every word keeps one epoch).
struct FlagChain {
    int wg0[MAXLEV];
    int nseg;
    int nflag;      // flagging workgroups; with lists, the list build follows them
    int lists;      // the launch also builds the work lists (v.ncls workgroups)
    int64_t nbt;    // blocks of every level
};

// The list build of workgroup w of W (defined with the list kernels below);
// WORDS: the new patch masks come from the flagging words of this launch.
template <int D, bool WORDS, int R>
__device__ void lists_body(const View &v, int64_t nbt, int w, int W);

// Word and bit of the new patch mask of block (bx, by, bz) of level l >= 1
// (grid G): the word of its pmax block (Morton order within the level), the
// bit of its Morton code within that block.
template <int D, int R>
__device__ __forceinline__ const unsigned long long *flag_word(const View &v, const Grid &G, int l, int bx, int by,
                                                               int bz, int &bit)
{
    constexpr int K = R == 1 ? 0 : R == 2 ? 1 : R == 4 ? 2 : 3;
    const int nbp = G.nb / R;
    int bits = 0;
    while ((1 << bits) < nbp) ++bits;
    const int b[3] = {bx, by, bz};
    int pm = 0;
    bit = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int hi = b[d] / R, lo = b[d] % R;
        for (int k = 0; k < bits; ++k) pm |= ((hi >> k) & 1) << (k * D + d);
#pragma unroll
        for (int k = 0; k < K; ++k) bit |= ((lo >> k) & 1) << (k * D + d);
    }
    int64_t s0 = 0;
#pragma unroll
    for (int k = 1; k < MAXLEV; ++k)
        if (k == l) s0 = v.pb[k];
    return v.fword + s0 + pm;
}

// Offset of level k of the split tree in the node-count array: the nodes of
// levels 0 .. k-1, (R >> j)^D of them each.
template <int D, int R>
__host__ __device__ constexpr int tree_offset(int k)
{
    int o = 0;
    for (int j = 0; j < k; ++j) o += D == 2 ? (R >> j) * (R >> j) : (R >> j) * (R >> j) * (R >> j);
    return o;
}

// Bit masks over the R^D blocks of a pmax block, bit s for the block at
// s = x + R (y + R z) (R^D <= 64): bits [lo u, (hi+1) u), and a bit at every
// multiple of stride, count of them.
__device__ __forceinline__ unsigned long long br_field(int lo, int hi, int u)
{
    const int top = (hi + 1) * u;
    return (top >= 64 ? ~0ull : (1ull << top) - 1ull) & ~((1ull << (lo * u)) - 1ull);
}
__host__ __device__ constexpr unsigned long long br_rep(int stride, int count)
{
    unsigned long long m = 0;
    for (int k = 0; k < count; ++k) m |= 1ull << (k * stride);
    return m;
}

// Berger-Rigoutsos clustering of one pmax block (the AMR method's patch
// generation, Sec. 2.2; Berger and Rigoutsos 1991) on the grid of its R^D
// blocks of BS^D cells, the smallest patches; a block's weight is the count
// of flagged cells among its (BS/2)^D parents.  A box of blocks (inclusive
// bounds) is
//   shrunk to its weighted blocks (none: dropped);
//   a patch when its weighted fraction of parent cells reaches eta, or when
//   it is one block;
//   else cut just above the zero of its signature (the weight per slice)
//   nearest the middle (ties: the lower slice), the axes taken longest
//   first (ties: x, y, z); else between slices i and i+1 where the second
//   difference of the signature changes sign, the largest jump of it over
//   all axes (ties: the axis order, then nearest the middle, then the lower
//   i); else halved along the longest axis, the lower half the smaller;
// and the lower part is clustered before the upper one.
//
// The weights are held as bit planes of 64-bit masks (W[b]: the blocks
// whose weight has bit b; M: the blocks with weight), so a box is a mask
// and every weight over a box or a slice is a sum of popcounts.  The
// outcome for a box depends on the box alone; br_decide computes it, packed:
// bits 0-17 the shrunk box (lo x, y, z, hi x, y, z, 3 bits each), 18-19
// the cut axis, 20-22 the last slice of the lower part, bit 23 a patch,
// bit 24 empty.
constexpr int BR_AX = 18, BR_AT = 20, BR_EMIT = 1 << 23, BR_EMPTY = 1 << 24;

template <int D, int R>
__device__ __forceinline__ int br_decide(int lo0, int lo1, int lo2, int hi0, int hi1, int hi2,
                                         const unsigned long long *W, unsigned long long M, double eta)
{
    constexpr int NSUB = D == 2 ? R * R : R * R * R;
    constexpr int q = BS / 2;
    constexpr int WB = D == 2 ? 5 : 7;   // bits of a weight (at most q^D = 16 or 64)
    constexpr unsigned long long X0 = br_rep(R, NSUB / R);            // slice x = 0
    constexpr unsigned long long Y0 = D == 2 ? br_rep(1, R) : br_rep(1, R) * br_rep(R * R, R);   // y = 0
    constexpr unsigned long long Z0 = br_rep(1, R * R);               // z = 0 (3D)
    auto slice = [&](int a, int i) { return a == 0 ? X0 << i : a == 1 ? Y0 << (R * i) : Z0 << (R * R * i); };
    auto weight = [&](unsigned long long m) {
        int t = 0;
#pragma unroll
        for (int bit = 0; bit < WB; ++bit) t += __popcll(W[bit] & m) << bit;
        return t;
    };
    unsigned long long m = (br_field(lo0, hi0, 1) * br_rep(R, NSUB / R)) &
                           br_field(lo1, hi1, R) * (D == 2 ? 1ull : br_rep(R * R, R));
    if (D == 3) m &= br_field(lo2, hi2, R * R);
    m &= M;
    if (m == 0) return BR_EMPTY;
    // shrink to the weighted blocks
    int occ0 = 0, occ1 = 0, occ2 = D == 3 ? 0 : 1;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        occ0 |= (m & (X0 << i)) ? 1 << i : 0;
        occ1 |= (m & (Y0 << (R * i))) ? 1 << i : 0;
        if (D == 3) occ2 |= (m & (Z0 << (R * R * i))) ? 1 << i : 0;
    }
    lo0 = __builtin_ctz(occ0);
    hi0 = 31 - __builtin_clz(occ0);
    lo1 = __builtin_ctz(occ1);
    hi1 = 31 - __builtin_clz(occ1);
    lo2 = __builtin_ctz(occ2);
    hi2 = 31 - __builtin_clz(occ2);
    const int shrunk = lo0 | lo1 << 3 | lo2 << 6 | hi0 << 9 | hi1 << 12 | hi2 << 15;
    const int tot = weight(m);   // every weighted block of the box lies in the shrunk one
    int64_t cells = (int64_t)(hi0 - lo0 + 1) * q * ((hi1 - lo1 + 1) * q);
    if (D == 3) cells *= (int64_t)(hi2 - lo2 + 1) * q;
    const bool single = lo0 == hi0 && lo1 == hi1 && lo2 == hi2;
    if (single || (double)tot >= eta * (double)cells) return shrunk | BR_EMIT;
    auto lo_of = [&](int a) { return a == 0 ? lo0 : a == 1 ? lo1 : lo2; };
    auto hi_of = [&](int a) { return a == 0 ? hi0 : a == 1 ? hi1 : hi2; };
    auto occ_of = [&](int a) { return a == 0 ? occ0 : a == 1 ? occ1 : occ2; };
    // axes, longest first (ties: the lower axis)
    int ax0 = 0, ax1 = 1, ax2 = 2;
    auto longer = [&](int a, int b) {
        const int la = hi_of(a) - lo_of(a), lb = hi_of(b) - lo_of(b);
        return lb > la || (lb == la && b < a);
    };
    if (longer(ax0, ax1)) { const int t = ax0; ax0 = ax1; ax1 = t; }
    if (D == 3) {
        if (longer(ax0, ax2)) { const int t = ax0; ax0 = ax2; ax2 = t; }
        if (longer(ax1, ax2)) { const int t = ax1; ax1 = ax2; ax2 = t; }
    }
    auto axis = [&](int k) { return k == 0 ? ax0 : k == 1 ? ax1 : ax2; };
    int cut_axis = -1, cut_at = 0;
    // a zero of the signature: an unoccupied slice inside the box
    for (int k = 0; k < D && cut_axis < 0; ++k) {
        const int a = axis(k), la = lo_of(a), ha = hi_of(a), f = occ_of(a);
        int best = -1, bd = 0;
        for (int i = la + 1; i <= ha - 1; ++i)
            if (!((f >> i) & 1)) {
                const int dd = abs(2 * i - (la + ha));
                if (best < 0 || dd < bd) {
                    best = i;
                    bd = dd;
                }
            }
        if (best >= 0) {
            cut_axis = a;
            cut_at = best;
        }
    }
    if (cut_axis < 0) {
        // the strongest inflection of the signatures (each slice's weight
        // taken once; the slices indexed by unrolled constants)
        int bs = 0, bdist = 0;
        for (int k = 0; k < D; ++k) {
            const int a = axis(k), la = lo_of(a), ha = hi_of(a);
            int sg[R];
#pragma unroll
            for (int i = 0; i < R; ++i) sg[i] = i >= la && i <= ha ? weight(m & slice(a, i)) : 0;
#pragma unroll
            for (int i = 1; i + 2 < R; ++i) {
                if (i < la + 1 || i + 1 > ha - 1) continue;
                const int d0 = sg[i - 1] - 2 * sg[i] + sg[i + 1], d1 = sg[i] - 2 * sg[i + 1] + sg[i + 2];
                if (!((d0 < 0 && d1 > 0) || (d0 > 0 && d1 < 0))) continue;
                const int st = abs(d0 - d1), dist = abs(2 * i + 1 - (la + ha));
                if (cut_axis < 0 || st > bs || (st == bs && a == cut_axis && dist < bdist)) {
                    cut_axis = a;
                    cut_at = i;
                    bs = st;
                    bdist = dist;
                }
            }
        }
    }
    if (cut_axis < 0) {
        cut_axis = ax0;
        cut_at = lo_of(ax0) + (hi_of(ax0) - lo_of(ax0) + 1) / 2 - 1;
    }
    return shrunk | cut_axis << BR_AX | cut_at << BR_AT;
}

// Boxes of an R^D grid of blocks numbered by their intervals: interval
// (lo, hi) of an axis is number lo R - lo (lo - 1) / 2 + hi - lo of NI =
// R (R + 1) / 2, the box is x + NI (y + NI z).
template <int D, int R>
struct BrBoxes {
    static constexpr int NI = R * (R + 1) / 2;
    static constexpr int N = D == 2 ? NI * NI : NI * NI * NI;
    static __device__ __forceinline__ int interval(int lo, int hi) { return lo * R - lo * (lo - 1) / 2 + hi - lo; }
    static __device__ __forceinline__ void bounds(int iv, int &lo, int &hi)
    {
        lo = 0;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (iv >= R - lo) {
                iv -= R - lo;
                ++lo;
            }
        hi = lo + iv;
    }
};

// R = pmax / BS (1, 2, 4 or 8): every size below is a compile-time constant,
// so the loops unroll and no index needs a runtime division.
template <int D, int R, bool CHAIN>
__global__ void __launch_bounds__(256) k_flag_tile(View v, int lvl_arg, FlagArgs fa, FlagChain fc)
{
    if constexpr (CHAIN) {
        if (fc.lists && (int)blockIdx.x >= fc.nflag) {
            lists_body<D, true, R>(v, fc.nbt, (int)blockIdx.x - fc.nflag, v.ncls);
            return;
        }
    }
    constexpr int NT = 256;                          // threads (the launch uses 256)
    constexpr int NSUB = D == 2 ? R * R : R * R * R;  // BS-blocks of the pmax block
    constexpr int K = R == 1 ? 0 : R == 2 ? 1 : R == 4 ? 2 : 3;   // levels of the split tree below the root
    constexpr int HP = 4 * R;                        // footprint side (level-lvl cells)
    constexpr int HE = HP + 2;                       // with a one-cell halo
    constexpr int NRAW = D == 2 ? HE * HE : HE * HE * HE;
    constexpr int NFOOT = D == 2 ? HP * HP : HP * HP * HP;
    // level-(lvl+1) cells 2x-2 .. 2x+3 of the footprint's x lie in virtual
    // level-(lvl+2) blocks (2x-2)>>2 .. (2x+3)>>2: NVB of them per axis
    constexpr int NVB = ((2 * (HP - 1) + 3) >> 2) - ((-2) >> 2) + 1;
    constexpr int NNEST = D == 2 ? NVB * NVB : NVB * NVB * NVB;
    __shared__ int cnt8[NSUB];
    __shared__ uint8_t emit8[NSUB];
    __shared__ int wsum[NT / 64];
    // LDS staging of what the flags of the footprint read: the raw flags
    // (significant detail of the cell or of its parent) over the footprint
    // and a one-cell halo, and the new patch masks of level lvl+2 over the
    // blocks the nesting test reaches (virtual block indices; the boundary
    // map is applied when staging: clamping or wrapping a block index is the
    // same as mapping the cells and dividing)
    __shared__ uint8_t sraw[NRAW];
    __shared__ uint8_t snest[NNEST];
    static_assert(!CHAIN || NSUB <= 48, "a pmax block's masks share a word with the epoch");
    const int done = v.meta->done;
    // level and pmax block of this workgroup
    int lvl = lvl_arg, m = blockIdx.x;
    int64_t slot0 = fa.slot0, slot2 = 0;
    Grid G = fa.G, F = fa.F, Cg = fa.C, F2 = fa.F2;
    if constexpr (CHAIN) {
        int seg = 0, first = 0;
#pragma unroll
        for (int k = 1; k < MAXLEV; ++k)
            if (k < fc.nseg && (int)blockIdx.x >= fc.wg0[k]) {
                seg = k;
                first = fc.wg0[k];
            }
        lvl = v.L - 2 - seg;
        m = blockIdx.x - first;
        G = grid_lane(v, lvl);
        F = grid_lane(v, lvl + 1);
        Cg = grid_lane(v, lvl >= 1 ? lvl - 1 : lvl);
        F2 = grid_lane(v, lvl + 2 < v.L ? lvl + 2 : lvl);
#pragma unroll
        for (int k = 1; k <= MAXLEV; ++k) {
            if (k == lvl + 1) slot0 = v.pb[k];
            if (k == lvl + 2) slot2 = v.pb[k];
        }
    }
    const bool hasc = lvl >= 1, nest = lvl + 2 < v.L;
    const int64_t slot = slot0 + m;
    // this regrid's epoch (the words of a chain keep one epoch)
    const unsigned long long ep =
        CHAIN ? ((__hip_atomic_load(v.fword + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 0xffffull) + 1) & 0xffffull
              : 0ull;
    int bp[3] = {0, 0, 0};
    {
        const int nbp = F.n / (R * BS);
        int bits = 0;
        while ((1 << bits) < nbp) ++bits;
        for (int k = 0; k < bits; ++k)
            for (int d = 0; d < D; ++d) bp[d] |= ((m >> (k * D + d)) & 1) << k;
    }
    const int n = G.n;
    const int o0[3] = {bp[0] * HP, bp[1] * HP, D == 3 ? bp[2] * HP : 0};
    int vb0[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) vb0[d] = (2 * o0[d] - 2) >> 2;
    // every staging read issued before the first LDS store (in chunks of
    // eight per thread when there are more); addresses are clamped to valid
    // ones so that no read waits behind a test (the grids of levels lvl-1
    // and lvl+2 stand in for missing levels with valid ones)
    // (a chain stages the nesting masks later, from the words)
    constexpr int IR = (NRAW + NT - 1) / NT, IN = CHAIN ? 0 : (NNEST + NT - 1) / NT, CH = 8;
    const int nb2 = F2.nb;
#pragma unroll
    for (int c0 = 0; c0 < IR + IN; c0 += CH) {
        uint8_t val[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int it = c0 + u;
            val[u] = 0;
            if (it < IR) {
                const int i0 = threadIdx.x + it * NT, i = i0 < NRAW ? i0 : NRAW - 1;
                const int ex = i % HE, ey = (i / HE) % HE, ez = D == 3 ? i / (HE * HE) : 0;
                const int qx = bcmap(o0[0] - 1 + ex, n, v.bc), qy = bcmap(o0[1] - 1 + ey, n, v.bc);
                const int qz = D == 3 ? bcmap(o0[2] - 1 + ez, n, v.bc) : 0;
                const uint8_t a = v.sig[G.coff + gidx(n, qx, qy, qz)];
                const uint8_t b = v.sig[Cg.coff + gidx(Cg.n, qx >> 1, qy >> 1, qz >> 1)];
                // preventive refinement (MR criterion): the parent's significance
                val[u] = a | (hasc && v.crit == 0 ? b : 0);
            } else if (it < IR + IN) {
                const int i0 = threadIdx.x + (it - IR) * NT, i = i0 < NNEST ? i0 : NNEST - 1;
                int b[3] = {i % NVB, (i / NVB) % NVB, D == 3 ? i / (NVB * NVB) : 0};
                for (int d = 0; d < D; ++d) {
                    const int q = vb0[d] + b[d];
                    b[d] = v.bc == 1 ? (q < 0 ? q + nb2 : q >= nb2 ? q - nb2 : q) : (q < 0 ? 0 : q >= nb2 ? nb2 - 1 : q);
                }
                val[u] = v.nact[F2.boff + b[0] + (int64_t)nb2 * (b[1] + (int64_t)nb2 * b[2])];
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int it = c0 + u;
            if (it < IR) {
                const int i = threadIdx.x + it * NT;
                if (i < NRAW) sraw[i] = val[u];
            } else if (it < IR + IN) {
                const int i = threadIdx.x + (it - IR) * NT;
                if (i < NNEST) snest[i] = val[u];
            }
        }
    }
    if (done) return;
    for (int s = threadIdx.x; s < NSUB; s += NT) {
        cnt8[s] = 0;
        emit8[s] = 0;
    }
    __syncthreads();
    // flag of each footprint cell: raw flags dilated by one cell, or the
    // nesting closure (a level-(lvl+1) cell within two cells of the new level
    // lvl+2)
    int mine = 0;   // flagged cells of this wave (ballot counts, lane-uniform)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NIT = (NFOOT + NT - 1) / NT;
    // raw flags of footprint cell k dilated by one cell
    auto dilated = [&](int k) {
        const int lx = k % HP, ly = (k / HP) % HP, lz = D == 3 ? (k / (HP * HP)) % HP : 0;
        int any = 0;
#pragma unroll
        for (int dz = (D == 3 ? 0 : 1); dz <= (D == 3 ? 2 : 1); ++dz)
#pragma unroll
            for (int dy = 0; dy <= 2; ++dy)
#pragma unroll
                for (int dx = 0; dx <= 2; ++dx)
                    any |= sraw[(lx + dx) + HE * ((ly + dy) + (D == 3 ? HE * (lz + dz) : 0))];
        return any;
    };
    // a chain dilates while the finer level's masks are on their way
    int anyv[CHAIN ? NIT : 1];
    if constexpr (CHAIN) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) anyv[it] = dilated(threadIdx.x + it * NT);
        // the new patch masks of level lvl+2 from the words of the level-(lvl+1)
        // workgroups that decided them: one word per virtual block
        if (nest) {
            const int nbp2 = nb2 / R;
            int bits2 = 0;
            while ((1 << bits2) < nbp2) ++bits2;
            int late = 0;
            for (int i = threadIdx.x; i < NNEST; i += NT) {
                int b[3] = {i % NVB, (i / NVB) % NVB, D == 3 ? i / (NVB * NVB) : 0};
                int pm = 0, bit = 0;
                for (int d = 0; d < D; ++d) {
                    const int q = vb0[d] + b[d];
                    const int bb = v.bc == 1 ? (q < 0 ? q + nb2 : q >= nb2 ? q - nb2 : q) : (q < 0 ? 0 : q >= nb2 ? nb2 - 1 : q);
                    const int hi = bb / R, lo = bb % R;
                    for (int k = 0; k < bits2; ++k) pm |= ((hi >> k) & 1) << (k * D + d);
#pragma unroll
                    for (int k = 0; k < K; ++k) bit |= ((lo >> k) & 1) << (k * D + d);
                }
                const unsigned long long *wp = v.fword + slot2 + pm;
                unsigned long long x = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int spin = 0; (x & 0xffffull) != ep; ++spin) {
                    if (spin >= v.wait_spin) {
                        late = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    x = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                snest[i] = (uint8_t)((x >> (16 + bit)) & 1ull);
            }
            if (late) atomicOr(&v.meta->status, 2);
        }
        __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int k = threadIdx.x + it * NT;
        const bool in = k < NFOOT;
        const int lx = k % HP, ly = (k / HP) % HP, lz = D == 3 ? (k / (HP * HP)) % HP : 0;
        int any;
        if constexpr (CHAIN) any = anyv[it];
        else any = dilated(k);
        if (nest && !any) {
            const int c[3] = {o0[0] + lx, o0[1] + ly, o0[2] + lz};
            // level-(lvl+1) cells 2c-2 .. 2c+3 lie in virtual level-(lvl+2)
            // blocks (2c-2)>>2 .. (2c+3)>>2: always two per axis
            int lo[3];
            for (int d = 0; d < 3; ++d) lo[d] = d < D ? ((2 * c[d] - 2) >> 2) - vb0[d] : 0;
#pragma unroll
            for (int bz = 0; bz < (D == 3 ? 2 : 1); ++bz)
#pragma unroll
                for (int by = 0; by < 2; ++by)
#pragma unroll
                    for (int bx = 0; bx < 2; ++bx) any |= snest[(lo[0] + bx) + NVB * ((lo[1] + by) + NVB * (lo[2] + bz))];
        }
        const bool fl = in && any != 0;
        if (in) v.flag[G.coff + gidx(n, o0[0] + lx, o0[1] + ly, o0[2] + lz)] = fl ? 1 : 0;
        const unsigned long long bal = __ballot(fl);
        mine += __popcll(bal);
        if constexpr (D == 2 && R == 4) {
            // a wave holds four footprint rows of 16 cells: sub-blocks
            // (lane mod 16) / 4 = j, whole; lane j counts sub-block j
            const int sy = (it * NT + wave * 64) / (4 * HP);
            if (lane < 4) cnt8[lane + R * sy] = __popcll(bal & (0x000F000F000F000Full << (4 * lane)));
        } else {
            if (fl) atomicAdd(&cnt8[(lx >> 2) + R * ((ly >> 2) + R * (lz >> 2))], 1);
        }
    }
    if (lane == 0) wsum[wave] = mine;
    // Each sub-block, taken in Morton order (the order in which a depth-first
    // recursion over children, x fastest, meets it), walks from the root to
    // the node that is emitted as a patch (or is empty).  The node's first
    // sub-block writes the patch; patches are ranked by that Morton order.
    // The walk stops at the first node, from the top, that is empty (then
    // every node below it is) or meets the split rule: the emitted node is
    // the highest nonempty node that meets it, found from the flagged-cell
    // counts cn[k] of the sub-block's nodes (k = 0: the sub-block).
    auto emit_level = [&](const int *cn) {
        int emit_k = -1;
#pragma unroll
        for (int k = 0; k <= K; ++k) {
            const int S = BS << k, hsz = S / 2;
            const long long cells = D == 2 ? (long long)hsz * hsz : (long long)hsz * hsz * hsz;
            if (cn[k] > 0 && (S == v.pmin || (double)cn[k] >= v.eta * (double)cells)) emit_k = k;
        }
        return emit_k;
    };
    auto morton_split = [](int mc, int &sx, int &sy, int &sz) {
        sx = sy = sz = 0;
#pragma unroll
        for (int b = 0; b < K; ++b) {
            sx |= ((mc >> (b * D)) & 1) << b;
            sy |= ((mc >> (b * D + 1)) & 1) << b;
            if (D == 3) sz |= ((mc >> (b * D + 2)) & 1) << b;
        }
    };
    int *out = v.pslot + slot * (int64_t)NSUB * 7;
    // a square patch of side S at block (sx, sy, sz) as row pos
    auto put_row = [&](int pos, int sx, int sy, int sz, int S) {
        out[7 * pos + 0] = lvl + 1;
        out[7 * pos + 1] = bp[0] * R * BS + sx * BS;
        out[7 * pos + 2] = bp[1] * R * BS + sy * BS;
        out[7 * pos + 3] = D == 3 ? bp[2] * R * BS + sz * BS : 0;
        out[7 * pos + 4] = S;
        out[7 * pos + 5] = S;
        out[7 * pos + 6] = D == 3 ? S : 1;
    };
    if constexpr (NSUB <= 64) {
        __syncthreads();
        // clustering, in parallel (thread = box; a thread takes KB boxes
        // where the R^D grid has more boxes than the workgroup threads):
        // the weight planes (every wave takes the same ballots), every box's
        // outcome, then the patch count of the clustering below every box
        // (bottom-up, one pass per level of the tree: a box's height is at
        // most D (R - 1)), then the position of every box the depth-first
        // walk meets (top-down from the whole block: a cut box's lower part
        // at its own position, its upper part after the lower part's
        // patches); the boxes met that are patches write their rows
        using BB = BrBoxes<D, R>;
        constexpr int KB = (BB::N + NT - 1) / NT;
        constexpr int BR_PASSES = D * (R - 1);
        constexpr int BR_ROOT = (R - 1) + BB::NI * ((R - 1) + BB::NI * (D == 3 ? R - 1 : 0));
        __shared__ int scnt[2][BB::N], spos[BB::N];
        __shared__ unsigned long long smember;
        __shared__ int snp;
        if (v.tiler == 1) {
            unsigned long long Wp[D == 2 ? 5 : 7], Mp;
            const int wlin = lane < NSUB ? cnt8[lane] : 0;
#pragma unroll
            for (int bit = 0; bit < (D == 2 ? 5 : 7); ++bit) Wp[bit] = __ballot((wlin >> bit) & 1);
            Mp = __ballot(wlin > 0);
            int d[KB], cl[KB], cu[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int b = threadIdx.x + k * NT;
                d[k] = BR_EMPTY;
                cl[k] = cu[k] = 0;
                if (b < BB::N) {
                    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                    BB::bounds(b % BB::NI, lo[0], hi[0]);
                    BB::bounds((b / BB::NI) % BB::NI, lo[1], hi[1]);
                    if (D == 3) BB::bounds(b / (BB::NI * BB::NI), lo[2], hi[2]);
                    d[k] = br_decide<D, R>(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], Wp, Mp, v.eta);
                    if (!(d[k] & (BR_EMPTY | BR_EMIT))) {
                        // the two parts of the cut
                        const int a = (d[k] >> BR_AX) & 3, at = (d[k] >> BR_AT) & 7;
                        const int slo[3] = {d[k] & 7, (d[k] >> 3) & 7, (d[k] >> 6) & 7};
                        const int shi[3] = {(d[k] >> 9) & 7, (d[k] >> 12) & 7, (d[k] >> 15) & 7};
                        int il[3], iu[3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            il[j] = BB::interval(slo[j], j == a ? at : shi[j]);
                            iu[j] = BB::interval(j == a ? at + 1 : slo[j], shi[j]);
                        }
                        cl[k] = il[0] + BB::NI * (il[1] + BB::NI * (D == 3 ? il[2] : 0));
                        cu[k] = iu[0] + BB::NI * (iu[1] + BB::NI * (D == 3 ? iu[2] : 0));
                    }
                    scnt[0][b] = (d[k] & BR_EMIT) ? 1 : 0;
                    spos[b] = b == BR_ROOT ? 0 : -1;
                }
            }
            auto is_cut = [&](int k) { return !(d[k] & (BR_EMPTY | BR_EMIT)); };
            if (threadIdx.x == 0) smember = 0ull;
            __syncthreads();
#pragma unroll
            for (int p = 0; p < BR_PASSES; ++p) {
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int b = threadIdx.x + k * NT;
                    if (b < BB::N)
                        scnt[(p + 1) & 1][b] = is_cut(k) ? scnt[p & 1][cl[k]] + scnt[p & 1][cu[k]] : scnt[p & 1][b];
                }
                __syncthreads();
            }
            const int *cnt = scnt[BR_PASSES & 1];
#pragma unroll
            for (int p = 0; p < BR_PASSES; ++p) {
                int at[KB];
#pragma unroll
                for (int k = 0; k < KB; ++k) {
                    const int b = threadIdx.x + k * NT;
                    at[k] = b < BB::N ? spos[b] : -1;
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    if (is_cut(k) && at[k] >= 0) {
                        spos[cl[k]] = at[k];
                        spos[cu[k]] = at[k] + cnt[cl[k]];
                    }
                __syncthreads();
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int b = threadIdx.x + k * NT;
                if (b < BB::N && (d[k] & BR_EMIT) && spos[b] >= 0) {
                    const int pos = spos[b], dk = d[k];
                    const int lo0 = dk & 7, lo1 = (dk >> 3) & 7, lo2 = (dk >> 6) & 7;
                    const int hi0 = (dk >> 9) & 7, hi1 = (dk >> 12) & 7, hi2 = (dk >> 15) & 7;
                    out[7 * pos + 0] = lvl + 1;
                    out[7 * pos + 1] = (bp[0] * R + lo0) * BS;
                    out[7 * pos + 2] = (bp[1] * R + lo1) * BS;
                    out[7 * pos + 3] = D == 3 ? (bp[2] * R + lo2) * BS : 0;
                    out[7 * pos + 4] = (hi0 - lo0 + 1) * BS;
                    out[7 * pos + 5] = (hi1 - lo1 + 1) * BS;
                    out[7 * pos + 6] = D == 3 ? (hi2 - lo2 + 1) * BS : 1;
                    unsigned long long bm = (br_field(lo0, hi0, 1) * br_rep(R, NSUB / R)) &
                                            br_field(lo1, hi1, R) * (D == 2 ? 1ull : br_rep(R * R, R));
                    if (D == 3) bm &= br_field(lo2, hi2, R * R);
                    atomicOr(&smember, bm);
                }
            }
            if (threadIdx.x == 0) snp = cnt[BR_ROOT];
            __syncthreads();
        }
        // the block tiler: one wave walks, lane = Morton code, so the
        // sub-blocks of a node of level k are an aligned group of 2^(D k)
        // lanes and its count is a sum over the group
        if (wave == 0) {
            const int mc = lane;
            int sx, sy, sz;
            morton_split(mc, sx, sy, sz);
            bool inp;
            int npatch;
            if (v.tiler == 1) {
                npatch = snp;
                inp = mc < NSUB && ((smember >> (sx + R * (sy + R * sz))) & 1ull);
            } else {
                int cn[K + 1];
                cn[0] = mc < NSUB ? cnt8[sx + R * (sy + R * sz)] : 0;
#pragma unroll
                for (int k = 1; k <= K; ++k) {
                    int t = cn[k - 1];
#pragma unroll
                    for (int o = 1 << (D * (k - 1)); o < (1 << (D * k)); o <<= 1) t += __shfl_xor(t, o);
                    cn[k] = t;
                }
                const int emit_k = mc < NSUB ? emit_level(cn) : -1;
                const int em = (1 << (emit_k < 0 ? 0 : emit_k)) - 1;
                const bool lead = emit_k >= 0 && (sx & em) == 0 && (sy & em) == 0 && (sz & em) == 0;
                const unsigned long long mask = __ballot(lead);
                const int pos = __popcll(mask & (lane ? (~0ull >> (64 - lane)) : 0ull));
                if (lead) put_row(pos, sx, sy, sz, BS << emit_k);
                inp = emit_k >= 0;
                npatch = __popcll(mask);
            }
            if (mc < NSUB) emit8[sx + R * (sy + R * sz)] = inp ? 1 : 0;
            if constexpr (CHAIN) {
                // publish the masks (bit = Morton code) for the next coarser level
                const unsigned long long pub = __ballot(inp && mc < NSUB);
                if (lane == 0)
                    __hip_atomic_store(v.fword + slot, ep | pub << 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (lane == 0) {
                int tot = 0;
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) tot += wsum[w];
                v.fcnt[slot] = tot;
                v.pcnt[slot] = npatch;
            }
        }
        __syncthreads();
    } else {
        // node counts in LDS: level k holds the nodes of 2^k BS-blocks per
        // side, (R >> k)^D of them
        __shared__ int ncnt[tree_offset<D, R>(K + 1)];
        __shared__ int wlead[NT / 64];
        __syncthreads();
        for (int s = threadIdx.x; s < NSUB; s += NT) ncnt[s] = cnt8[s];
#pragma unroll
        for (int k = 1; k <= K; ++k) {
            __syncthreads();
            const int r = R >> k, rc = R >> (k - 1);
            const int nn = D == 2 ? r * r : r * r * r;
            const int o1 = tree_offset<D, R>(k - 1), o2 = tree_offset<D, R>(k);
            for (int i = threadIdx.x; i < nn; i += NT) {
                const int ix = i % r, iy = (i / r) % r, iz = D == 3 ? i / (r * r) : 0;
                int c = 0;
#pragma unroll
                for (int ch = 0; ch < (1 << D); ++ch)
                    c += ncnt[o1 + (2 * ix + (ch & 1)) + rc * ((2 * iy + ((ch >> 1) & 1)) + rc * (2 * iz + ((ch >> 2) & 1)))];
                ncnt[o2 + i] = c;
            }
        }
        __syncthreads();
        int nlead_total = 0;
#pragma unroll
        for (int c0 = 0; c0 < NSUB; c0 += NT) {
            const int mc = c0 + threadIdx.x;   // Morton code of this lane's sub-block
            int sx, sy, sz;
            morton_split(mc, sx, sy, sz);
            int emit_k = -1;
            if (mc < NSUB) {
                int cn[K + 1];
#pragma unroll
                for (int k = 0; k <= K; ++k) {
                    const int r = R >> k;
                    cn[k] = ncnt[tree_offset<D, R>(k) + (sx >> k) + r * ((sy >> k) + r * (sz >> k))];
                }
                emit_k = emit_level(cn);
            }
            const int em = (1 << (emit_k < 0 ? 0 : emit_k)) - 1;
            const bool lead = emit_k >= 0 && (sx & em) == 0 && (sy & em) == 0 && (sz & em) == 0;
            if (mc < NSUB) emit8[sx + R * (sy + R * sz)] = emit_k >= 0 ? 1 : 0;
            const unsigned long long mask = __ballot(lead);
            if (lane == 0) wlead[wave] = __popcll(mask);
            __syncthreads();
            int pos = nlead_total + __popcll(mask & (lane ? (~0ull >> (64 - lane)) : 0ull));
            for (int w = 0; w < wave; ++w) pos += wlead[w];
            if (lead) put_row(pos, sx, sy, sz, BS << emit_k);
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) nlead_total += wlead[w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            int tot = 0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) tot += wsum[w];
            v.fcnt[slot] = tot;
            v.pcnt[slot] = nlead_total;
        }
    }
    for (int s = threadIdx.x; s < NSUB; s += NT) {
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
// Classification of block gb (the blocks of every level numbered
// consecutively): code and ghost mask (written, with the new patch
// membership); false when the step is done (nothing written).  The new
// masks come from the mask array, or (WORDS) from the flagging words of
// the same launch once they carry epoch ep (a bounded wait: past the bound
// late is set).  Level 0 is always in a patch.
template <int D, bool WORDS, int R>
__device__ __forceinline__ bool classify_block(const View &v, int64_t gb, int done, unsigned long long ep, int &late,
                                               int &code, uint32_t &gm, int &lvl, int &nchild)
{
    lvl = 0;
    for (int k = 1; k < MAXLEV && k < v.L; ++k) lvl += gb >= v.gt[k].boff ? 1 : 0;
    const Grid G = grid_lane(v, lvl);
    const int nb = G.nb;
    const int b = (int)(gb - G.boff);
    const int bx = b % nb, by = (b / nb) % nb, bz = D == 3 ? b / (nb * nb) : 0;
    constexpr int NN = D == 3 ? 27 : 9, NC = D == 3 ? 8 : 4;
    const int r3 = D == 3 ? 1 : 0;
    const bool hasf = lvl + 1 < v.L;
    const Grid F = grid_lane(v, hasf ? lvl + 1 : lvl);
    uint8_t na, oa, ch[8] = {0, 0, 0, 0, 0, 0, 0, 0}, nbv[27];
    // every mask read (the block, its children, its neighbours) is issued
    // before any is tested
    oa = v.act[gb];
    if constexpr (!WORDS) {
        na = v.nact[gb];
        if (hasf) {
            for (int i = 0; i < NC; ++i) {
                const int x = i & 1, y = (i >> 1) & 1, z = i >> 2;
                ch[i] = v.nact[F.boff + (2 * bx + x) + (int64_t)F.nb * ((2 * by + y) + (int64_t)F.nb * (2 * bz + z))];
            }
        }
        int j = 0;
        for (int dz = -r3; dz <= r3; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int qx = bcmap(bx + dx, nb, v.bc), qy = bcmap(by + dy, nb, v.bc);
                    const int qz = D == 3 ? bcmap(bz + dz, nb, v.bc) : 0;
                    nbv[j++] = lvl >= 1 ? v.nact[G.boff + qx + (int64_t)nb * (qy + (int64_t)nb * qz)] : 0;
                }
        issued((int)na, (int)oa, (int)nbv[0]);
        if (done) return false;   // read with the masks above: one round trip for both
    } else {
        // neighbours (the block itself in the middle) on level lvl >= 1,
        // children on level lvl+1; unused words read at a valid address
        const unsigned long long *pn[NN], *pc[NC];
        int bn[NN], bcb[NC];
        unsigned long long xn[NN], xc[NC];
        int j = 0;
        for (int dz = -r3; dz <= r3; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int qx = bcmap(bx + dx, nb, v.bc), qy = bcmap(by + dy, nb, v.bc);
                    const int qz = D == 3 ? bcmap(bz + dz, nb, v.bc) : 0;
                    pn[j] = lvl >= 1 ? flag_word<D, R>(v, G, lvl, qx, qy, qz, bn[j]) : v.fword;
                    if (lvl < 1) bn[j] = 0;
                    xn[j] = __hip_atomic_load(pn[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ++j;
                }
        for (int i = 0; i < NC; ++i) {
            const int x = i & 1, y = (i >> 1) & 1, z = i >> 2;
            pc[i] = hasf ? flag_word<D, R>(v, F, lvl + 1, 2 * bx + x, 2 * by + y, 2 * bz + z, bcb[i]) : v.fword;
            if (!hasf) bcb[i] = 0;
            xc[i] = __hip_atomic_load(pc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        issued((int)oa, (int)xn[0], (int)xc[0]);
        if (done) return false;   // nothing was flagged: no word is raised
        // every round reads again all the words not yet raised, together
        for (int spin = 0;; ++spin) {
            bool ok = true;
#pragma unroll
            for (int i = 0; i < NN; ++i) ok = ok && (lvl < 1 || (xn[i] & 0xffffull) == ep);
#pragma unroll
            for (int i = 0; i < NC; ++i) ok = ok && (!hasf || (xc[i] & 0xffffull) == ep);
            if (ok) break;
            if (spin >= v.wait_spin) {
                late = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int i = 0; i < NN; ++i)
                if (lvl >= 1 && (xn[i] & 0xffffull) != ep)
                    xn[i] = __hip_atomic_load(pn[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (hasf && (xc[i] & 0xffffull) != ep)
                    xc[i] = __hip_atomic_load(pc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int i = 0; i < NN; ++i) nbv[i] = lvl >= 1 ? (uint8_t)((xn[i] >> (16 + bn[i])) & 1ull) : 0;
        for (int i = 0; i < NC; ++i) ch[i] = hasf ? (uint8_t)((xc[i] >> (16 + bcb[i])) & 1ull) : 0;
        na = lvl >= 1 ? nbv[NN / 2] : 1;
        if (lvl < 1) for (int i = 0; i < NN; ++i) nbv[i] = 0;
    }
    const int j = NN;
    const bool a = na != 0;
    const bool old = oa != 0;
    nchild = 0;
    if (a)
        for (int i = 0; i < 8; ++i) nchild += ch[i];
    const int nch_all = D == 2 ? 4 : 8;
    bool ghost = false;
    gm = 0;
    if (!a) {
        for (int i = 0; i < j; ++i) gm |= (nbv[i] ? 1u : 0u) << i;
        ghost = gm != 0;
    }
    code = 0;
    if (a && nchild < nch_all) code |= 1;
    if (a && nchild > 0) code |= 2;
    if (ghost) code |= 4;
    if (a && !old && lvl >= 1) code |= 8;
    code |= nchild << 4;
    v.code[gb] = (uint8_t)code;
    v.gmask[gb] = gm;
    v.act[gb] = a ? 1 : 0;
    return true;
}

// Cells per level (leaf, patch) and entries per list of one classified block.
template <int D>
__device__ __forceinline__ void count_block(unsigned long long (*part)[NPART], int *lcnt, int lvl, int code,
                                            int nchild)
{
    constexpr int cpb = D == 2 ? BS * BS : BS * BS * BS;
    constexpr int cpc = cpb >> D;   // cells of a coarse block covered by one child block
    if (code & 3) {
        atomicAdd(&part[lvl][0], (unsigned long long)(cpb - nchild * cpc));
        atomicAdd(&part[lvl][1], (unsigned long long)cpb);
    }
    // entries in the leaf, covered, ghost, new, patch lists
    if (code & 1) atomicAdd(&lcnt[0], 1);
    if (code & 2) atomicAdd(&lcnt[1], 1);
    if (code & 4) atomicAdd(&lcnt[2], 1);
    if (code & 8) atomicAdd(&lcnt[3], 1);
    if (code & 3) atomicAdd(&lcnt[4], 1);
}

template <int D>
__global__ void __launch_bounds__(256) k_classify(View v, int64_t nbt)
{
    __shared__ unsigned long long part[MAXLEV][NPART];
    __shared__ int lcnt[5];
    const int done = v.meta->done;
    if (threadIdx.x < MAXLEV * NPART) part[threadIdx.x / NPART][threadIdx.x % NPART] = 0ull;
    if (threadIdx.x < 5) lcnt[threadIdx.x] = 0;
    __syncthreads();
    // workgroup w classifies the contiguous range [w chunk, (w+1) chunk)
    const int64_t chunk = (nbt + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = blockIdx.x * chunk, g1 = g0 + chunk < nbt ? g0 + chunk : nbt;
    for (int64_t gb = g0 + threadIdx.x; gb < g1; gb += blockDim.x) {
        int code, lvl, nchild, late = 0;
        uint32_t gm;
        if (!classify_block<D, false, 1>(v, gb, done, 0ull, late, code, gm, lvl, nchild)) break;
        count_block<D>(part, lcnt, lvl, code, nchild);
    }
    if (done) return;
    __syncthreads();
    if (threadIdx.x < 5) v.wcnt[(int64_t)blockIdx.x * 5 + threadIdx.x] = lcnt[threadIdx.x];
    if (threadIdx.x < MAXLEV * NPART)
        v.cpart[(int64_t)blockIdx.x * MAXLEV * NPART + threadIdx.x] =
            (long long)part[threadIdx.x / NPART][threadIdx.x % NPART];
}

// Sum over the workgroup of each thread's list counts acc[] into base[].
__device__ __forceinline__ void workgroup_sum5(int *acc, int (*wsum)[5], int *base)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = 0; k < 5; ++k)
        for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
    if (lane == 0)
        for (int k = 0; k < 5; ++k) wsum[wave][k] = acc[k];
    __syncthreads();
    if (tid < 5) {
        int s = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += wsum[i][tid];
        base[tid] = s;
    }
    __syncthreads();
}

// Entries of blocks g0 .. g1-1 in the leaf, covered, ghost, new and patch
// lists, from base[] on (order: level, then block index, x fastest); the
// thread holding the first block of a level records where that level starts
// in every list.  block(gb, k) gives the code and ghost mask of block gb, the
// k-th of this range.
template <typename F>
__device__ __forceinline__ void write_lists(const View &v, int64_t g0, int64_t g1, int *base,
                                            const int64_t *lstart, F block)
{
    constexpr int NL = 5;
    __shared__ int wc[4][NL];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    Tile *lists[NL] = {v.leaf, v.cov, v.ghost, v.fresh, v.actv};
    for (int64_t c = g0; c < g1; c += blockDim.x) {
        const int64_t gb = c + tid;
        int code = 0, lvl = 0;
        uint32_t gm = 0;
        if (gb < g1) {
            block(gb, gb - g0, code, gm);
            code &= 15;
            if (code & 3) code |= 16;  // bit 4: in a patch
            for (int k = 1; k < MAXLEV && k < v.L; ++k) lvl += gb >= v.gt[k].boff ? 1 : 0;
        }
        int pre[NL];
        for (int k = 0; k < NL; ++k) {
            const unsigned long long mask = __ballot((code >> k) & 1);
            pre[k] = __popcll(mask & (lane ? (~0ull >> (64 - lane)) : 0ull));
            if (lane == 0) wc[wave][k] = __popcll(mask);
        }
        __syncthreads();
        // every LDS read of the offsets issued at once (at most four waves)
        const int64_t ls = lstart[lvl];
        const bool first = gb < g1 && gb == ls;   // first block of its level
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            int off = base[k] + pre[k];
#pragma unroll
            for (int i = 0; i < 3; ++i) off += i < wave ? wc[i][k] : 0;
            if ((code >> k) & 1)
                lists[k][off] = Tile{k == LST_GHOST ? (int)(lvl | (gm << Tile::GRID_BITS)) : lvl, (int)(gb - ls)};
            if (first) v.meta->loff[k][lvl] = off;
        }
        __syncthreads();
        if (tid < NL) {
            const int nw = (int)(blockDim.x >> 6);
            int s = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) s += i < nw ? wc[i][tid] : 0;
            base[tid] += s;
        }
        __syncthreads();
    }
}

// The last workgroup has seen every entry: the list lengths.
__device__ __forceinline__ void write_list_lengths(const View &v, const int *base)
{
    const int tid = threadIdx.x;
    if (tid < 5)
        for (int l = v.L; l <= MAXLEV; ++l) v.meta->loff[tid][l] = base[tid];
    if (tid == 0) {
        v.meta->nleaf = base[0];
        v.meta->nghost = base[2];
    }
}

// Compaction of the classified blocks into the leaf, covered, ghost, new and
// all-patch lists, with the same contiguous ranges as the classification:
// workgroup w sums the list counts of the ranges before its own and writes
// its entries from there.  (The patch table is read from the per pmax-block
// slots when it is asked for.)
template <int D>
__global__ void __launch_bounds__(256) k_compact(View v, int64_t nbt)
{
    constexpr int NL = 5;                  // leaf, covered, ghost, new, patch blocks
    __shared__ int base[NL];
    __shared__ int wsum[4][NL];
    __shared__ int64_t lstart[MAXLEV + 1];
    const int tid = threadIdx.x;
    const int W = gridDim.x, w = blockIdx.x;
    // first reads, independent of each other: the done flag, the level
    // starts and the list counts of the ranges before this one
    const int done = v.meta->done;
    if (tid <= MAXLEV) lstart[tid] = tid < v.L && tid < MAXLEV ? v.gt[tid].boff : nbt;
    const int64_t chunk = (nbt + W - 1) / W;
    const int64_t g0 = w * chunk, g1 = g0 + chunk < nbt ? g0 + chunk : nbt;
    // codes of the first chunk of this range
    const int code0 = g0 + tid < g1 ? v.code[g0 + tid] : 0;
    const uint32_t gm0 = g0 + tid < g1 ? v.gmask[g0 + tid] : 0u;
    int acc[NL] = {0, 0, 0, 0, 0};
    for (int i = tid; i < w; i += blockDim.x)
        for (int k = 0; k < NL; ++k) acc[k] += v.wcnt[(int64_t)i * 5 + k];
    issued(acc[0], acc[1], acc[2], acc[3], acc[4], code0, gm0);
    if (done) return;
    workgroup_sum5(acc, wsum, base);
    write_lists(v, g0, g1, base, lstart, [&](int64_t gb, int64_t k, int &code, uint32_t &gm) {
        code = k < (int64_t)blockDim.x ? code0 : v.code[gb];
        gm = k < (int64_t)blockDim.x ? gm0 : v.gmask[gb];
    });
    if (w == W - 1) write_list_lengths(v, base);
}

// Classification and compaction in one launch, for ranges of at most
// LISTS_MAXCHUNK blocks (the codes stay in LDS).  Each workgroup classifies
// its range, publishes its list counts as two words that carry an epoch
// one above the previous build's, and adds up the counts of the ranges
// before its own once their words carry the new epoch.  Only lower-numbered
// workgroups are waited for, and the wait is bounded: past the bound the
// workgroup sets status flag 2 and writes no entries.  The words start with
// one epoch (cleared with the hierarchy) and every build that is not done
// raises all of them, so they keep one epoch.
constexpr int LISTS_MAXCHUNK = 1024;

template <int D, bool WORDS, int R>
__device__ void lists_body(const View &v, int64_t nbt, int w, int W)
{
    constexpr int NL = 5;
    __shared__ uint8_t scode[LISTS_MAXCHUNK];
    __shared__ uint32_t sgm[LISTS_MAXCHUNK];
    __shared__ unsigned long long part[MAXLEV][NPART];
    __shared__ int lcnt[NL];
    __shared__ int base[NL];
    __shared__ int wsum[4][NL];
    __shared__ int64_t lstart[MAXLEV + 1];
    __shared__ int late;
    const int tid = threadIdx.x;
    unsigned long long *word = v.lword;
    const int done = v.meta->done;
    const unsigned long long own = __hip_atomic_load(word + 2 * w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid < MAXLEV * NPART) part[tid / NPART][tid % NPART] = 0ull;
    if (tid < NL) lcnt[tid] = 0;
    if (tid <= MAXLEV) lstart[tid] = tid < v.L && tid < MAXLEV ? v.gt[tid].boff : nbt;
    if (tid == 0) late = 0;
    __syncthreads();
    const int64_t chunk = (nbt + W - 1) / W;
    const int64_t g0 = w * chunk, g1 = g0 + chunk < nbt ? g0 + chunk : nbt;
    // the epoch of this launch; with WORDS also that of the flagging words, which
    // are raised with the list words by every such launch (both start at
    // zero with the hierarchy)
    const unsigned long long e = ((own & 0xffffull) + 1) & 0xffffull;
    int mlate = 0;
    for (int64_t gb = g0 + tid; gb < g1; gb += blockDim.x) {
        int code, lvl, nchild;
        uint32_t gm;
        if (!classify_block<D, WORDS, R>(v, gb, done, e, mlate, code, gm, lvl, nchild)) break;
        scode[gb - g0] = (uint8_t)code;
        sgm[gb - g0] = gm;
        count_block<D>(part, lcnt, lvl, code, nchild);
    }
    if (done) return;
    if (mlate) late = 1;
    __syncthreads();
    if (tid == 0) {
        // counts of at most LISTS_MAXCHUNK: 16 bits each
        const unsigned long long c[NL] = {(unsigned long long)lcnt[0], (unsigned long long)lcnt[1],
                                          (unsigned long long)lcnt[2], (unsigned long long)lcnt[3],
                                          (unsigned long long)lcnt[4]};
        __hip_atomic_store(word + 2 * w, e | c[0] << 16 | c[1] << 32 | c[2] << 48, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(word + 2 * w + 1, e | c[3] << 16 | c[4] << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid < MAXLEV * NPART)
        v.cpart[(int64_t)w * MAXLEV * NPART + tid] = (long long)part[tid / NPART][tid % NPART];
    // the counts of the ranges before this one: thread i waits for range i
    // (both of its words read in one trip)
    int acc[NL] = {0, 0, 0, 0, 0};
    // the epoch waited for (a test setting makes it one no workgroup publishes)
    const unsigned long long ew = v.wait_stale ? ((e + 1) & 0xffffull) : e;
    for (int i = tid; i < w; i += blockDim.x) {
        unsigned long long x0 = __hip_atomic_load(word + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long x1 = __hip_atomic_load(word + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int spin = 0; (x0 & 0xffffull) != ew || (x1 & 0xffffull) != ew; ++spin) {
            if (spin >= v.wait_spin) {
                late = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            x0 = __hip_atomic_load(word + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            x1 = __hip_atomic_load(word + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        acc[0] += (int)((x0 >> 16) & 0xffff);
        acc[1] += (int)((x0 >> 32) & 0xffff);
        acc[2] += (int)((x0 >> 48) & 0xffff);
        acc[3] += (int)((x1 >> 16) & 0xffff);
        acc[4] += (int)((x1 >> 32) & 0xffff);
    }
    workgroup_sum5(acc, wsum, base);   // its barriers also publish late
    if (late) {
        if (tid == 0) atomicOr(&v.meta->status, 2);
        return;
    }
    write_lists(v, g0, g1, base, lstart, [&](int64_t, int64_t k, int &code, uint32_t &gm) {
        code = scode[k];
        gm = sgm[k];
    });
    if (w == W - 1) write_list_lengths(v, base);
}

template <int D>
__global__ void __launch_bounds__(256) k_lists(View v, int64_t nbt)
{
    lists_body<D, false, 1>(v, nbt, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------------------
// CFL: time step from the per-workgroup maxima of the reduction kernel
// ----------------------------------------------------------------------------
// dt = min over levels of cfl dx_l / smax_l (hierarchy; with local time
// stepping the level-0 step dt_0 = min over levels (cfl dx_l / smax_l) 2^l
// and dt_l = dt_0 / 2^l) or per instance (batch), clipped to reach t_end.
// A step that starts at t >= t_end is marked done and skipped by every later
// kernel of the step; otherwise the step is committed: t += dt, steps += 1,
// leaf updates counted.  One workgroup.
__global__ void __launch_bounds__(256) k_cfl_final_batch(View v)
{
#pragma clang fp contract(off)
    for (int g = threadIdx.x; g < v.ngrid; g += blockDim.x) {
        const unsigned long long b = atomicExch(&v.smax[g], 0ull);
        const double s = __longlong_as_double((long long)b);
        double dt = b ? (v.cfl * v.grids[g].dx) / s : 0.0;
        const double t = v.t[g];
        if (dt > v.t_end - t) dt = v.t_end - t;
        if (dt > v.t_rem) dt = v.t_rem;
        if (!(dt > 0.0)) dt = 0.0;
        v.dt[g] = dt;
        v.t0[g] = t;
        v.t[g] = t + dt;
    }
    if (threadIdx.x == 0) {
        v.meta->done = 0;
        v.meta->steps += 1;
    }
}

// Hierarchy of NG levels: one wave reads the CFL slots of those levels and
// of the leaf count (lane j slot j), clears them for the next producers,
// and lane 0 turns the maxima into dt and commits the step.
template <int NG>
__global__ void __launch_bounds__(64) k_cfl_final(View v)
{
#pragma clang fp contract(off)
    static_assert(CFL_NSLOT == 64, "one slot per lane");
    const int lane = threadIdx.x;
    // every read in one trip: the time, the step counters (read after the
    // slots are cleared below, which may alias them, they would take a
    // second trip), the level spacings and the slots
    const double t = v.t[0];
    const int steps0 = v.meta->steps;
    const long long upd0 = v.meta->leaf_updates;
    double dx[NG];
#pragma unroll
    for (int l = 0; l < NG; ++l) dx[l] = v.gt[l].dx;
    unsigned long long q[NG + 1];
#pragma unroll
    for (int l = 0; l < NG; ++l) q[l] = v.cfls[cfl_slot(l, lane)];
    q[NG] = v.cfls[cfl_slot(MAXLEV, lane)];
    issued(steps0, upd0);
#pragma unroll
    for (int l = 0; l < NG; ++l) issued(dx[l]);
    double sm[NG];
#pragma unroll
    for (int l = 0; l < NG; ++l) {
        double m = __longlong_as_double((long long)q[l]);
        for (int o = 32; o > 0; o >>= 1) {
            const double r = __shfl_xor(m, o);
            m = r > m ? r : m;
        }
        sm[l] = m;
    }
    unsigned long long cnt = q[NG];
    for (int o = 32; o > 0; o >>= 1) cnt += (unsigned long long)__shfl_xor((long long)cnt, o);
#pragma unroll
    for (int l = 0; l < NG; ++l) v.cfls[cfl_slot(l, lane)] = 0ull;
    v.cfls[cfl_slot(MAXLEV, lane)] = 0ull;
    if (lane != 0) return;
    double dt = __builtin_inf();
#pragma unroll
    for (int l = 0; l < NG; ++l) {
        if (sm[l] > 0.0) {
            double d = (v.cfl * dx[l]) / sm[l];
            if (v.lts) d = d * (double)(1 << l);
            if (d < dt) dt = d;
        }
    }
    const long long upd = (long long)cnt;
    const int done = t < v.t_end && v.t_rem > 0.0 ? 0 : 1;
    if (dt > v.t_end - t) dt = v.t_end - t;
    if (dt > v.t_rem) dt = v.t_rem;
    if (v.lts) {
        double dl = dt;
#pragma unroll
        for (int l = 0; l < NG; ++l) {
            v.dt[l] = dl;
            dl = dl * 0.5;
        }
    } else {
        v.dt[0] = dt;
    }
    v.meta->done = done;
    v.t0[0] = t;
    if (!done) {
        v.t[0] = t + dt;
        v.meta->steps = steps0 + 1;
        v.meta->leaf_updates = upd0 + upd;
    }
}

// The step committed by the last CFL reduction takes the time step dt_ext
// instead (per instance for a batch; a hierarchy's level-0 step, halved per
// level with local time stepping): t = t0 + dt.  One workgroup.
__global__ void __launch_bounds__(256) k_set_dt(View v, const double *dt_ext)
{
#pragma clang fp contract(off)
    if (v.mode != MODE_HIER) {
        for (int g = threadIdx.x; g < v.ngrid; g += blockDim.x) {
            const double dt = dt_ext[g] > 0.0 ? dt_ext[g] : 0.0;
            v.dt[g] = dt;
            v.t[g] = v.t0[g] + dt;
        }
        return;
    }
    if (threadIdx.x != 0) return;
    const double dt = dt_ext[0] > 0.0 ? dt_ext[0] : 0.0;
    if (v.lts) {
        double dl = dt;
        for (int l = 0; l < v.L && l < MAXLEV; ++l) {
            v.dt[l] = dl;
            dl = dl * 0.5;
        }
    } else {
        v.dt[0] = dt;
    }
    if (!v.meta->done) v.t[0] = v.t0[0] + dt;
}

__global__ void k_copy_f64(double *dst, const double *src, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Significance of every detail against the threshold of its level (levels
// 0 .. L-2, the per-cell arrays of the MR analysis): D >= eps_l.
__global__ void k_threshold(View v, int64_t ncell)
{
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ncell; j += (int64_t)gridDim.x * blockDim.x) {
        int k = 0;
        for (int q = 1; q < MAXLEV && q < v.L - 1; ++q) k += j >= v.gt[q].coff ? 1 : 0;
        v.sig[j] = v.D[j] >= v.eps_lv[k] ? 1 : 0;
    }
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
    const FlagChain fc{};
    FlagArgs fa;
    fa.G = v.gt[lvl];
    fa.F = v.gt[lvl + 1];
    fa.C = v.gt[lvl >= 1 ? lvl - 1 : lvl];
    fa.F2 = v.gt[lvl + 2 < v.L ? lvl + 2 : lvl];
    fa.slot0 = v.pb[lvl + 1];
    const int R = v.pmax / BS;
    if (v.dim == 2) {
        switch (R) {
        case 1: k_flag_tile<2, 1, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        case 2: k_flag_tile<2, 2, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        case 4: k_flag_tile<2, 4, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        default: k_flag_tile<2, 8, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        }
    } else {
        switch (R) {
        case 1: k_flag_tile<3, 1, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        case 2: k_flag_tile<3, 2, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        case 4: k_flag_tile<3, 4, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        default: k_flag_tile<3, 8, false><<<nblocks, 256, 0, s>>>(v, lvl, fa, fc); break;
        }
    }
}

bool flag_chain_ok(const View &v)
{
    const int R = v.pmax / BS;
    return v.mode == MODE_HIER && !v.flags1 && v.L >= 3 &&
           ((v.dim == 2 && R <= 4) || (v.dim == 3 && R <= 2));
}

static bool lists_single(const View &v, int64_t nbt)
{
    return !v.lists2 && (nbt + v.ncls - 1) / v.ncls <= LISTS_MAXCHUNK;
}

bool flag_chain_lists(const View &v, int64_t nbt) { return flag_chain_ok(v) && lists_single(v, nbt); }

void launch_flag_chain(const View &v, const int *wg0, int nseg, int nflag, int64_t nbt, bool lists, hipStream_t s)
{
    FlagChain fc{};
    for (int k = 0; k < nseg && k < MAXLEV; ++k) fc.wg0[k] = wg0[k];
    fc.nseg = nseg;
    fc.nflag = nflag;
    fc.lists = lists ? 1 : 0;
    fc.nbt = nbt;
    const int total = nflag + (lists ? v.ncls : 0);
    const FlagArgs fa{};
    const int R = v.pmax / BS;
    if (v.dim == 2) {
        switch (R) {
        case 1: k_flag_tile<2, 1, true><<<total, 256, 0, s>>>(v, 0, fa, fc); break;
        case 2: k_flag_tile<2, 2, true><<<total, 256, 0, s>>>(v, 0, fa, fc); break;
        default: k_flag_tile<2, 4, true><<<total, 256, 0, s>>>(v, 0, fa, fc); break;
        }
    } else {
        switch (R) {
        case 1: k_flag_tile<3, 1, true><<<total, 256, 0, s>>>(v, 0, fa, fc); break;
        default: k_flag_tile<3, 2, true><<<total, 256, 0, s>>>(v, 0, fa, fc); break;
        }
    }
}

void launch_cfl_final(const View &v, hipStream_t s)
{
    if (v.mode != MODE_HIER) {
        k_cfl_final_batch<<<1, 256, 0, s>>>(v);
        return;
    }
    switch (v.ngrid) {
    case 1: k_cfl_final<1><<<1, 64, 0, s>>>(v); break;
    case 2: k_cfl_final<2><<<1, 64, 0, s>>>(v); break;
    case 3: k_cfl_final<3><<<1, 64, 0, s>>>(v); break;
    case 4: k_cfl_final<4><<<1, 64, 0, s>>>(v); break;
    case 5: k_cfl_final<5><<<1, 64, 0, s>>>(v); break;
    case 6: k_cfl_final<6><<<1, 64, 0, s>>>(v); break;
    case 7: k_cfl_final<7><<<1, 64, 0, s>>>(v); break;
    case 8: k_cfl_final<8><<<1, 64, 0, s>>>(v); break;
    case 9: k_cfl_final<9><<<1, 64, 0, s>>>(v); break;
    default: k_cfl_final<MAXLEV><<<1, 64, 0, s>>>(v); break;
    }
}

void launch_build_lists(const View &v, int64_t nbt, hipStream_t s)
{
    if (lists_single(v, nbt)) {
        if (v.dim == 2) k_lists<2><<<v.ncls, 256, 0, s>>>(v, nbt);
        else k_lists<3><<<v.ncls, 256, 0, s>>>(v, nbt);
        return;
    }
    if (v.dim == 2) {
        k_classify<2><<<v.ncls, 256, 0, s>>>(v, nbt);
        k_compact<2><<<v.ncls, 256, 0, s>>>(v, nbt);
    } else {
        k_classify<3><<<v.ncls, 256, 0, s>>>(v, nbt);
        k_compact<3><<<v.ncls, 256, 0, s>>>(v, nbt);
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

void launch_set_dt(const View &v, const double *dt_ext, hipStream_t s) { k_set_dt<<<1, 256, 0, s>>>(v, dt_ext); }

void launch_copy_f64(double *dst, const double *src, int n, hipStream_t s)
{
    k_copy_f64<<<grid_for(n, 64, 4096), 64, 0, s>>>(dst, src, n);
}

void launch_threshold(const View &v, int64_t ncell, hipStream_t s)
{
    k_threshold<<<grid_for(ncell, 256, 4096), 256, 0, s>>>(v, ncell);
}

}  // namespace eu
