// eu_internal.hpp -- data structures shared by the host library and the
// gfx950 kernels.  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eu {

constexpr int BS = 8;          // block side in cells: the unit of patches and tiles
constexpr int MAXLEV = 10;
constexpr int NPART = 2;       // classification partial sums per level
// CFL slots: row l < MAXLEV holds, in each of CFL_NSLOT slots, the largest
// signal speed on level l over the workgroups that add into that slot
// (workgroup b into slot b mod CFL_NSLOT, atomic max of the FP64 bits, which
// order like the non-negative speeds); row MAXLEV the count of leaf cells
// advanced (atomic add).  Each slot has a 128-byte line of its own: atomics
// on one line serialise.  The slots start at zero and their reader clears
// them.
constexpr int CFL_STRIDE = MAXLEV + 1;   // rows
constexpr int CFL_NSLOT = 64;            // slots per row
constexpr int CFL_LINE = 16;             // 8-byte words per slot (one 128-byte line)
constexpr int CFL_MAXBLK = 2048;         // workgroups of the CFL reduction (at most)
__host__ __device__ constexpr int cfl_slot(int row, int slot) { return (row * CFL_NSLOT + slot) * CFL_LINE; }

// One dense grid: a level of the hierarchy, the single uniform grid, or one
// instance of a batch.  Field f of cell (x, y, z) lives at
//   state[off + f * ncell + x + n * (y + n * z)].
struct Grid {
    int64_t off;     // element offset of field 0 in every state array
    int64_t ncell;   // n^d (field stride)
    int64_t boff;    // offset of this grid's blocks in the block-mask arrays
    int64_t coff;    // offset of this grid's cells in the per-cell MR arrays (-1: none)
    int n;           // cells per side
    int nb;          // blocks per side (n / BS)
    int fine;        // grid index of the next finer level (-1: none)
    int coarse;      // grid index of the next coarser level (-1: none)
    int lvl;         // level (0 for uniform and batch grids)
    int pad;
    double dx;       // cell width
    int64_t rcoff;   // local time stepping: coarse-side flux registers of this level (-1: none)
    int64_t rfoff;   // local time stepping: fine-side flux registers of this level (-1: none)
};

// A tile of work: one BS^d block of one grid.  In the ghost list the grid
// field also carries the block's neighbour mask (Tile::GRID_BITS up).
struct Tile {
    static constexpr int GRID_BITS = 4;   // grid index < 16 in the ghost list (levels)
    int grid;
    int block;       // block index within the grid, x fastest
};

// Work item of the strip kernels (grids of one level): the 64 columns xb ..
// xb+63 of grid `grid`.  2D: rows y0 .. y0+ny-1, one wave.  3D: output
// rows y0 .. y0+ny-1 of planes z0 .. z0+nz-1, one workgroup.
struct Strip {
    int grid, xb, y0, ny, z0, nz;
};

// Device-resident counters written by the mesh kernels.
struct Meta {
    int nleaf;                 // tiles in the leaf list (blocks holding leaves)
    int nghost;                // tiles in the ghost list
    int status;                // bit 0: non-physical state met; bit 1 (value 2): a bounded
                               // wait between workgroups timed out
    int done;                  // the current step starts at t >= t_end: skip it
    int steps;                 // steps taken since initialisation
    long long leaf_updates;    // leaf cells advanced since initialisation
    // work lists by level: level l of list k occupies entries
    // [loff[k][l], loff[k][l+1]); loff[k][l] for l >= L is the list length
    int loff[5][MAXLEV + 1];
};

// work lists (index k of Meta::loff)
enum { LST_LEAF = 0, LST_COV = 1, LST_GHOST = 2, LST_NEW = 3, LST_ACT = 4 };

enum { MODE_HIER = 0, MODE_BATCH = 1 };

// Everything a kernel needs, passed by value.
struct View {
    int dim, nv, L, ngrid, bc, mode;
    int lts;                          // local time stepping (recursive level cycle)
    int pmin, pmax;
    double gamma, cfl, t_end, eps, eta;
    int crit;                         // refinement criterion: 0 MR details, 1 scaled gradients
    double eps_p;                     // gradient criterion: pressure threshold (<= 0: none)
    double eps_lv[MAXLEV];            // MR criterion: threshold of the details of each level
    int rk;                           // MR scheme: 0 midpoint rule, 1 Heun
    int ausm_cs;                      // AUSM+ interface sound speed: 0 mean, 1 critical
    int tiler;                        // 0 block split, 1 Berger-Rigoutsos clustering
    int cfl_max;                      // CFL signal speed: 0 sum_d (|v_d| + c), 1 max_d (|v_d| + c)
    const Grid *grids;                // device copy of the grid table
    Grid gt[MAXLEV];                  // the first MAXLEV grids (every level of a hierarchy), by
                                      // value: kernels read them with their arguments
    void *Q, *Qs, *Qo;                // state arrays (element type per precision)
    uint8_t *act, *nact;              // per-block patch membership (current / new)
    uint8_t *sig, *flag;              // per-cell significance and refinement flags
    uint8_t *code;                    // per-block classification of the new hierarchy
    uint32_t *gmask;                  // per ghost block: which of its 3^D neighbour blocks are
                                      // in a patch (bit (dx+1) + 3 (dy+1) [+ 9 (dz+1) in 3D])
    double *D;                        // per-cell FP64 detail norm
    Tile *leaf, *cov, *ghost, *fresh; // work lists
    Tile *actv;                       // every block in a patch, by level
    void *reg;                        // local time stepping flux registers (state type)
    int *pslot;                       // per pmax-block patch rows (7 ints each)
    int *pcnt;                        // per pmax-block patch counts
    int *fcnt;                        // per pmax-block flagged-cell counts
    long long *cpart;                 // per classification workgroup and level (NPART values):
                                      // leaf cells, patch cells
    int ncls;                         // workgroups of the classification kernel
    int lists2;                       // build the lists with two kernels (ranges past the
                                      // single launch's LDS, or forced for tests)
    int nbt;                          // blocks of every grid (list capacity)
    int *wcnt;                        // per classification workgroup: entries of each list
    unsigned long long *lword;        // per classification workgroup: its list counts with an
                                      // epoch, two words (single-launch list build)
    unsigned long long *fword;        // per pmax-block slot: the new patch mask of its blocks
                                      // with an epoch (single-launch flagging)
    int flags1;                       // flag the levels with one launch each (forced for tests)
    int64_t *pbase;                   // per-level offset into pslot / pcnt
    int64_t pb[MAXLEV + 1];           // the same offsets, by value
    Meta *meta;
    unsigned long long *smax;         // per grid: max wave-speed sum (FP64 bits)
    double *dt, *t;                   // per grid (batch) or entry 0 (hierarchy)
    double *t0;                       // time at the start of the step the CFL reduction committed
    double t_rem;                     // the CFL step is also clipped to this (INFINITY: no clip)
    int wait_spin;                    // bound of the waits between workgroups (polls)
    int wait_stale;                   // tests: the list build waits for an epoch no workgroup
                                      // publishes, so its bounded waits give up
    double *partial;                  // per tile x nv partial totals
    unsigned long long *cfls;         // CFL slots (cfl_slot())
    double *totals;                   // per group x nv
    const int *grp_off, *grp_cnt;     // batch: tile range of each instance
    int64_t nslot;                    // pmax blocks of levels 1 .. L-1
    int max_tiles;                    // capacity of the leaf list
};

}  // namespace eu
