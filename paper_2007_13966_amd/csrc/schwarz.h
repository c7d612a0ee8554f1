// Multilevel restricted additive Schwarz preconditioner: level hierarchy,
// overlapping subdomains with ILU(0) factors, interpolation between levels.
#pragma once

#include <memory>

#include "krylov.h"

namespace nks {

// Subdomain (overlapping box Omega_i^delta) of one level, device POD.
struct SubDev {
    int blk;
    int ex, ey, ez;              // extended box extents
    int ox, oy, oz;              // extended box origin in block coordinates
    int lx0, lx1, ly0, ly1, lz0, lz1;   // owned range, extended-box coordinates
    int fac_off;                 // first extended cell in factor / zext storage
    int next;                    // extended cells
    int lvl_off;                 // first entry of this subdomain's level pointers
    int nlev;                    // wavefront levels
    int inv_off;                 // first entry of the padded-tile inverse map
    int gorg;                    // global index of the extended box's origin cell
    int gnx, gny;                // row and column counts of its block (strides of y and z)
};

// Per block box layout of a level (for the AS / right-RAS gather)
struct BlkPart {
    int px, py, pz, first;
};

// 1D interpolation tables of one direction for all blocks (fine -> coarse)
struct Interp1 {
    // fine index row (block-local index + row offset of the block): <= 4 (coarse, w)
    std::vector<int> rcnt, rj;
    std::vector<double> rw;
    // coarse index column: up to cs (fine, w), cs the longest column
    std::vector<int> ccnt, ci;
    std::vector<double> cw;
    int cs = 1;
    std::vector<int> roff, coff;   // per block offsets into rows / cols
    DBuf<int> d_rcnt, d_rj, d_ccnt, d_ci, d_roff, d_coff;
    DBuf<double> d_rw, d_cw;
};

struct Level {
    Space sp;                    // this level's cells (owned here for coarse levels)
    Space *spp = nullptr;        // the space in use (fine level: the grid's)
    Op own;                      // coarse-level operator (Galerkin product)
    Op *A = nullptr;             // operator in use (fine level: the Jacobian)
    Stencil fst;                 // factor stencil: the operator's offsets plus ILU(k) fill
    DBuf<int> amap;              // factor stencil entry -> operator stencil entry (-1: fill)
    int delta = 1;
    int lb = 1, lc = 1;          // wavefront level function t = x + lb*y + lc*z
    int R = 1;                   // padding of the LDS tile (stencil reach)
    int nsub = 0, next_total = 0, lvl_total = 0, inv_total = 0;
    int max_tile = 0;            // largest padded tile (cells)
    int max_next = 0;
    int max_lvl = 0;             // largest hyperplane (cells)
    int max_nlev = 0;            // most hyperplanes of a subdomain
    std::vector<SubDev> hsub;
    DBuf<SubDev> sub;
    std::vector<BlkPart> hpart;
    DBuf<BlkPart> part;
    DBuf<int> lvlptr;            // per subdomain: nlev+1 offsets (relative to fac_off)
    DBuf<int> loc;               // per extended cell (level order): padded-tile index
    DBuf<int> inv;               // per padded-tile cell: level-order index or -1
    DBuf<int> lexi;              // per extended cell (level order): lexicographic ext index
    // ILU(0) factors: K coefficient arrays over the extended cells (level order)
    DBuf<double> w64;            // FP64 factorisation workspace (hyperplane order)
    DBuf<double> f64;            // FP64 factors (FP64 mode)
    DBuf<float> f32;             // FP32 factors (FP32 mode)
    DBuf<uint16_t> f16;          // BF16 factors (BF16 mode)
    DBuf<int> lexg;              // per extended cell (hyperplane order): lexicographic storage slot
    // 2D levels use the register-wavefront sweep: factors stored in
    // lexicographic order, stencil mapped onto a row template
    bool rows2d = false;
    // 3D levels with the 7-point stencil, rows of at most 64 cells and at most
    // four slabs of at most 64 (y, z) rows per box use the 3D row sweep;
    // factors stored in lexicographic order
    bool rows3d = false;
    bool rows3d_multi = false;   // more than 64 (y, z) rows: slabs of z planes, one wavefront each
    int rows3d_slabs = 1;        // most slabs of a box
    std::vector<int> hkmap3;     // 3D sweep: lower (z, y, x) and upper (x, y, z) slots -> stencil index
    int box = 0;                 // 0: 5-point cross, 1: 5x5 box, 2: 21-point (5x5 without corners)
    DBuf<int> slotmap;           // box slot -> stencil index (-1: absent)
    std::vector<int> hslot;      // host copy of slotmap
    DBuf<double> invd64;         // 1/u_ii
    DBuf<float> invd32;
    DBuf<double> zext;           // per extended cell solution (AS / right-RAS gather)
    int form = 0, form_wgs = 0;  // kernel form (NKS_SWEEP_*) and workgroups of the last sweep
    // 2D levels of small boxes: groups of consecutive boxes of one block
    // swept together, their rows packed into one wavefront
    int pk_groups = 0;           // 0: one box per workgroup
    size_t pk_max_n = 0;         // most extended cells of a group
    DBuf<int2> pk_lane;          // per group: 64 lanes of {box, row} (row -1: idle)
    DBuf<int> pk_steps;          // per group: sweep steps of its longest box
    DBuf<int> pk_box;            // per group: first box (groups + 1 entries)
    DBuf<int> pk_e2g;            // per extended cell: cell of the level's space, high bit where owned
    DBuf<int> err;               // zero-pivot flag
    // ILU(0) elimination table of the stencil: for lower offset k, pairs (k2, t)
    // with off[k] + off[k2] = off[t], k2 an upper offset
    DBuf<int> upd_ptr, upd_k2, upd_t;
    int nupd = 0;                // entries of upd_k2 / upd_t
    int max_upd = 0;             // most updates of one lower entry
    DBuf<int> lin_pad;           // padded-tile linear offset of each stencil entry
    // interpolation from the next coarser level to this one
    Interp1 ip[3];
    DBuf<int> rap_slot;          // coarse offset -> slot table for the Galerkin product
    std::unique_ptr<Grid> cg;    // rediscretised coarse levels: this level's upscaled grid
    DBuf<double> cstate;         // and the coarsened state its Jacobian is taken at
    int rap_R = 0;
    // 2D levels: column-wise Galerkin product, windows of at most
    // rap_wx x rap_wy fine cells (0: the general kernel)
    int rap_wx = 0, rap_wy = 0;
    // its tables, fixed by the interpolation: per coarse cell {block, x and y
    // column, J_x | J_y << 16}; per column its window {first cell, width};
    // per column and coarse offset o the weights p(f, column - o) over the
    // window widened by the fine stencil's reach
    DBuf<int4> rap_cell;
    DBuf<int2> rap_win[2];
    DBuf<double> rap_tab[2];
    // work vectors
    DBuf<double> r, t, bc, xc;
};

struct TileDims {
    int PX, PY, PZ, R, Rz;       // padded LDS tile and stencil reach
};

// The coarsest level's GMRES as one persistent launch (a workgroup per
// reservoir): lane groups of packed boxes, index maps between the cells and
// the boxes' extended cells, per-cell factor runs, the Krylov basis.
struct CoarsePersist {
    bool on = false;
    int ncap = 0;                // cells of the largest reservoir on the level
    int max_ne = 0;              // extended cells of the largest reservoir's boxes
    size_t lds = 0;
    DBuf<int> efirst, gfirst, gsteps, ext2loc, own2ext, kmap;
    DBuf<int2> glane;
    DBuf<double> r64;            // per-cell factor runs, in the preconditioner's precision
    DBuf<float> r32;
    DBuf<uint16_t> r16;
    DBuf<double> V, res;
    DBuf<int> its;
};

struct Ras {
    Grid *g = nullptr;
    Matrix *J = nullptr;
    nks_ras_desc d{};
    int L = 1;
    std::vector<std::unique_ptr<Level>> lev;    // lev[0] finest
    std::vector<TileDims> tiles_;
    Gmres coarse;
    int lds_bytes = 65536;
    int n_cu = 1;                // compute units of the device
    // coarse GMRES iterations per captured graph after a first chunk of twice
    // as many (measured on the batch: shorter chunks, or a first chunk sized
    // to the previous solve, cost more in host polls and graph instances
    // than the iterations they save)
    int graph_chunk = 4;
    int coarse_its_last = 0;
    long coarse_its_total = 0;
    long coarse_calls = 0;

    void build(Matrix *J, const nks_ras_desc &d);     // structure (once)
    void factor(bool ilu = true);                      // numeric: Galerkin products, and the
                                                       // subdomain factors when ilu is set
    void apply(const double *r, double *z, const int *mask);
    void apply_level(int l, const double *r, double *z, const int *mask, bool accumulate);
    void vcycle(int l, const double *b, double *x, const int *mask);
    void coarse_solve(const double *b, double *x, const int *mask);
    CoarsePersist cp;
    void setup_persistent();                           // decides cp.on (after build)
    void pack_runs();                                  // per-cell runs of the coarsest factors
    void coarse_persistent(const double *b, double *x, const int *mask);
    // no host round trip inside apply: one level, or the persistent coarse solve
    bool capturable() const { return L == 1 || cp.on; }
    void restrict_to(int l, const double *rf, double *rc, const int *mask);
    void prolong_add(int l, const double *ec, double *zf, const int *mask);
    void check_pivots();
    int *hpiv = nullptr;         // pinned staging for the per-level zero-pivot flags
    ~Ras();
};

}  // namespace nks
