// Internal declarations of libnks (gfx950).  Host structures own device
// buffers; kernels receive plain pointers and small POD descriptors.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nks.h"

namespace nks {

// ------------------------------------------------------------------ errors
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const char *fmt, ...);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPC(x) ::nks::hip_check((x), #x, __FILE__, __LINE__)
#define KCHECK() ::nks::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ------------------------------------------------------------------ allocation
struct Alloc {
    nks_alloc_fn fa = nullptr;
    nks_free_fn ff = nullptr;
    void *ctx = nullptr;
    void *get(size_t bytes);
    void put(void *p);
};

template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    Alloc *al = nullptr;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), al(o.al) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; al = o.al;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (p && al) al->put(p);
        p = nullptr;
        n = 0;
    }
    void alloc(Alloc *a, size_t count) {
        if (p && n >= count && al == a) return;
        release();
        al = a;
        n = count;
        p = count ? static_cast<T *>(a->get(count * sizeof(T))) : nullptr;
    }
    void upload(Alloc *a, const std::vector<T> &h, hipStream_t s) {
        alloc(a, h.size());
        if (!h.empty()) {
            HIPC(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
            HIPC(hipStreamSynchronize(s));   // h may be a temporary
        }
    }
};

// ------------------------------------------------------------------ geometry
// One reservoir ("block") of a level: box dims and first cell.
struct Blk {
    int nx, ny, nz, off;
};

// Reduction chunk: a run of cells inside one block.
struct Chunk {
    int blk, start, end, pad;
};

constexpr int CHUNK = 256;       // minimum cells per reduction chunk
constexpr int MAXCH = 256;       // at most this many chunks per reservoir (one per reduction thread)
constexpr int RED_THREADS = 256;
constexpr int TILE = 256;        // cells per elementwise workgroup
constexpr int MAXB = 4096;       // reservoirs per grid

// Vector space of one level: N cells in B blocks plus its reduction chunks.
struct Space {
    int N = 0, B = 0;
    std::vector<Blk> hblk;
    DBuf<Blk> blk;
    std::vector<Chunk> hchunk;
    DBuf<Chunk> chunk;
    std::vector<int> hcfirst;    // first chunk of each block, B+1 entries
    DBuf<int> cfirst;
    // runs of at most TILE cells inside one block: a workgroup each for the
    // elementwise and stencil kernels (chunks can be much longer)
    std::vector<Chunk> htile;
    DBuf<Chunk> tile;
    void build(Alloc *al, const std::vector<Blk> &b, hipStream_t s);
};

// device: block containing cell i (binary search over B blocks)
__device__ __forceinline__ int find_blk(const Blk *blk, int B, int i) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (blk[mid].off <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ stencil operators
constexpr int MAXK = 125;        // up to a 5x5x5 box of offsets

struct Stencil {
    int K = 0;                   // number of offsets
    int R = 1;                   // max |offset| per direction
    int diag = 0;                // index of (0,0,0)
    std::vector<int8_t> off;     // 3*K, sorted by (dz, dy, dx) = lexicographic cell order
    DBuf<int8_t> doff;
};

// Structured FP64 operator on a Space: coef[k*N + i] couples cell i with
// cell i + off[k] (zero where that neighbour is outside the block).
struct Op {
    Space *sp = nullptr;
    Stencil st;
    DBuf<double> coef;
};

// ------------------------------------------------------------------ grid
struct Grid {
    Alloc al;
    hipStream_t s = nullptr;
    int dim = 2;
    Space sp;
    std::vector<double> hdx, hdy, hdz;   // per block
    DBuf<double> geo;                    // 3*B: dx, dy, dz per block
    DBuf<double> tx, ty, tz;             // face to the + neighbour
    DBuf<double> pv;                     // V phi
    DBuf<double> src;                    // well source Q R T / W
    DBuf<double> kx, ky, kz;             // copies for the dlogK adjoint and boundary faces
    DBuf<int> bct;                       // 6*B boundary types (-x,+x,-y,+y,-z,+z), empty: all closed
    DBuf<double> bcv;                    // 6*B boundary values
    double a = 0, b = 0, RT = 0, W = 0, mu = 0, g = 0;
    int accum = NKS_ACCUM_CONSERVATIVE;
    // scratch
    DBuf<double> m, dm, hist, tmp;
    DBuf<double> d2m;                    // chain-rule accumulation only
    DBuf<int> flags;                     // per block: non-physical state
};

struct Matrix {
    Grid *g = nullptr;
    Op op;
    // the state the Jacobian was last evaluated at (rediscretised coarse
    // levels are evaluated from it)
    DBuf<double> state;
    double dt = 0.0;
    int order = 1;
    bool has_state = false;
};

// Jacobian evaluation bookkeeping: copy p into J.state (asynchronous)
void remember_state(Matrix &J, const double *p, double dt, int order);

// ------------------------------------------------------------------ rediscretised coarse grids
// The grid of ratio r coarser than f: every size above one a multiple of r,
// each permeability component the mean of the children's, pore volume their
// sum, cells r times larger, the same fluid, gravity and outer faces, no
// wells, conservative accumulation.  Fails with NKS_EINVAL otherwise.
void coarsen_grid(const Grid &f, int ratio, Grid &c);
// pc = mean of each coarse cell's children in pf
void launch_coarsen_mean(const Grid &f, const Grid &c, const double *pf, double *pc);
void launch_props(Grid &g, const double *p);
void launch_flux(Grid &g, const double *p, double dt, int order, double *F, double *J);

// ------------------------------------------------------------------ reductions
// Per-block sums, deterministic (fixed order), results on the device.
struct Reducer {
    DBuf<double> part;           // nchunks * maxcols
    DBuf<unsigned> counter;
    int maxcols = 0;
    void ensure(Alloc *al, const Space &sp, int cols, hipStream_t s);
};

// ------------------------------------------------------------------ kernels (host launchers)
void launch_spmv(const Op &A, const double *x, double *y, const double *b, const int *mask,
                 hipStream_t s);             // y = A x, or y = b - A x when b != nullptr
void launch_spmv_t(const Op &A, const double *x, double *y, const int *opp, hipStream_t s);
void launch_spmv_abs(const Op &A, const double *x, double *y, hipStream_t s);
void launch_transpose_op(const Op &A, Op &AT, const int *opp, hipStream_t s);   // same stencil, opp[q] = slot of -off_q
void launch_axpby(const Space &sp, double a, const double *x, double b, double *y,
                  const int *mask, hipStream_t s);   // y = a x + b y
void launch_copy_scale_blk(const Space &sp, const double *x, const double *scale, int col,
                           double *y, const int *mask, hipStream_t s);
void launch_block_dots(const Space &sp, Reducer &R, const double *x, const double *const *ys,
                       int ncols, double *out, const int *mask, hipStream_t s);
// norms squared per block of x: out[b]
void launch_block_norm2(const Space &sp, Reducer &R, const double *x, double *out,
                        const int *mask, hipStream_t s);

std::string fmt(const char *f, ...);

// Raise a kernel's dynamic LDS limit once per (kernel, size) instead of per launch.
void set_lds(const void *fn, size_t bytes);

// Event timing of named launches (active only after nks_profile_enable(1)).
bool prof_on();
// nks_profile_enable(2): work otherwise replayed from captured graphs runs as
// plain launches, so every launch is recorded
bool prof_direct();
// Events around a span of stream work (several kernels); includes any idle
// time between them.
struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s = nullptr;
    const char *name = nullptr;
    int level = -1;
    ProfScope(const char *name, hipStream_t s, int level = -1);
    ~ProfScope();
};

// An event pair to be bound to one kernel dispatch; false when profiling is
// off or the stream is being captured.
bool prof_pair(const char *name, int level, hipStream_t s, hipEvent_t *a, hipEvent_t *b);

// Device counters of a record's profiled launches ([0] extended cells, [1]
// owned cells of the subdomains a sweep did not find masked out); zeroed when
// recording starts.  Valid for a launch whose prof_pair returned true.
// host waits on the device (synchronisations and event waits on the solver
// paths), counted for the step statistics
void count_host_wait();
long host_waits();
constexpr int PROF_UNIT_SLOTS = 256;   // counter pairs per record, summed when read
unsigned long long *prof_units(const char *name, int level);

// A subdomain sweep: as launch_timed, and while that launch is profiled its
// arguments carry the record's cell counters (args.units), so the swept cells
// of each profiled launch are counted on the device.
template <typename Args>
inline void launch_sweep(const char *name, int level, void (*kernel)(Args), dim3 grid, dim3 block, size_t sh,
                         hipStream_t s, Args args) {
    hipEvent_t a = nullptr, b = nullptr;
    args.units = nullptr;
    if (prof_pair(name, level, s, &a, &b)) args.units = prof_units(name, level);
    else a = b = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)sh, s, a, b, 0u, args);
}

// Launch one kernel; while profiling, the events ride on the dispatch packet
// itself, so the recorded time is the kernel's execution alone.
template <typename... KArgs, typename... Args>
inline void launch_timed(const char *name, int level, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                         size_t sh, hipStream_t s, Args... args) {
    hipEvent_t a = nullptr, b = nullptr;
    if (!prof_pair(name, level, s, &a, &b)) a = b = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)sh, s, a, b, 0u, static_cast<KArgs>(args)...);
}

}  // namespace nks
