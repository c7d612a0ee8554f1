// C ABI of libnks: argument checks, handle lifetime, error translation, and
// the host-side control of the inexact Newton step (Section 3).
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <set>
#include <mutex>
#include <cstdarg>
#include <cstdio>

#include "schwarz.h"

namespace nks {

static thread_local std::string g_last_error;

std::string fmt(const char *f, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof(buf), f, ap);
    va_end(ap);
    return buf;
}

void fail(int code, const char *f, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof(buf), f, ap);
    va_end(ap);
    throw Error{code, buf};
}

void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? NKS_ENOMEM : NKS_EHIP, "%s failed: %s (%s:%d)", what,
             hipGetErrorString(e), file, line);
    }
}

void *Alloc::get(size_t bytes) {
    void *p = nullptr;
    if (fa) {
        p = fa(bytes, ctx);
        if (!p) fail(NKS_ENOMEM, "allocator callback returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(NKS_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        }
    }
    return p;
}

void Alloc::put(void *p) {
    if (!p) return;
    if (ff) ff(p, ctx);
    else (void)hipFree(p);
}

// ------------------------------------------------------------------ profiling
struct ProfRec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
// device cell counters per record (two each), kept across enable / disable
static std::map<std::string, unsigned long long *> g_prof_units;
static std::mutex g_prof_mu;
static std::map<std::string, ProfRec> g_prof;
static bool g_prof_on = false;
static bool g_prof_direct = false;           // mode 2: captured chunks run as plain launches
static std::set<std::string> g_prof_keep;   // record names kept (empty: all)
static std::vector<hipEvent_t> g_event_pool;

static bool prof_wanted(const std::string &key) { return g_prof_keep.empty() || g_prof_keep.count(key) != 0; }

bool prof_on() { return g_prof_on; }
bool prof_direct() { return g_prof_on && g_prof_direct; }

static std::atomic<long> g_host_waits{0};
void count_host_wait() { g_host_waits.fetch_add(1, std::memory_order_relaxed); }
long host_waits() { return g_host_waits.load(std::memory_order_relaxed); }

void set_lds(const void *fn, size_t bytes) {
    static std::mutex mu;
    static std::map<const void *, size_t> done;
    std::lock_guard<std::mutex> lk(mu);
    auto it = done.find(fn);
    if (it != done.end() && it->second >= bytes) return;
    HIPC(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    done[fn] = bytes;
}

static hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    return e;
}

ProfScope::ProfScope(const char *nm, hipStream_t st, int lvl) : s(st), name(nm), level(lvl) {
    if (!g_prof_on) return;
    if (!prof_wanted(level >= 0 ? fmt("%s_l%d", name, level) : std::string(name))) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    a = take_event();
    b = take_event();
    HIPC(hipEventRecord(a, s));
}

ProfScope::~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    (void)hipEventRecord(b, s);
    std::string key = level >= 0 ? fmt("%s_l%d", name, level) : std::string(name);
    g_prof[key].ev.push_back({a, b});
}

bool prof_pair(const char *nm, int lvl, hipStream_t s, hipEvent_t *a, hipEvent_t *b) {
    if (!g_prof_on) return false;
    std::string key = lvl >= 0 ? fmt("%s_l%d", nm, lvl) : std::string(nm);
    if (!prof_wanted(key)) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return false;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    *a = take_event();
    *b = take_event();
    g_prof[key].ev.push_back({*a, *b});
    return true;
}

unsigned long long *prof_units(const char *nm, int lvl) {
    std::string key = lvl >= 0 ? fmt("%s_l%d", nm, lvl) : std::string(nm);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    unsigned long long *&u = g_prof_units[key];
    if (!u) {
        const size_t bytes = 2 * PROF_UNIT_SLOTS * sizeof(unsigned long long);
        if (hipMalloc((void **)&u, bytes) != hipSuccess) {
            (void)hipGetLastError();
            u = nullptr;
            return nullptr;
        }
        HIPC(hipMemset(u, 0, bytes));
    }
    return u;
}

static void prof_clear() {
    for (auto &kv : g_prof_units)
        if (kv.second) HIPC(hipMemset(kv.second, 0, 2 * PROF_UNIT_SLOTS * sizeof(unsigned long long)));
    for (auto &kv : g_prof)
        for (auto &p : kv.second.ev) {
            g_event_pool.push_back(p.first);
            g_event_pool.push_back(p.second);
        }
    g_prof.clear();
}

// launchers defined in physics.hip
void grid_setup_kernels(Grid &g, const double *kx, const double *ky, const double *kz, const double *phi);
void launch_history(Grid &g, const double *pn, const double *pnm1, int order);
void launch_props(Grid &g, const double *p);
void launch_flux(Grid &g, const double *p, double dt, int order, double *F, double *J);
void launch_hydrostatic(Grid &g, double p_top, double *p);
void launch_residual_into(Grid &g, const double *p, const double *pn, const double *pnm1, double dt,
                          int order, double *F, double *hist, double *m, double *dm, int *flags);
void launch_dlogk_t(Grid &g, const double *p, const double *lam, double *out, bool accumulate);
void launch_adj_rhs(Grid &g, const double *pn, double dt, double c1, const double *l1, double c2,
                    const double *l2, const double *dg, double *out);

static inline int nblk(int n, int t) { return (n + t - 1) / t; }

// pt = p + lam[b] s, a workgroup per tile (a run of cells of one reservoir)
__global__ void k_trial(const Chunk *tiles, const double *p, const double *s, const double *lam, double *pt) {
    const Chunk ch = tiles[blockIdx.x];
    const int i = ch.start + (int)threadIdx.x;
    if (i < ch.end) pt[i] = p[i] + lam[ch.blk] * s[i];
}

__global__ void k_neg(int N, const double *x, double *y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = -x[i];
}

// y = x on the reservoirs with mask[b] set, a workgroup per tile
__global__ void k_copy_mask(const Chunk *tiles, const double *x, double *y, const int *mask) {
    const Chunk ch = tiles[blockIdx.x];
    const int i = ch.start + (int)threadIdx.x;
    if (i < ch.end && mask[ch.blk]) y[i] = x[i];
}

__global__ void k_zero(int N, double *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) x[i] = 0.0;
}

// Newton workspace kept on the grid between calls
struct NewtonWork {
    DBuf<double> F, Ft, s, b, pt, Js, lam, red2;
    DBuf<int> mask;
    DBuf<const double *> ysp;     // {Js}: the slope reduction's column
    const double *ysp_host = nullptr;
    Reducer red;
    std::unique_ptr<Matrix> J;
    std::unique_ptr<Ras> M;
    nks_ras_desc rd{};
    Gmres gm;
    // pinned host staging for the per-reservoir scalars (asynchronous copies):
    // doubles norms[B], slope[B], lam[B]; ints flags[B], mask[B]
    void *hpin = nullptr;
    int hpin_b = 0;
    double *h_norm = nullptr, *h_slope = nullptr, *h_lam = nullptr;
    int *h_flags = nullptr, *h_mask = nullptr;
    void pin(int B) {
        if (hpin && hpin_b >= B) return;
        if (hpin) HIPC(hipHostFree(hpin));
        HIPC(hipHostMalloc(&hpin, (size_t)B * (3 * sizeof(double) + 2 * sizeof(int))));
        hpin_b = B;
        h_norm = static_cast<double *>(hpin);
        h_slope = h_norm + B;
        h_lam = h_slope + B;
        h_flags = reinterpret_cast<int *>(h_lam + B);
        h_mask = h_flags + B;
    }
    ~NewtonWork() {
        if (hpin) (void)hipHostFree(hpin);
    }
};

static void stencil_fine(Stencil &st, int dim, Alloc *al, hipStream_t s) {
    std::vector<int8_t> off;
    if (dim == 3) off = {0, 0, -1, 0, -1, 0, -1, 0, 0, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1};
    else off = {0, -1, 0, -1, 0, 0, 0, 0, 0, 1, 0, 0, 0, 1, 0};
    st.off = off;
    st.K = (int)off.size() / 3;
    st.diag = st.K / 2;
    st.R = 1;
    st.doff.upload(al, off, s);
}

static bool same_desc(const nks_ras_desc &a, const nks_ras_desc &b) {
    return memcmp(&a, &b, sizeof(a)) == 0;
}

// opp[q] = slot of the offset -off_q; the stencils here are point-symmetric
static std::vector<int> opposite_slots(const Stencil &st) {
    std::vector<int> opp(st.K, -1);
    for (int k = 0; k < st.K; ++k)
        for (int q = 0; q < st.K; ++q)
            if (st.off[3 * q] == -st.off[3 * k] && st.off[3 * q + 1] == -st.off[3 * k + 1] &&
                st.off[3 * q + 2] == -st.off[3 * k + 2])
                opp[k] = q;
    for (int k = 0; k < st.K; ++k)
        if (opp[k] < 0) fail(NKS_EINVAL, "stencil is not point-symmetric");
    return opp;
}

// A matrix on the fine stencil of grid g
static void fine_matrix(Matrix &M, Grid &g) {
    M.g = &g;
    M.op.sp = &g.sp;
    stencil_fine(M.op.st, g.dim, &g.al, g.s);
    M.op.coef.alloc(&g.al, (size_t)M.op.st.K * g.sp.N);
}

// The transpose of a Schwarz preconditioner built on J: the same boxes and
// levels built on J^T, with left- and right-RAS exchanged.  ILU(0) of A^T on
// a symmetric pattern is the transpose of ILU(0) of A and the Galerkin product
// commutes with transposition, so for one level this is exactly M^T.  The
// transpose of a multilevel composition reverses the order of its factors, so
// the pre- and post-smoothing counts trade places and left and right Kaskade
// exchange; the result is the transpose of the cycle on J up to its inexact
// coarse solve.
struct TransposedRas {
    Matrix JT;
    DBuf<int> opp;
    std::unique_ptr<Ras> MT;
    nks_ras_desc d{};
    bool stale = true;
    void refresh(Matrix &J, const nks_ras_desc &dd) {
        Grid &g = *J.g;
        if (dd.coarse_op != NKS_COARSE_GALERKIN)
            fail(NKS_EINVAL, "the transposed preconditioner needs Galerkin coarse operators");
        if (!MT || !same_desc(d, dd)) {
            fine_matrix(JT, g);
            std::vector<int> o = opposite_slots(J.op.st);
            opp.upload(&g.al, o, g.s);
            nks_ras_desc dt = dd;
            dt.variant = dd.variant == NKS_LEFT_RAS ? NKS_RIGHT_RAS
                                                    : (dd.variant == NKS_RIGHT_RAS ? NKS_LEFT_RAS : dd.variant);
            dt.mu = dd.nu;
            dt.nu = dd.mu;
            dt.cycle = dd.cycle == NKS_LEFT_KASKADE ? NKS_RIGHT_KASKADE
                                                    : (dd.cycle == NKS_RIGHT_KASKADE ? NKS_LEFT_KASKADE : dd.cycle);
            // the exchanged variant may rule out the persistent coarse solve
            if (dt.coarse_kernel == NKS_COARSE_PERSISTENT) dt.coarse_kernel = NKS_COARSE_AUTO;
            MT.reset(new Ras());
            MT->build(&JT, dt);
            d = dd;
            stale = true;
        }
        if (stale) {
            launch_transpose_op(J.op, JT.op, opp.p, g.s);
            MT->factor();
            MT->check_pivots();
            stale = false;
        }
    }
};

// Workspace of the discrete adjoint
struct AdjointWork {
    Matrix J;
    TransposedRas T;
    Gmres gm;
    DBuf<double> rhs, lam[3];
    bool ready = false;
};

}  // namespace nks

using namespace nks;

// A grid's memory backs its matrices and preconditioners (their buffers come
// from its allocator), so each of them holds a reference to the grid; a
// preconditioner reads its matrix (the finest level's operator), so it holds
// a reference to that matrix too.  Each object goes when its own handle and
// the last reference to it are gone, in whatever order the caller destroys
// the handles.
struct nks_grid {
    Grid g;
    std::unique_ptr<NewtonWork> nw;
    std::unique_ptr<AdjointWork> aw;
    int refs = 1;
};
struct nks_matrix {
    Matrix m;
    nks_grid *owner;
    DBuf<int> opp;       // opposite stencil slots, for transposes
    int refs = 1;
};
struct nks_ras {
    Ras r;
    TransposedRas t;     // built on first use of the transpose
    nks_grid *owner = nullptr;
    nks_matrix *mat = nullptr;   // the matrix the finest level reads
};

static void grid_release(nks_grid *g) {
    if (--g->refs == 0) {
        (void)hipStreamSynchronize(g->g.s);
        delete g;
    }
}

static void matrix_release(nks_matrix *J) {
    if (--J->refs == 0) {
        nks_grid *owner = J->owner;
        (void)hipStreamSynchronize(J->m.g->s);
        delete J;
        grid_release(owner);
    }
}

template <typename F>
static int guard(F &&f) {
    try {
        g_last_error.clear();
        f();
        return NKS_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return NKS_EINVAL;
    }
}

static void sync_upload_done(hipStream_t s) { HIPC(hipStreamSynchronize(s)); }

extern "C" {

const char *nks_last_error(void) { return g_last_error.c_str(); }

int nks_profile_enable(int enable) {
    return guard([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (enable) {
            HIPC(hipDeviceSynchronize());
            prof_clear();
        }
        g_prof_on = enable != 0;
        g_prof_direct = enable == 2;
    });
}


int nks_profile_filter(const char *names) {
    return guard([&] {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_keep.clear();
        if (!names) return;
        std::string cur;
        for (const char *c = names;; ++c) {
            if (*c == ',' || *c == '\0') {
                if (!cur.empty()) g_prof_keep.insert(cur);
                cur.clear();
                if (*c == '\0') break;
            } else {
                cur.push_back(*c);
            }
        }
    });
}

// per-launch durations of one record (ms); synchronises on each event
static std::vector<double> prof_durations(const char *name) {
    std::vector<double> out;
    auto it = g_prof.find(name);
    if (it == g_prof.end()) return out;
    for (auto &p : it->second.ev) {
        HIPC(hipEventSynchronize(p.second));
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, p.first, p.second));
        out.push_back(ms);
    }
    return out;
}

int nks_profile_query(const char *name, int *count, double *total_ms) {
    return guard([&] {
        if (!name || !count || !total_ms) fail(NKS_EINVAL, "bad arguments");
        std::lock_guard<std::mutex> lk(g_prof_mu);
        std::vector<double> d = prof_durations(name);
        *count = (int)d.size();
        *total_ms = 0.0;
        for (double x : d) *total_ms += x;
    });
}

int nks_profile_durations(const char *name, double *ms, int cap, int *count) {
    return guard([&] {
        if (!name || !count || cap < 0 || (cap > 0 && !ms)) fail(NKS_EINVAL, "bad arguments");
        std::lock_guard<std::mutex> lk(g_prof_mu);
        std::vector<double> d = prof_durations(name);
        *count = (int)d.size();
        for (int i = 0; i < cap && i < (int)d.size(); ++i) ms[i] = d[i];
    });
}
int nks_profile_units(const char *name, double *cells) {
    return guard([&] {
        if (!name || !cells) fail(NKS_EINVAL, "bad arguments");
        cells[0] = cells[1] = 0.0;
        unsigned long long *u = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            auto it = g_prof_units.find(name);
            if (it != g_prof_units.end()) u = it->second;
        }
        if (!u) return;
        HIPC(hipDeviceSynchronize());
        std::vector<unsigned long long> h(2 * PROF_UNIT_SLOTS);
        HIPC(hipMemcpy(h.data(), u, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        for (int k = 0; k < PROF_UNIT_SLOTS; ++k) {
            cells[0] += (double)h[2 * k];
            cells[1] += (double)h[2 * k + 1];
        }
    });
}

const char *nks_version(void) { return "libnks 0.1 (gfx950)"; }

int nks_setup_grid(const nks_grid_desc *d, nks_grid **out) {
    return guard([&] {
        if (!d || !out || d->nres < 1 || !d->res) fail(NKS_EINVAL, "bad grid descriptor");
        auto *h = new nks_grid();
        std::unique_ptr<nks_grid> hold(h);
        Grid &g = h->g;
        g.al.fa = d->alloc;
        g.al.ff = d->free;
        g.al.ctx = d->alloc_ctx;
        if ((d->alloc == nullptr) != (d->free == nullptr)) fail(NKS_EINVAL, "alloc and free must be given together");
        g.s = (hipStream_t)d->stream;
        std::vector<Blk> blks;
        std::vector<double> geo;
        int dim = 0;
        for (int b = 0; b < d->nres; ++b) {
            const nks_reservoir_desc &r = d->res[b];
            if (r.nx < 1 || r.ny < 1 || r.nz < 1 || !(r.dx > 0) || !(r.dy > 0) || !(r.dz > 0))
                fail(NKS_EINVAL, "reservoir %d: bad dimensions", b);
            if (!r.kx || !r.ky || !r.kz || !r.phi) fail(NKS_EINVAL, "reservoir %d: missing arrays", b);
            const int rd = r.nz > 1 ? 3 : 2;
            if (dim && rd != dim) fail(NKS_EINVAL, "reservoirs mix 2D and 3D grids");
            dim = rd;
            blks.push_back({r.nx, r.ny, r.nz, 0});
            geo.push_back(r.dx);
            geo.push_back(r.dy);
            geo.push_back(r.dz);
        }
        g.dim = dim;
        g.sp.build(&g.al, blks, g.s);
        const int N = g.sp.N, B = g.sp.B;
        g.geo.upload(&g.al, geo, g.s);
        g.tx.alloc(&g.al, N); g.ty.alloc(&g.al, N); g.tz.alloc(&g.al, N);
        g.pv.alloc(&g.al, N);
        g.kx.alloc(&g.al, N); g.ky.alloc(&g.al, N); g.kz.alloc(&g.al, N);
        DBuf<double> phi;
        phi.alloc(&g.al, N);
        for (int b = 0; b < B; ++b) {
            const nks_reservoir_desc &r = d->res[b];
            const size_t n = (size_t)r.nx * r.ny * r.nz, o = g.sp.hblk[b].off;
            HIPC(hipMemcpyAsync(g.kx.p + o, r.kx, n * 8, hipMemcpyDeviceToDevice, g.s));
            HIPC(hipMemcpyAsync(g.ky.p + o, r.ky, n * 8, hipMemcpyDeviceToDevice, g.s));
            HIPC(hipMemcpyAsync(g.kz.p + o, r.kz, n * 8, hipMemcpyDeviceToDevice, g.s));
            HIPC(hipMemcpyAsync(phi.p + o, r.phi, n * 8, hipMemcpyDeviceToDevice, g.s));
        }
        grid_setup_kernels(g, g.kx.p, g.ky.p, g.kz.p, phi.p);
        const nks_fluid &f = d->fluid;
        if (!(f.T > 0) || !(f.Tc > 0) || !(f.pc > 0) || !(f.R > 0) || !(f.W > 0) || !(f.mu > 0))
            fail(NKS_EINVAL, "bad fluid constants");
        // acentric factor from the normal boiling point (Section 2's
        // correlation in the reduced boiling temperature) when Tb is given
        double w = f.omega;
        if (f.Tb != 0.0) {
            if (!(f.Tb > 0.0) || !(f.Tb < f.Tc)) fail(NKS_EINVAL, "Tb must lie in (0, Tc)");
            const double tr = f.Tb / f.Tc, u = 1.0 - tr;
            const double u15 = u * std::sqrt(u), u25 = u15 * u, u5 = u25 * u25;
            const double f0 = (-5.97616 * u + 1.29874 * u15 - 0.60394 * u25 - 1.06841 * u5) / tr;
            const double f1 = (-5.03365 * u + 1.11505 * u15 - 5.41217 * u25 - 7.46628 * u5) / tr;
            w = (-std::log(f.pc / 101325.0) - f0) / f1;
        }
        // attraction and covolume of the PR equation of state (the criticality relations for a(T) and b (Section 2))
        const double mw = w <= 0.491 ? 0.37464 + 1.54226 * w - 0.26992 * w * w
                                     : 0.3796 + 1.485 * w - 0.1644 * w * w + 0.01667 * w * w * w;
        const double al = 1.0 + mw * (1.0 - std::sqrt(f.T / f.Tc));
        g.a = 0.45724 * f.R * f.R * f.Tc * f.Tc / f.pc * al * al;
        g.b = 0.0778 * f.R * f.Tc / f.pc;
        g.RT = f.R * f.T;
        g.W = f.W;
        g.mu = f.mu;
        g.g = d->gravity ? d->g : 0.0;
        // well source per cell, summed over wells in a fixed order
        std::vector<double> src(N, 0.0);
        for (int b = 0; b < B; ++b) {
            const nks_reservoir_desc &r = d->res[b];
            const int n = r.nx * r.ny * r.nz;
            for (int k = 0; k < r.nwells; ++k) {
                const int c = r.well_cell[k];
                if (c < 0 || c >= n) fail(NKS_EINVAL, "reservoir %d: well cell %d out of range", b, c);
                src[g.sp.hblk[b].off + c] += r.well_rate[k] * g.RT / g.W;
            }
        }
        g.src.upload(&g.al, src, g.s);
        // outer-face boundary conditions, 6 per reservoir
        std::vector<int> bct(6 * (size_t)B, NKS_BC_CLOSED);
        std::vector<double> bcv(6 * (size_t)B, 0.0);
        bool any_bc = false;
        for (int b = 0; b < B; ++b) {
            const nks_reservoir_desc &r = d->res[b];
            if ((r.bc_type == nullptr) != (r.bc_value == nullptr))
                fail(NKS_EINVAL, "reservoir %d: bc_type and bc_value must be given together", b);
            if (!r.bc_type) continue;
            for (int f = 0; f < 6; ++f) {
                const int t = r.bc_type[f];
                const double v = r.bc_value[f];
                if (t < NKS_BC_CLOSED || t > NKS_BC_NEUMANN) fail(NKS_EINVAL, "reservoir %d face %d: bad type %d", b, f, t);
                if (t == NKS_BC_DIRICHLET && !(v > 0.0)) fail(NKS_EINVAL, "reservoir %d face %d: p^D must be > 0", b, f);
                if (t == NKS_BC_NEUMANN && !std::isfinite(v)) fail(NKS_EINVAL, "reservoir %d face %d: bad q^N", b, f);
                bct[6 * b + f] = t;
                bcv[6 * b + f] = t == NKS_BC_CLOSED ? 0.0 : v;
                any_bc = any_bc || t != NKS_BC_CLOSED;
            }
        }
        if (any_bc) {
            g.bct.upload(&g.al, bct, g.s);
            g.bcv.upload(&g.al, bcv, g.s);
        }
        if (d->accum != NKS_ACCUM_CONSERVATIVE && d->accum != NKS_ACCUM_CHAIN_RULE)
            fail(NKS_EINVAL, "unknown accumulation form %d", d->accum);
        g.accum = d->accum;
        g.m.alloc(&g.al, N);
        g.dm.alloc(&g.al, N);
        if (g.accum == NKS_ACCUM_CHAIN_RULE) g.d2m.alloc(&g.al, N);
        g.hist.alloc(&g.al, N);
        g.tmp.alloc(&g.al, N);
        g.flags.alloc(&g.al, B);
        HIPC(hipMemsetAsync(g.flags.p, 0, sizeof(int) * B, g.s));
        sync_upload_done(g.s);
        *out = hold.release();
    });
}

int nks_destroy_grid(nks_grid *g) {
    return guard([&] {
        if (g) grid_release(g);
    });
}

int nks_grid_info(const nks_grid *g, int *ncells, int *nres, int *offsets) {
    return guard([&] {
        if (!g) fail(NKS_EINVAL, "null grid");
        if (ncells) *ncells = g->g.sp.N;
        if (nres) *nres = g->g.sp.B;
        if (offsets) {
            for (int b = 0; b < g->g.sp.B; ++b) offsets[b] = g->g.sp.hblk[b].off;
            offsets[g->g.sp.B] = g->g.sp.N;
        }
    });
}

int nks_hydrostatic_init(nks_grid *g, double p_top, double *p) {
    return guard([&] {
        if (!g || !p || !(p_top > 0)) fail(NKS_EINVAL, "bad arguments");
        launch_hydrostatic(g->g, p_top, p);
    });
}

int nks_residual(nks_grid *g, const double *p, const double *pn, const double *pnm1, double dt, int order,
                 double *F) {
    return guard([&] {
        if (!g || !p || !pn || !F || !(dt > 0) || (order != 1 && order != 2) || (order == 2 && !pnm1))
            fail(NKS_EINVAL, "bad arguments");
        launch_history(g->g, pn, pnm1, order);
        launch_props(g->g, p);
        launch_flux(g->g, p, dt, order, F, nullptr);
    });
}

}  // extern "C"

namespace nks {

// Fixed device scratch of nks_residual_noalloc: the history term, m and dm/dp
// (NKS_NOALLOC_MAX_CELLS doubles each), then MAXB ints of non-physical flags.
// Host code never passes the symbol itself to a kernel: each device's address
// of its copy comes from hipGetSymbolAddress, looked up once per device.
constexpr size_t NOALLOC_CELLS = NKS_NOALLOC_MAX_CELLS;
constexpr size_t NOALLOC_DOUBLES = 3 * NOALLOC_CELLS + MAXB / 2;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

static std::mutex g_scratch_mu;
static std::map<int, double *> g_scratch_ptr;

// Address of `scratch` on the device of stream s (looked up with that device current).
static double *scratch_on(hipStream_t s) {
    int dev = 0;
    HIPC(hipStreamGetDevice(s, &dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    int cur = 0;
    HIPC(hipGetDevice(&cur));
    if (cur != dev) HIPC(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) HIPC(hipSetDevice(cur));
    HIPC(e);
    if (!ptr) fail(NKS_EHIP, "no device address for the residual scratch on device %d", dev);
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
    return static_cast<double *>(ptr);
}

}  // namespace nks

extern "C" {

int nks_residual_noalloc(nks_grid *g, const double *p, const double *pn, const double *pnm1, double dt,
                         int order, double *F) {
    return guard([&] {
        if (!g || !p || !pn || !F || !(dt > 0) || (order != 1 && order != 2) || (order == 2 && !pnm1))
            fail(NKS_EINVAL, "bad arguments");
        Grid &G = g->g;
        if ((size_t)G.sp.N > NOALLOC_CELLS)
            fail(NKS_EINVAL, "nks_residual_noalloc: %d cells exceed the fixed scratch of %zu cells", G.sp.N,
                 NOALLOC_CELLS);
        if (G.sp.B > MAXB) fail(NKS_EINVAL, "nks_residual_noalloc: %d reservoirs exceed %d", G.sp.B, MAXB);
        double *base = scratch_on(G.s);
        double *hist = base;
        double *m = base + NOALLOC_CELLS;
        double *dm = base + 2 * NOALLOC_CELLS;
        int *flags = reinterpret_cast<int *>(base + 3 * NOALLOC_CELLS);
        launch_residual_into(G, p, pn, pnm1, dt, order, F, hist, m, dm, flags);
    });
}

int nks_matrix_create(nks_grid *g, nks_matrix **out) {
    return guard([&] {
        if (!g || !out) fail(NKS_EINVAL, "bad arguments");
        std::unique_ptr<nks_matrix> hold(new nks_matrix());
        nks_matrix *m = hold.get();
        m->owner = g;
        m->m.g = &g->g;
        m->m.op.sp = &g->g.sp;
        stencil_fine(m->m.op.st, g->g.dim, &g->g.al, g->g.s);
        m->m.op.coef.alloc(&g->g.al, (size_t)m->m.op.st.K * g->g.sp.N);
        HIPC(hipMemsetAsync(m->m.op.coef.p, 0, sizeof(double) * m->m.op.st.K * g->g.sp.N, g->g.s));
        sync_upload_done(g->g.s);
        g->refs++;
        *out = hold.release();
    });
}

int nks_destroy_matrix(nks_matrix *J) {
    return guard([&] {
        if (J) matrix_release(J);
    });
}

int nks_jacobian(nks_grid *g, const double *p, const double *pn, const double *pnm1, double dt, int order,
                 nks_matrix *J, double *F) {
    return guard([&] {
        if (!g || !p || !pn || !J || !(dt > 0) || (order != 1 && order != 2) || (order == 2 && !pnm1))
            fail(NKS_EINVAL, "bad arguments");
        if (J->m.g != &g->g) fail(NKS_EINVAL, "matrix belongs to another grid");
        launch_history(g->g, pn, pnm1, order);
        launch_props(g->g, p);
        launch_flux(g->g, p, dt, order, F, J->m.op.coef.p);
        remember_state(J->m, p, dt, order);
    });
}

static void export_op(const Op &A, hipStream_t s, int *rp, int *ci, double *v, int *nnz_out) {
    const Space &S = *A.sp;
    std::vector<double> c((size_t)A.st.K * S.N);
    HIPC(hipMemcpyAsync(c.data(), A.coef.p, c.size() * 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    int nnz = 0;
    if (rp) rp[0] = 0;
    for (int b = 0; b < S.B; ++b) {
        const Blk &k = S.hblk[b];
        for (int z = 0; z < k.nz; ++z)
            for (int y = 0; y < k.ny; ++y)
                for (int x = 0; x < k.nx; ++x) {
                    const int i = k.off + x + k.nx * (y + k.ny * z);
                    for (int q = 0; q < A.st.K; ++q) {
                        const int xx = x + A.st.off[3 * q], yy = y + A.st.off[3 * q + 1], zz = z + A.st.off[3 * q + 2];
                        if (xx < 0 || xx >= k.nx || yy < 0 || yy >= k.ny || zz < 0 || zz >= k.nz) continue;
                        if (ci) {
                            ci[nnz] = k.off + xx + k.nx * (yy + k.ny * zz);
                            v[nnz] = c[(size_t)q * S.N + i];
                        }
                        ++nnz;
                    }
                    if (rp) rp[i + 1] = nnz;
                }
    }
    if (nnz_out) *nnz_out = nnz;
}

int nks_matrix_nnz(const nks_matrix *J, int *nnz) {
    return guard([&] {
        if (!J || !nnz) fail(NKS_EINVAL, "bad arguments");
        export_op(J->m.op, J->m.g->s, nullptr, nullptr, nullptr, nnz);
    });
}

int nks_matrix_export_csr(const nks_matrix *J, int *rp, int *ci, double *v) {
    return guard([&] {
        if (!J || !rp || !ci || !v) fail(NKS_EINVAL, "bad arguments");
        export_op(J->m.op, J->m.g->s, rp, ci, v, nullptr);
    });
}

int nks_matrix_apply(nks_matrix *J, const double *x, double *y) {
    return guard([&] {
        if (!J || !x || !y) fail(NKS_EINVAL, "bad arguments");
        launch_spmv(J->m.op, x, y, nullptr, nullptr, J->m.g->s);
    });
}

int nks_jacobian_transpose_apply(nks_matrix *J, const double *x, double *y) {
    return guard([&] {
        if (!J || !x || !y) fail(NKS_EINVAL, "bad arguments");
        const Stencil &st = J->m.op.st;
        std::vector<int> opp(st.K);
        for (int k = 0; k < st.K; ++k)
            for (int q = 0; q < st.K; ++q)
                if (st.off[3 * q] == -st.off[3 * k] && st.off[3 * q + 1] == -st.off[3 * k + 1] &&
                    st.off[3 * q + 2] == -st.off[3 * k + 2])
                    opp[k] = q;
        DBuf<int> d;
        d.upload(&J->m.g->al, opp, J->m.g->s);
        launch_spmv_t(J->m.op, x, y, d.p, J->m.g->s);
        HIPC(hipStreamSynchronize(J->m.g->s));
    });
}

int nks_residual_dlogk_transpose_apply(nks_grid *g, const double *p, const double *lam, double *out) {
    return guard([&] {
        if (!g || !p || !lam || !out) fail(NKS_EINVAL, "bad arguments");
        launch_dlogk_t(g->g, p, lam, out, false);
    });
}

int nks_matrix_transpose(nks_matrix *J, nks_matrix *JT) {
    return guard([&] {
        if (!J || !JT || J == JT) fail(NKS_EINVAL, "bad arguments");
        if (J->m.g != JT->m.g) fail(NKS_EINVAL, "matrices belong to different grids");
        if (!J->opp.p) {
            std::vector<int> o = opposite_slots(J->m.op.st);
            J->opp.upload(&J->m.g->al, o, J->m.g->s);
        }
        launch_transpose_op(J->m.op, JT->m.op, J->opp.p, J->m.g->s);
    });
}

static void check_ras_desc(const nks_ras_desc *d) {
    if (!d || d->px < 1 || d->py < 1 || d->pz < 1 || d->levels < 1 || d->levels > 6)
        fail(NKS_EINVAL, "bad preconditioner descriptor");
    for (int l = 0; l < d->levels; ++l)
        if (d->overlap[std::min(l, 7)] < 0) fail(NKS_EINVAL, "negative overlap");
    if (d->variant < 0 || d->variant > 2 || d->interp_order < 1 || d->interp_order > 3 || d->cycle < 0 ||
        d->cycle > 4 || d->mu < 0 || d->nu < 0 || d->precision < 0 || d->precision > 2 ||
        d->coarse_restart < 1 || d->coarse_maxit < 1 || d->tx < 0 || d->ty < 0 || d->tz < 0 || d->fill < 0 ||
        d->fill > 4 || d->ratio < 0 || d->ratio == 1 || d->ratio > 16 ||
        (d->coarse_op != NKS_COARSE_GALERKIN && d->coarse_op != NKS_COARSE_REDISCRETIZED) ||
        d->coarse_kernel < NKS_COARSE_AUTO || d->coarse_kernel > NKS_COARSE_PERSISTENT)
        fail(NKS_EINVAL, "bad preconditioner option");
}

int nks_ras_setup(nks_matrix *J, const nks_ras_desc *d, nks_ras **inout) {
    return guard([&] {
        if (!J || !inout) fail(NKS_EINVAL, "bad arguments");
        check_ras_desc(d);
        nks_ras *M = *inout;
        std::unique_ptr<nks_ras> hold;
        if (M && M->owner != J->owner) fail(NKS_EINVAL, "the preconditioner belongs to another grid");
        if (!M) {
            hold.reset(new nks_ras());
            M = hold.get();
            M->r.build(&J->m, *d);
        } else if (M->r.J != &J->m || !same_desc(M->r.d, *d)) {
            M->r.build(&J->m, *d);
        }
        M->r.factor();
        M->t.stale = true;
        if (M->mat != J) {
            J->refs++;
            if (M->mat) matrix_release(M->mat);
            M->mat = J;
        }
        if (hold) {
            M->owner = J->owner;
            J->owner->refs++;
            *inout = hold.release();
        }
    });
}

int nks_destroy_ras(nks_ras *M) {
    return guard([&] {
        if (M) {
            nks_grid *owner = M->owner;
            nks_matrix *mat = M->mat;
            (void)hipStreamSynchronize(M->r.g->s);
            delete M;
            if (mat) matrix_release(mat);
            if (owner) grid_release(owner);
        }
    });
}

int nks_ras_apply(nks_ras *M, const double *r, double *z) {
    return guard([&] {
        if (!M || !r || !z) fail(NKS_EINVAL, "bad arguments");
        M->r.apply(r, z, nullptr);
    });
}

int nks_ras_apply_level(nks_ras *M, int level, const double *r, double *z) {
    return guard([&] {
        if (!M || !r || !z || level < 0 || level >= M->r.L) fail(NKS_EINVAL, "bad arguments");
        M->r.apply_level(level, r, z, nullptr, false);
    });
}

int nks_ras_coarse_solve(nks_ras *M, const double *b, double *x) {
    return guard([&] {
        if (!M || !b || !x || M->r.L < 2) fail(NKS_EINVAL, "bad arguments");
        M->r.coarse_solve(b, x, nullptr);
    });
}

int nks_ras_coarse_stats(nks_ras *M, int *its, double *res) {
    return guard([&] {
        if (!M || M->r.L < 2) fail(NKS_EINVAL, "bad arguments");
        Ras &R = M->r;
        const int B = R.lev[R.L - 1]->spp->B;
        std::vector<int> hi(B, 0), conv;
        std::vector<double> hr(B, 0.0);
        if (R.cp.on) {
            HIPC(hipMemcpyAsync(hi.data(), R.cp.its.p, sizeof(int) * B, hipMemcpyDeviceToHost, R.g->s));
            HIPC(hipMemcpyAsync(hr.data(), R.cp.res.p, sizeof(double) * B, hipMemcpyDeviceToHost, R.g->s));
            HIPC(hipStreamSynchronize(R.g->s));
        } else {
            R.coarse.stats(hi, hr, conv, R.g->s);
        }
        for (int b = 0; b < B; ++b) {
            if (its) its[b] = hi[b];
            if (res) res[b] = hr[b];
        }
    });
}

int nks_ras_apply_transpose(nks_ras *M, const double *r, double *z) {
    return guard([&] {
        if (!M || !r || !z) fail(NKS_EINVAL, "bad arguments");
        M->t.refresh(*M->r.J, M->r.d);
        M->t.MT->apply(r, z, nullptr);
    });
}

int nks_ras_level_info(nks_ras *M, int level, int *info) {
    return guard([&] {
        if (!M || !info || level < 0 || level >= M->r.L) fail(NKS_EINVAL, "bad arguments");
        Level &V = *M->r.lev[level];
        int nnz = 0;
        export_op(*V.A, M->r.g->s, nullptr, nullptr, nullptr, &nnz);
        info[0] = V.spp->N;
        info[1] = V.A->st.K;
        info[2] = V.nsub;
        info[3] = V.spp->hblk[0].nx;
        info[4] = V.spp->hblk[0].ny;
        info[5] = V.spp->hblk[0].nz;
        info[6] = M->r.L;
        info[7] = nnz;
    });
}

int nks_ras_level_sweep(nks_ras *M, int level, int *form, int *workgroups) {
    return guard([&] {
        if (!M || !form || !workgroups || level < 0 || level >= M->r.L) fail(NKS_EINVAL, "bad arguments");
        *form = M->r.lev[level]->form;
        *workgroups = M->r.lev[level]->form_wgs;
    });
}

int nks_ras_level_export(nks_ras *M, int level, int *rp, int *ci, double *v) {
    return guard([&] {
        if (!M || !rp || !ci || !v || level < 0 || level >= M->r.L) fail(NKS_EINVAL, "bad arguments");
        export_op(*M->r.lev[level]->A, M->r.g->s, rp, ci, v, nullptr);
    });
}

int nks_ras_restrict(nks_ras *M, int level, const double *rf, double *rc) {
    return guard([&] {
        if (!M || !rf || !rc || level < 0 || level + 1 >= M->r.L) fail(NKS_EINVAL, "bad arguments");
        M->r.restrict_to(level, rf, rc, nullptr);
    });
}

int nks_ras_prolong_add(nks_ras *M, int level, const double *ec, double *zf) {
    return guard([&] {
        if (!M || !ec || !zf || level < 0 || level + 1 >= M->r.L) fail(NKS_EINVAL, "bad arguments");
        M->r.prolong_add(level, ec, zf, nullptr);
    });
}

int nks_gmres_solve(nks_matrix *J, nks_ras *M, const double *b, double *x, const nks_gmres_desc *d,
                    nks_gmres_stats *st) {
    return guard([&] {
        if (!J || !b || !x || !d || d->restart < 1 || d->restart > 30 || d->maxit < 1)
            fail(NKS_EINVAL, "bad arguments");
        Grid &g = *J->m.g;
        if (d->transpose && M) M->t.refresh(*M->r.J, M->r.d);
        auto &nwp = J->owner->nw;
        if (!nwp) nwp.reset(new NewtonWork());
        Gmres &gm = nwp->gm;
        gm.ensure(&g.al, g.sp, d->restart, d->flexible != 0, g.s);
        DBuf<int> opp;
        if (d->transpose) {
            const Stencil &st2 = J->m.op.st;
            std::vector<int> o(st2.K);
            for (int k = 0; k < st2.K; ++k) o[k] = st2.K - 1 - k;
            opp.upload(&g.al, o, g.s);
        }
        MatVec A = [&](const double *xx, double *yy, const double *bb, const int *mk) {
            if (d->transpose) {
                launch_spmv_t(J->m.op, xx, yy, opp.p, g.s);
                if (bb) launch_axpby(g.sp, 1.0, bb, -1.0, yy, nullptr, g.s);
            } else {
                launch_spmv(J->m.op, xx, yy, bb, mk, g.s);
            }
        };
        Precond P = [&](const double *r, double *z, const int *mk) {
            if (M && d->transpose) M->t.MT->apply(r, z, mk);
            else if (M) M->r.apply(r, z, mk);
            else launch_axpby(g.sp, 1.0, r, 0.0, z, mk, g.s);
        };
        GmOpts o;
        o.rtol = d->rtol;
        o.atol = d->atol;
        o.maxit = d->maxit;
        o.flexible = d->flexible != 0;
        o.check_every = 1;
        gm.solve(A, P, b, x, false, o, nullptr, g.s, d->transpose ? nullptr : &J->m.op);
        std::vector<int> its, conv;
        std::vector<double> res;
        gm.stats(its, res, conv, g.s);
        if (M) {
            if (d->transpose) M->t.MT->check_pivots();
            else M->r.check_pivots();
        }
        if (st) {
            st->iterations = 0;
            st->total_iterations = 0;
            st->residual = 0;
            st->converged = 0;
            for (int k = 0; k < g.sp.B; ++k) {
                st->iterations = std::max(st->iterations, its[k]);
                st->total_iterations += its[k];
                st->residual = std::max(st->residual, res[k]);
                st->converged += conv[k];
                if (st->its) st->its[k] = its[k];
                if (st->res) st->res[k] = res[k];
            }
        }
    });
}

// ------------------------------------------------------------------ Newton
static double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int nks_newton_step(nks_grid *gh, double *p, const double *pn, const double *pnm1, double dt, int order,
                    const nks_newton_desc *nd, const nks_ras_desc *rd, nks_newton_stats *st) {
    return guard([&] {
        if (!gh || !p || !pn || !nd || !rd || !(dt > 0) || (order != 1 && order != 2) || (order == 2 && !pnm1))
            fail(NKS_EINVAL, "bad arguments");
        check_ras_desc(rd);
        if (nd->restart < 1 || nd->restart > 30) fail(NKS_EINVAL, "restart must be in [1, 30]");
        if (nd->lag < 0) fail(NKS_EINVAL, "lag must be >= 0");
        Grid &g = gh->g;
        const int N = g.sp.N, B = g.sp.B;
        hipStream_t s = g.s;
        if (!gh->nw) gh->nw.reset(new NewtonWork());
        NewtonWork &W = *gh->nw;
        Alloc *al = &g.al;
        W.F.alloc(al, N); W.Ft.alloc(al, N); W.s.alloc(al, N); W.b.alloc(al, N);
        W.pt.alloc(al, N); W.Js.alloc(al, N);
        W.lam.alloc(al, B);
        W.red2.alloc(al, 2 * B);
        W.mask.alloc(al, B);
        W.red.ensure(al, g.sp, 1, s);
        W.pin(B);
        if (!W.J) {
            W.J.reset(new Matrix());
            W.J->g = &g;
            W.J->op.sp = &g.sp;
            stencil_fine(W.J->op.st, g.dim, al, s);
            W.J->op.coef.alloc(al, (size_t)W.J->op.st.K * N);
        }
        if (!W.M || !same_desc(W.rd, *rd)) {
            // captured FGMRES chunks hold the old preconditioner's buffers
            W.gm.invalidate_graphs();
            W.M.reset(new Ras());
            W.M->build(W.J.get(), *rd);
            W.rd = *rd;
        }
        const bool flex = nd->flexible < 0 ? (rd->levels > 1 || rd->precision != NKS_FP64) : nd->flexible != 0;
        W.gm.ensure(al, g.sp, nd->restart, flex, s);
        if (W.ysp_host != W.Js.p) {
            std::vector<const double *> hv(1, W.Js.p);
            W.ysp.upload(al, hv, s);
            W.ysp_host = W.Js.p;
        }
        nks_newton_stats S{};
        const long waits0 = host_waits();
        double t0 = now();
        // residual and norms at the initial guess
        HIPC(hipMemsetAsync(g.flags.p, 0, sizeof(int) * B, s));
        launch_history(g, pn, pnm1, order);
        std::vector<double> hn(B), hs(B), ht(B), hslope(B), lam(B), lam_prev(B), f_prev(B), stop(B);
        std::vector<int> act(B), flags(B), acc(B), why(B, 0);
        // per-reservoir norms and non-physical flags: one round trip through
        // pinned memory (it also completes any copy queued before it)
        auto norms = [&](const double *x, std::vector<double> &out) {
            launch_block_norm2(g.sp, W.red, x, W.red2.p, nullptr, s);
            HIPC(hipMemcpyAsync(W.h_norm, W.red2.p, 8 * B, hipMemcpyDeviceToHost, s));
            HIPC(hipMemcpyAsync(W.h_flags, g.flags.p, 4 * B, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            count_host_wait();
            for (int b = 0; b < B; ++b) {
                out[b] = std::sqrt(W.h_norm[b]);
                flags[b] = W.h_flags[b];
            }
        };
        // the host copies are staged in pinned memory; every upload is
        // followed by a round trip before its staging slot is written again
        auto upload_mask = [&]() {
            for (int b = 0; b < B; ++b) W.h_mask[b] = act[b];
            HIPC(hipMemcpyAsync(W.mask.p, W.h_mask, 4 * B, hipMemcpyHostToDevice, s));
        };
        launch_props(g, p);
        launch_flux(g, p, dt, order, W.F.p, nullptr);
        norms(W.F.p, hn);
        const std::vector<double> f0 = hn;
        S.t_residual += now() - t0;
        for (int b = 0; b < B; ++b) {
            if (flags[b] || !std::isfinite(hn[b])) fail(NKS_ENONPHYSICAL, "reservoir %d: non-physical initial state", b);
            stop[b] = std::max(nd->eps_r * hn[b], nd->eps_a);
            act[b] = hn[b] > stop[b];
            if (!act[b]) why[b] = NKS_STOP_TOL;
            S.fnorm0 = std::max(S.fnorm0, hn[b]);
        }
        int status = 0;
        int k = 0;
        for (; k < nd->max_newton; ++k) {
            bool any = false;
            for (int b = 0; b < B; ++b) any |= act[b] != 0;
            if (!any) break;
            upload_mask();
            double t1 = now();
            {
                ProfScope ps("residual_jacobian", s);
                launch_flux(g, p, dt, order, nullptr, W.J->op.coef.p);   // props at p are current
                if (rd->coarse_op == NKS_COARSE_REDISCRETIZED) remember_state(*W.J, p, dt, order);
            }
            // rounding floor: ||F|| <= u || |J| |p| || means p solves F = 0 as
            // well as F can be evaluated in binary64
            if (nd->floor_test) {
                launch_spmv_abs(W.J->op, p, W.Js.p, s);
                std::vector<double> fl(B);
                norms(W.Js.p, fl);
                bool changed = false, left = false;
                for (int b = 0; b < B; ++b) {
                    if (act[b] && hn[b] <= std::ldexp(fl[b], -53)) {
                        act[b] = 0;
                        why[b] = NKS_STOP_FLOOR;
                        changed = true;
                    }
                    left |= act[b] != 0;
                }
                if (!left) break;
                if (changed) upload_mask();
            }
            double t2 = now();
            S.t_jacobian += t2 - t1;
            // coarse operators, and the subdomain factors every lag-th
            // iteration (in between the last factors are kept); zero pivots
            // are read back after the solve (with its stats)
            W.M->factor(nd->lag <= 1 || k % nd->lag == 0);
            double t3 = now();
            S.t_setup += t3 - t2;
            // J s = -F on the active reservoirs
            k_neg<<<nblk(N, 256), 256, 0, s>>>(N, W.F.p, W.b.p);
            k_zero<<<nblk(N, 256), 256, 0, s>>>(N, W.s.p);
            MatVec A = [&](const double *xx, double *yy, const double *bb, const int *mk) {
                launch_spmv(W.J->op, xx, yy, bb, mk, s);
            };
            Precond P = [&](const double *r, double *z, const int *mk) { W.M->apply(r, z, mk); };
            GmOpts o;
            o.rtol = nd->eta_r;
            o.atol = nd->eta_a;
            o.maxit = nd->maxit;
            o.flexible = flex;
            o.check_every = 1;
            // a preconditioner without host round trips is captured with the
            // Arnoldi step, two iterations per graph
            o.graph_chunk = W.M->capturable() ? 2 : 0;
            W.gm.solve(A, P, W.b.p, W.s.p, true, o, W.mask.p, s, &W.J->op);
            S.graph_chunk = W.gm.gchunk;
            std::vector<int> its, conv;
            std::vector<double> res;
            W.gm.stats(its, res, conv, s);
            W.M->check_pivots();
            int lits = 0;
            for (int b = 0; b < B; ++b) if (act[b]) lits = std::max(lits, its[b]);
            S.linear_its += lits;
            if (k < 64) S.lits[k] = lits;
            double t4 = now();
            S.t_gmres += t4 - t3;
            // relative step test on the full Newton step: a step this small is
            // taken as it is (lambda = 1, no decrease test, since at the
            // rounding floor ||F|| cannot decrease) and the reservoir stops
            std::vector<double> snorm(B, 0.0), xnorm(B, 0.0);
            std::vector<int> small(B, 0);
            if (nd->stol > 0.0) {
                norms(W.s.p, snorm);
                norms(p, xnorm);
                for (int b = 0; b < B; ++b) small[b] = act[b] && snorm[b] <= nd->stol * xnorm[b];
            }
            // slope of f = ||F||^2/2 along s: F^T J s, read back with the
            // first trial norm (no round trip of its own)
            launch_spmv(W.J->op, W.s.p, W.Js.p, nullptr, nullptr, s);
            launch_block_dots(g.sp, W.red, W.F.p, W.ysp.p, 1, W.red2.p + B, nullptr, s);
            HIPC(hipMemcpyAsync(W.h_slope, W.red2.p + B, 8 * B, hipMemcpyDeviceToHost, s));
            // backtracking (Dennis-Schnabel): lambda = 1, then quadratic, then
            // cubic models, each new lambda within [0.1, 0.5] of the last
            for (int b = 0; b < B; ++b) {
                lam[b] = act[b] ? 1.0 : 0.0;
                acc[b] = act[b] ? 0 : 1;
            }
            int bt = 0;
            bool failed = false;
            for (;; ++bt) {
                for (int b = 0; b < B; ++b) W.h_lam[b] = lam[b];
                HIPC(hipMemcpyAsync(W.lam.p, W.h_lam, 8 * B, hipMemcpyHostToDevice, s));
                k_trial<<<(int)g.sp.htile.size(), TILE, 0, s>>>(g.sp.tile.p, p, W.s.p, W.lam.p, W.pt.p);
                HIPC(hipMemsetAsync(g.flags.p, 0, sizeof(int) * B, s));
                launch_props(g, W.pt.p);
                launch_flux(g, W.pt.p, dt, order, W.Ft.p, nullptr);
                norms(W.Ft.p, ht);
                if (bt == 0)
                    for (int b = 0; b < B; ++b) hslope[b] = W.h_slope[b];
                bool all = true;
                for (int b = 0; b < B; ++b) {
                    if (acc[b]) continue;
                    const double fx = 0.5 * hn[b] * hn[b];
                    const bool bad = flags[b] || !std::isfinite(ht[b]);
                    if (!bad && ((small[b] && bt == 0) || ht[b] <= (1.0 - nd->alpha * lam[b]) * hn[b])) {
                        acc[b] = 1;
                        continue;
                    }
                    if (bt >= nd->max_backtracks) {
                        failed = true;
                        acc[b] = 1;
                        continue;
                    }
                    all = false;
                    const double ft = bad ? INFINITY : 0.5 * ht[b] * ht[b];
                    const double sl = hslope[b];
                    double lt;
                    if (!std::isfinite(ft) || sl >= 0.0) {
                        lt = 0.5 * lam[b];
                    } else if (bt == 0) {
                        lt = -sl / (2.0 * (ft - fx - sl));
                    } else {
                        const double l1 = lam[b], l2 = lam_prev[b];
                        const double t1v = ft - fx - l1 * sl, t2v = f_prev[b] - fx - l2 * sl;
                        const double ca = (t1v / (l1 * l1) - t2v / (l2 * l2)) / (l1 - l2);
                        const double cb = (-l2 * t1v / (l1 * l1) + l1 * t2v / (l2 * l2)) / (l1 - l2);
                        if (ca == 0.0) lt = -sl / (2.0 * cb);
                        else {
                            const double disc = cb * cb - 3.0 * ca * sl;
                            lt = disc >= 0.0 ? (-cb + std::sqrt(disc)) / (3.0 * ca) : 0.5 * l1;
                        }
                    }
                    if (!(lt <= 0.5 * lam[b])) lt = 0.5 * lam[b];
                    if (!(lt >= 0.1 * lam[b])) lt = 0.1 * lam[b];
                    lam_prev[b] = lam[b];
                    f_prev[b] = ft;
                    lam[b] = lt;
                }
                if (all || failed) break;
            }
            double minlam = 1.0;
            for (int b = 0; b < B; ++b) if (act[b]) minlam = std::min(minlam, lam[b]);
            if (failed) {
                status = 2;
                S.newton_its = k + 1;
                break;
            }
            // accept: p, F <- trial values on the active reservoirs
            k_copy_mask<<<(int)g.sp.htile.size(), TILE, 0, s>>>(g.sp.tile.p, W.pt.p, p, W.mask.p);
            k_copy_mask<<<(int)g.sp.htile.size(), TILE, 0, s>>>(g.sp.tile.p, W.Ft.p, W.F.p, W.mask.p);
            if (nd->stol > 0.0) norms(p, xnorm);
            double fmax = 0.0;
            for (int b = 0; b < B; ++b) {
                if (act[b]) {
                    hn[b] = ht[b];
                    if (hn[b] <= stop[b]) { act[b] = 0; why[b] = NKS_STOP_TOL; }
                    else if (small[b] && lam[b] == 1.0) { act[b] = 0; why[b] = NKS_STOP_STEP; }
                    if (act[b] && nd->stol > 0.0 && lam[b] * snorm[b] <= nd->stol * xnorm[b]) {
                        act[b] = 0;
                        why[b] = NKS_STOP_STEP;
                    }
                }
                fmax = std::max(fmax, hn[b]);
            }
            // props must describe the accepted p for the next Jacobian
            launch_props(g, p);
            S.t_linesearch += now() - t4;
            if (k < 64) {
                S.fnorms[k] = fmax;
                S.lambdas[k] = minlam;
            }
            S.newton_its = k + 1;
        }
        if (status == 0) {
            for (int b = 0; b < B; ++b) if (act[b]) status = 1;
        }
        S.fnorm = 0.0;
        for (int b = 0; b < B; ++b) S.fnorm = std::max(S.fnorm, hn[b]);
        S.status = status;
        HIPC(hipStreamSynchronize(s));
        count_host_wait();
        S.host_waits = (int)(host_waits() - waits0);
        if (st) {
            S.stop_reason = st->stop_reason;
            S.rel_res = st->rel_res;
            for (int b = 0; b < B; ++b) {
                if (S.stop_reason) S.stop_reason[b] = why[b];
                if (S.rel_res) S.rel_res[b] = f0[b] > 0.0 ? hn[b] / f0[b] : 0.0;
            }
            *st = S;
        }
        if (status != 0) fail(NKS_ENOTCONVERGED, status == 2 ? "line search failed" : "Newton iteration limit");
    });
}

}  // extern "C"

// ------------------------------------------------------------------ discrete adjoint
int nks_adjoint(nks_grid *gh, int nsteps, const double *const *p_hist, const int *orders, double dt,
                const double *const *dGdp, const nks_ras_desc *rd, const nks_gmres_desc *gd, double *grad,
                double *const *lam_out, nks_adjoint_stats *st) {
    return guard([&] {
        if (!gh || nsteps < 1 || !p_hist || !orders || !(dt > 0) || !dGdp || !rd || !gd || !grad)
            fail(NKS_EINVAL, "bad arguments");
        if (gd->restart < 1 || gd->restart > 30 || gd->maxit < 1) fail(NKS_EINVAL, "bad GMRES descriptor");
        check_ras_desc(rd);
        if (gh->g.accum != NKS_ACCUM_CONSERVATIVE)
            fail(NKS_EINVAL, "the discrete adjoint is defined for the conservative accumulation only");
        for (int n = 0; n <= nsteps; ++n)
            if (!p_hist[n]) fail(NKS_EINVAL, "p_hist[%d] is null", n);
        for (int n = 1; n <= nsteps; ++n)
            if (orders[n - 1] != 1 && !(orders[n - 1] == 2 && n >= 2))
                fail(NKS_EINVAL, "step %d: order must be 1, or 2 from the second step on", n);
        Grid &g = gh->g;
        const int N = g.sp.N;
        hipStream_t s = g.s;
        Alloc *al = &g.al;
        if (!gh->aw) gh->aw.reset(new AdjointWork());
        AdjointWork &W = *gh->aw;
        if (!W.ready) {
            fine_matrix(W.J, g);
            W.rhs.alloc(al, N);
            for (auto &l : W.lam) l.alloc(al, N);
            W.ready = true;
        }
        W.gm.ensure(al, g.sp, gd->restart, gd->flexible != 0, s);
        nks_adjoint_stats S{};
        double t0 = now();
        // lam[n % 3] holds lambda_n; lambda_{n+1}, lambda_{n+2} are the two before it
        for (int n = nsteps; n >= 1; --n) {
            const double *l1 = n + 1 <= nsteps ? W.lam[(n + 1) % 3].p : nullptr;
            const double *l2 = n + 2 <= nsteps && orders[n + 1] == 2 ? W.lam[(n + 2) % 3].p : nullptr;
            const double c1 = n + 1 <= nsteps ? (orders[n] == 2 ? -2.0 : -1.0) : 0.0;
            launch_adj_rhs(g, p_hist[n], dt, c1, l1, 0.5, l2, dGdp[n], W.rhs.p);
            // J_n at the converged p^n (its accumulation coefficient depends on the order)
            launch_props(g, p_hist[n]);
            launch_flux(g, p_hist[n], dt, orders[n - 1], nullptr, W.J.op.coef.p);
            W.T.stale = true;
            W.T.refresh(W.J, *rd);
            Ras &MT = *W.T.MT;
            Matrix &JT = W.T.JT;
            double *lam = W.lam[n % 3].p;
            launch_axpby(g.sp, 0.0, W.rhs.p, 0.0, lam, nullptr, s);
            MatVec A = [&](const double *xx, double *yy, const double *bb, const int *mk) {
                launch_spmv(JT.op, xx, yy, bb, mk, s);
            };
            Precond P = [&](const double *r, double *z, const int *mk) { MT.apply(r, z, mk); };
            GmOpts o;
            o.rtol = gd->rtol;
            o.atol = gd->atol;
            o.maxit = gd->maxit;
            o.flexible = gd->flexible != 0;
            o.check_every = 1;
            W.gm.solve(A, P, W.rhs.p, lam, true, o, nullptr, s, &JT.op);
            std::vector<int> its, conv;
            std::vector<double> res;
            W.gm.stats(its, res, conv, s);
            int lits = 0, nconv = 0;
            for (int b = 0; b < g.sp.B; ++b) {
                lits = std::max(lits, its[b]);
                nconv += conv[b];
            }
            if (n - 1 < 64) S.linear_its[n - 1] = lits;
            S.total_linear_its += lits;
            if (nconv < g.sp.B) S.status = 1;
            if (lam_out && lam_out[n])
                HIPC(hipMemcpyAsync(lam_out[n], lam, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
            // dG/dln K += (dF^n/dln K)^T lambda_n
            launch_dlogk_t(g, p_hist[n], lam, grad, n != nsteps);
        }
        HIPC(hipStreamSynchronize(s));
        S.t_total = now() - t0;
        if (st) *st = S;
        if (S.status) fail(NKS_ENOTCONVERGED, "an adjoint linear solve did not converge");
    });
}

// ------------------------------------------------------------------ tile / overlap autotuner
int nks_ras_autotune(nks_grid *gh, const double *p, const double *pn, const double *pnm1, double dt, int order,
                     const nks_ras_desc *base, const int *tiles, int ntiles, const int *overlaps, int noverlaps,
                     const int *ratios, int nratios, const nks_gmres_desc *gd, int repeats, nks_ras_desc *best,
                     nks_autotune_entry *table) {
    return guard([&] {
        if (!gh || !p || !pn || !(dt > 0) || (order != 1 && order != 2) || (order == 2 && !pnm1) || !base ||
            !tiles || ntiles < 1 || !overlaps || noverlaps < 1 || !gd || !best || repeats < 1 ||
            (nratios > 0 && !ratios))
            fail(NKS_EINVAL, "bad arguments");
        const int base_ratio = base->ratio;
        if (nratios < 1) {
            ratios = &base_ratio;
            nratios = 1;
        }
        for (int i = 0; i < nratios; ++i)
            if (ratios[i] != 0 && (ratios[i] < 2 || ratios[i] > 16)) fail(NKS_EINVAL, "ratios must be 2..16");
        if (gd->restart < 1 || gd->restart > 30 || gd->maxit < 1) fail(NKS_EINVAL, "bad GMRES descriptor");
        check_ras_desc(base);
        for (int i = 0; i < ntiles; ++i)
            if (tiles[i] < 1) fail(NKS_EINVAL, "tile edges must be positive");
        for (int i = 0; i < noverlaps; ++i)
            if (overlaps[i] < 0) fail(NKS_EINVAL, "overlaps must be non-negative");
        Grid &g = gh->g;
        const int N = g.sp.N;
        hipStream_t s = g.s;
        Alloc *al = &g.al;
        // the first Newton system at the given state: J s = -F
        Matrix J;
        fine_matrix(J, g);
        DBuf<double> F, b, x;
        F.alloc(al, N);
        b.alloc(al, N);
        x.alloc(al, N);
        launch_history(g, pn, pnm1 ? pnm1 : pn, order);
        launch_props(g, p);
        launch_flux(g, p, dt, order, F.p, J.op.coef.p);
        remember_state(J, p, dt, order);
        launch_axpby(g.sp, -1.0, F.p, 0.0, b.p, nullptr, s);
        Gmres gm;
        gm.ensure(al, g.sp, gd->restart, gd->flexible != 0, s);
        double best_t = INFINITY;
        int k = 0;
        bool any = false;
        for (int it = 0; it < ntiles; ++it) {
            for (int io = 0; io < noverlaps; ++io) for (int ir = 0; ir < nratios; ++ir, ++k) {
                nks_ras_desc d = *base;
                d.tx = d.ty = tiles[it];
                d.tz = g.dim == 3 ? tiles[it] : 0;
                for (int l = 0; l < 8; ++l) d.overlap[l] = overlaps[io];
                d.ratio = ratios[ir];
                nks_autotune_entry e{};
                e.tile = tiles[it];
                e.overlap = overlaps[io];
                e.ratio = ratios[ir] > 0 ? ratios[ir] : 2;
                e.ok = 0;
                try {
                    Ras M;
                    M.build(&J, d);
                    double t_setup = 0, t_solve = 0;
                    int its = 0;
                    // repeats + 1 runs, the first untimed (LDS attributes, first touch)
                    for (int r = 0; r <= repeats; ++r) {
                        HIPC(hipStreamSynchronize(s));
                        double t0 = now();
                        M.factor();
                        M.check_pivots();
                        HIPC(hipStreamSynchronize(s));
                        double t1 = now();
                        launch_axpby(g.sp, 0.0, b.p, 0.0, x.p, nullptr, s);
                        MatVec A = [&](const double *xx, double *yy, const double *bb, const int *mk) {
                            launch_spmv(J.op, xx, yy, bb, mk, s);
                        };
                        Precond P = [&](const double *rr, double *zz, const int *mk) { M.apply(rr, zz, mk); };
                        GmOpts o;
                        o.rtol = gd->rtol;
                        o.atol = gd->atol;
                        o.maxit = gd->maxit;
                        o.flexible = gd->flexible != 0;
                        gm.solve(A, P, b.p, x.p, true, o, nullptr, s, &J.op);
                        std::vector<int> itv, conv;
                        std::vector<double> res;
                        gm.stats(itv, res, conv, s);
                        double t2 = now();
                        if (r > 0) {
                            t_setup += t1 - t0;
                            t_solve += t2 - t1;
                        }
                        its = 0;
                        for (int q = 0; q < g.sp.B; ++q) its = std::max(its, itv[q]);
                    }
                    e.setup_ms = 1e3 * t_setup / repeats;
                    e.solve_ms = 1e3 * t_solve / repeats;
                    e.iterations = its;
                    e.ok = 1;
                    const double t = e.setup_ms + e.solve_ms;
                    if (t < best_t) {
                        best_t = t;
                        *best = d;
                        any = true;
                    }
                } catch (const Error &err) {
                    (void)hipGetLastError();
                    (void)hipStreamSynchronize(s);
                }
                if (table) table[k] = e;
            }
        }
        if (!any) fail(NKS_EINVAL, "no candidate tile/overlap could be set up");
    });
}
