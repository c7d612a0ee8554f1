// (F)GMRES device state and host driver.
#pragma once

#include <functional>
#include <map>
#include <tuple>

#include "nks_internal.h"

namespace nks {

// y = A x (b == nullptr) or y = b - A x; only blocks with mask[b] != 0 when mask given
using MatVec = std::function<void(const double *x, double *y, const double *b, const int *mask)>;
// z = M^{-1} r on blocks with mask[b] != 0
using Precond = std::function<void(const double *r, double *z, const int *mask)>;


struct GmDev {
    double *H;
    double *cs, *sn;
    double *g;
    double *y;
    double *hj;
    double *tol, *beta, *res;
    int *active, *conv, *kdim, *its, *upd;
    int *active2;     // second activity buffer: iteration j reads buffer j%2, writes the other
    int *flag;        // host-mapped, m + 1 slots of nb: iteration j's activity (slot j), a cycle's start (slot m)
    int nb;
    int m, maxit;
    double rtol, atol;
};


struct GmOpts {
    double rtol = 1e-5, atol = 1e-8;
    int maxit = 10000;
    bool flexible = false;
    int check_every = 1;
    int graph_chunk = 0;   // > 0: replay captured chunks of this many iterations (A and M must be capturable)
    bool single_pass = false;   // classical Gram-Schmidt without reorthogonalisation (loose solves)
};

struct Gmres {
    Alloc *al = nullptr;
    const Space *sp = nullptr;
    int m = 0, nb = 0, nn = 0;
    struct Col {
        double *p = nullptr;   // a column of Vall
    };
    DBuf<double> Vall;         // Krylov basis, (m + 1) columns of stride ld
    long ld = 0;
    std::vector<Col> V;
    std::vector<DBuf<double>> Z;
    DBuf<double> w, r, t, H, cs, sn, g, y, hj, scal;
    DBuf<int> ints;
    DBuf<const double *> vptr, zptr;
    Reducer red;
    int *hint = nullptr;
    volatile int *hflag = nullptr;   // mapped pinned flags (host view)
    int *dflag = nullptr;            // device view
    int flag_b = 0, flag_m = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // captured iteration chunks [j0, j1) (valid while the buffers behind A and M are)
    std::map<std::pair<int, int>, hipGraphExec_t> gexec;
    int gchunk = 0;
    // what the captured kernels hold by value besides the buffers: the
    // iteration limit, the Gram-Schmidt form, flexibility, the operator
    std::tuple<int, int, int, const void *> gkey{-1, -1, -1, nullptr};
    bool graphs_ok = true;
    void invalidate_graphs();

    void ensure(Alloc *al, const Space &sp, int m, bool flexible, hipStream_t s);
    GmDev dev(double rtol, double atol, int maxit);
    bool any_active(hipStream_t s);
    // x: initial guess unless x_zero (then x must already hold zeros).  Aop:
    // the stencil operator behind A, when it is one (fuses the product with
    // the first Gram-Schmidt pass); A is still used for residuals.
    void solve(const MatVec &A, const Precond &M, const double *b, double *x, bool x_zero,
               const GmOpts &o, const int *outer_mask, hipStream_t s, const Op *Aop = nullptr);
    void stats(std::vector<int> &its, std::vector<double> &res, std::vector<int> &conv,
               hipStream_t s);
    ~Gmres();
};

}  // namespace nks
