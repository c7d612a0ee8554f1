// Stencil SpMV, per-reservoir reductions and right-preconditioned
// GMRES / FGMRES(m) (Section 3, eq. jacobian; Remark 2 for the flexible
// variant).  Orthogonalisation is classical Gram-Schmidt with one
// reorthogonalisation pass (two fused multi-dot + update passes), FP64.
// Every reduction is deterministic: per-chunk partial sums, then a fixed-
// order sum per reservoir done by the last workgroup to finish.
#include <functional>

#include "krylov.h"

namespace nks {

static inline int nblk(int n, int t) { return (n + t - 1) / t; }

// ---------------------------------------------------------------- spaces
void Space::build(Alloc *al, const std::vector<Blk> &b, hipStream_t s) {
    hblk = b;
    B = (int)b.size();
    N = 0;
    hchunk.clear();
    hcfirst.assign(B + 1, 0);
    for (int k = 0; k < B; ++k) {
        hblk[k].off = N;
        const int n = b[k].nx * b[k].ny * b[k].nz;
        hcfirst[k] = (int)hchunk.size();
        for (int c = 0; c < n; c += CHUNK) hchunk.push_back({k, N + c, N + std::min(n, c + CHUNK), 0});
        N += n;
    }
    hcfirst[B] = (int)hchunk.size();
    blk.upload(al, hblk, s);
    chunk.upload(al, hchunk, s);
    cfirst.upload(al, hcfirst, s);
}

void Reducer::ensure(Alloc *al, const Space &sp, int cols, hipStream_t s) {
    const size_t need = (size_t)sp.hchunk.size() * std::max(cols, 1);
    if (part.n < need) part.alloc(al, need);
    if (!counter.p) {
        counter.alloc(al, 1);
        HIPC(hipMemsetAsync(counter.p, 0, sizeof(unsigned), s));
    }
    maxcols = std::max(maxcols, cols);
}

// ---------------------------------------------------------------- stencil SpMV
struct SpmvArgs {
    const Blk *blk;
    int B, N, K;
    const int8_t *off;
    const double *coef;
    const double *x, *b;
    double *y;
    const int *mask;
};

__global__ void k_spmv(SpmvArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int bi = find_blk(a.blk, a.B, i);
    if (a.mask && !a.mask[bi]) return;
    const Blk k = a.blk[bi];
    const int l = i - k.off;
    const int x = l % k.nx, y = (l / k.nx) % k.ny, z = l / (k.nx * k.ny);
    double s = 0.0;
    for (int q = 0; q < a.K; ++q) {
        const int dx = a.off[3 * q], dy = a.off[3 * q + 1], dz = a.off[3 * q + 2];
        const int xx = x + dx, yy = y + dy, zz = z + dz;
        if (xx < 0 || xx >= k.nx || yy < 0 || yy >= k.ny || zz < 0 || zz >= k.nz) continue;
        s += a.coef[(size_t)q * a.N + i] * a.x[i + dx + k.nx * (dy + k.ny * dz)];
    }
    a.y[i] = a.b ? a.b[i] - s : s;
}

// y = A^T x: y_i = sum_q A[opp(q)][i + off_q] x[i + off_q]
__global__ void k_spmv_t(SpmvArgs a, const int *opp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int bi = find_blk(a.blk, a.B, i);
    const Blk k = a.blk[bi];
    const int l = i - k.off;
    const int x = l % k.nx, y = (l / k.nx) % k.ny, z = l / (k.nx * k.ny);
    double s = 0.0;
    for (int q = 0; q < a.K; ++q) {
        const int dx = a.off[3 * q], dy = a.off[3 * q + 1], dz = a.off[3 * q + 2];
        const int xx = x + dx, yy = y + dy, zz = z + dz;
        if (xx < 0 || xx >= k.nx || yy < 0 || yy >= k.ny || zz < 0 || zz >= k.nz) continue;
        const int j = i + dx + k.nx * (dy + k.ny * dz);
        s += a.coef[(size_t)opp[q] * a.N + j] * a.x[j];
    }
    a.y[i] = s;
}

static SpmvArgs spmv_args(const Op &A, const double *x, double *y, const double *b, const int *mask) {
    SpmvArgs a;
    a.blk = A.sp->blk.p;
    a.B = A.sp->B;
    a.N = A.sp->N;
    a.K = A.st.K;
    a.off = A.st.doff.p;
    a.coef = A.coef.p;
    a.x = x;
    a.b = b;
    a.y = y;
    a.mask = mask;
    return a;
}

void launch_spmv(const Op &A, const double *x, double *y, const double *b, const int *mask,
                 hipStream_t s) {
    SpmvArgs a = spmv_args(A, x, y, b, mask);
    ProfScope ps("spmv", s, A.st.K <= 7 ? 0 : 1);
    k_spmv<<<nblk(a.N, 256), 256, 0, s>>>(a);
    KCHECK();
}

void launch_spmv_t(const Op &A, const double *x, double *y, const int *opp, hipStream_t s) {
    SpmvArgs a = spmv_args(A, x, y, nullptr, nullptr);
    k_spmv_t<<<nblk(a.N, 256), 256, 0, s>>>(a, opp);
    KCHECK();
}

// ---------------------------------------------------------------- elementwise
__global__ void k_axpby(const Blk *blk, int B, int N, double a, const double *x, double b,
                        double *y, const int *mask) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (mask && !mask[find_blk(blk, B, i)]) return;
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

void launch_axpby(const Space &sp, double a, const double *x, double b, double *y, const int *mask,
                  hipStream_t s) {
    k_axpby<<<nblk(sp.N, 256), 256, 0, s>>>(sp.blk.p, sp.B, sp.N, a, x, b, y, mask);
    KCHECK();
}

// y = x * scale[blk] (per-block factor), or y = x / scale[blk] when inv
__global__ void k_scale_blk(const Blk *blk, int B, int N, const double *x, const double *scale,
                            int stride, int col, int inv, double *y, const int *mask) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    if (mask && !mask[b]) return;
    const double f = scale[(size_t)b * stride + col];
    y[i] = inv ? x[i] / f : x[i] * f;
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v, double *sh) {
    // wavefront reduce by shuffles, then across the (<= 4) wavefronts
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 0; k < nw; ++k) t += sh[k];
    }
    return t;   // valid in thread 0
}

__device__ __forceinline__ double coherent_load(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the last workgroup to arrive.
__device__ __forceinline__ bool last_block(unsigned *counter, int nblocks) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(counter, 1u);
        is_last = (t == (unsigned)(nblocks - 1));
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

// Final per-block sums of `cols` partial columns into out[b*cols + c]; the
// last workgroup calls this, then resets the counter.
__device__ void finish_sums(const Chunk *, const int *cfirst, int B, int cols, const double *part,
                            double *out) {
    for (int t = threadIdx.x; t < B * cols; t += blockDim.x) {
        const int b = t / cols, c = t % cols;
        double s = 0.0;
        for (int q = cfirst[b]; q < cfirst[b + 1]; ++q) s += coherent_load(&part[(size_t)q * cols + c]);
        out[t] = s;
    }
}

// dots of x with ncols vectors ys[c] per block: out[b*ncols + c]
__global__ void k_block_dots(const Chunk *chunks, int nch, const int *cfirst, int B,
                             const double *x, const double *const *ys, int ncols, double *part,
                             unsigned *counter, double *out, const int *mask, int square) {
    __shared__ double sh[8];
    const Chunk ch = chunks[blockIdx.x];
    const bool on = !mask || mask[ch.blk];
    for (int c = 0; c < ncols; ++c) {
        double v = 0.0;
        if (on) {
            const double *y = square ? x : ys[c];
            for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) v += x[i] * y[i];
        }
        v = block_sum(v, sh);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * ncols + c] = v;
    }
    if (last_block(counter, nch)) {
        finish_sums(chunks, cfirst, B, ncols, part, out);
        __syncthreads();
        if (threadIdx.x == 0) *counter = 0u;
    }
}

void launch_block_dots(const Space &sp, Reducer &R, const double *x, const double *const *ys,
                       int ncols, double *out, const int *mask, hipStream_t s) {
    k_block_dots<<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(
        sp.chunk.p, (int)sp.hchunk.size(), sp.cfirst.p, sp.B, x, ys, ncols, R.part.p,
        R.counter.p, out, mask, 0);
    KCHECK();
}

void launch_block_norm2(const Space &sp, Reducer &R, const double *x, double *out, const int *mask,
                        hipStream_t s) {
    k_block_dots<<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(
        sp.chunk.p, (int)sp.hchunk.size(), sp.cfirst.p, sp.B, x, nullptr, 1, R.part.p,
        R.counter.p, out, mask, 1);
    KCHECK();
}

// ---------------------------------------------------------------- GMRES kernels

// ||r||^2 per block -> epilogue decides who iterates in the new cycle.
// set_tol: r == b (x0 = 0) so the same norm also sets tol = max(rtol||b||, atol).
__global__ void k_gm_start(const Chunk *chunks, int nch, const int *cfirst, int B, const double *r,
                           double *part, unsigned *counter, GmDev st, const int *outer,
                           int set_tol, int first) {
    __shared__ double sh[8];
    const Chunk ch = chunks[blockIdx.x];
    double v = 0.0;
    for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) v += r[i] * r[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
    if (last_block(counter, nch)) {
        for (int b = threadIdx.x; b < B; b += blockDim.x) {
            double s = 0.0;
            for (int q = cfirst[b]; q < cfirst[b + 1]; ++q) s += coherent_load(&part[q]);
            const double beta = sqrt(s);
            if (first) {
                st.its[b] = 0;
                st.conv[b] = (outer && !outer[b]) ? 1 : 0;
            }
            if (set_tol) st.tol[b] = fmax(st.rtol * beta, st.atol);
            st.beta[b] = beta;
            st.res[b] = beta;
            st.kdim[b] = 0;
            for (int k = 0; k <= st.m; ++k) st.g[(size_t)b * (st.m + 1) + k] = 0.0;
            st.g[(size_t)b * (st.m + 1)] = beta;
            int act = 0;
            if (!st.conv[b]) {
                if (beta <= st.tol[b]) st.conv[b] = 1;
                else if (st.its[b] < st.maxit) act = 1;
            }
            st.active[b] = act;
        }
        __syncthreads();
        if (threadIdx.x == 0) *counter = 0u;
    }
}

// tol from ||b|| (when x0 != 0)
__global__ void k_gm_tol(const Chunk *chunks, int nch, const int *cfirst, int B, const double *bv,
                         double *part, unsigned *counter, GmDev st) {
    __shared__ double sh[8];
    const Chunk ch = chunks[blockIdx.x];
    double v = 0.0;
    for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) v += bv[i] * bv[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
    if (last_block(counter, nch)) {
        for (int b = threadIdx.x; b < B; b += blockDim.x) {
            double s = 0.0;
            for (int q = cfirst[b]; q < cfirst[b + 1]; ++q) s += coherent_load(&part[q]);
            st.tol[b] = fmax(st.rtol * sqrt(s), st.atol);
        }
        __syncthreads();
        if (threadIdx.x == 0) *counter = 0u;
    }
}

// Pass of classical Gram-Schmidt on column j: h = V[0..j]^T w (per block),
// accumulated into H[:, j] (first pass overwrites).
__global__ void k_gm_dots(const Chunk *chunks, int nch, const int *cfirst, int B, const double *w,
                          const double *const *V, int j, double *part, unsigned *counter, GmDev st,
                          int first_pass) {
    __shared__ double sh[8];
    const Chunk ch = chunks[blockIdx.x];
    const bool on = st.active[ch.blk];
    const int nc = j + 1;
    for (int c = 0; c < nc; ++c) {
        double v = 0.0;
        if (on) {
            const double *vc = V[c];
            for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) v += w[i] * vc[i];
        }
        v = block_sum(v, sh);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * nc + c] = v;
    }
    if (last_block(counter, nch)) {
        for (int t = threadIdx.x; t < B * nc; t += blockDim.x) {
            const int b = t / nc, c = t % nc;
            if (!st.active[b]) continue;
            double s = 0.0;
            for (int q = cfirst[b]; q < cfirst[b + 1]; ++q) s += coherent_load(&part[(size_t)q * nc + c]);
            st.hj[(size_t)b * (st.m + 1) + c] = s;
            double &h = st.H[((size_t)b * (st.m + 1) + c) * st.m + j];
            h = first_pass ? s : h + s;
        }
        __syncthreads();
        if (threadIdx.x == 0) *counter = 0u;
    }
}

// w -= sum_c hj[c] V[c]; on the last pass also ||w||^2, then the Givens step.
__global__ void k_gm_update(const Chunk *chunks, int nch, const int *cfirst, int B, double *w,
                            const double *const *V, int j, double *part, unsigned *counter,
                            GmDev st, int last_pass) {
    __shared__ double sh[8];
    __shared__ double hc[32];
    const Chunk ch = chunks[blockIdx.x];
    const bool on = st.active[ch.blk];
    const int nc = j + 1;
    if (threadIdx.x < nc && on) hc[threadIdx.x] = st.hj[(size_t)ch.blk * (st.m + 1) + threadIdx.x];
    __syncthreads();
    double v = 0.0;
    if (on) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double t = w[i];
            for (int c = 0; c < nc; ++c) t -= hc[c] * V[c][i];
            w[i] = t;
            v += t * t;
        }
    }
    if (!last_pass) return;
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
    if (last_block(counter, nch)) {
        for (int b = threadIdx.x; b < B; b += blockDim.x) {
            if (!st.active[b]) continue;
            double s = 0.0;
            for (int q = cfirst[b]; q < cfirst[b + 1]; ++q) s += coherent_load(&part[q]);
            const double hn = sqrt(s);
            const int m = st.m;
            double *H = st.H + (size_t)b * (m + 1) * m;
            double *cs = st.cs + (size_t)b * m, *sn = st.sn + (size_t)b * m;
            double *g = st.g + (size_t)b * (m + 1);
            H[(j + 1) * m + j] = hn;
            for (int k = 0; k < j; ++k) {
                const double a0 = H[k * m + j], a1 = H[(k + 1) * m + j];
                H[k * m + j] = cs[k] * a0 + sn[k] * a1;
                H[(k + 1) * m + j] = -sn[k] * a0 + cs[k] * a1;
            }
            const double a0 = H[j * m + j], a1 = hn;
            const double den = sqrt(a0 * a0 + a1 * a1);
            cs[j] = den > 0.0 ? a0 / den : 1.0;
            sn[j] = den > 0.0 ? a1 / den : 0.0;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            st.its[b] += 1;
            st.kdim[b] = j + 1;
            st.hj[(size_t)b * (m + 1) + m] = hn;   // for the normalisation of v_{j+1}
            const double res = fabs(g[j + 1]);
            st.res[b] = res;
            if (res <= st.tol[b] || hn == 0.0) {
                st.conv[b] = 1;
                st.active[b] = 0;
            } else if (st.its[b] >= st.maxit || j + 1 == m) {
                st.active[b] = 0;   // restart (or stop at maxit)
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) *counter = 0u;
    }
}

// v_{j+1} = w / h_{j+1,j} for blocks still iterating
__global__ void k_gm_next(const Blk *blk, int B, int N, const double *w, double *vn, GmDev st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    if (!st.active[b]) return;
    vn[i] = w[i] / st.hj[(size_t)b * (st.m + 1) + st.m];
}

// v_0 = r / beta for blocks iterating in this cycle
__global__ void k_gm_v0(const Blk *blk, int B, int N, const double *r, double *v0, GmDev st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    if (!st.active[b]) return;
    v0[i] = r[i] / st.beta[b];
}

// back substitution H y = g over the kdim leading columns of each block
__global__ void k_gm_solve_y(int B, GmDev st) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int m = st.m, k = st.kdim[b];
    const double *H = st.H + (size_t)b * (m + 1) * m;
    const double *g = st.g + (size_t)b * (m + 1);
    double *y = st.y + (size_t)b * m;
    for (int r = k - 1; r >= 0; --r) {
        double s = g[r];
        for (int c = r + 1; c < k; ++c) s -= H[r * m + c] * y[c];
        y[r] = s / H[r * m + r];
    }
    st.upd[b] = k > 0;
}

// x += sum_{c < kdim} y[c] Zc   (or u = sum y[c] Vc when accumulate == 0)
__global__ void k_gm_combine(const Blk *blk, int B, int N, const double *const *Z, double *x,
                             GmDev st, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    const int k = st.kdim[b];
    if (k == 0) return;
    const double *y = st.y + (size_t)b * st.m;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += y[c] * Z[c][i];
    x[i] = accumulate ? x[i] + s : s;
}

// ---------------------------------------------------------------- host driver
void Gmres::ensure(Alloc *al_, const Space &sp_, int m_, bool flexible, hipStream_t s) {
    al = al_;
    sp = &sp_;
    const int B = sp_.B, N = sp_.N;
    if (m_ != m || B != nb || N != nn || (flexible && Z.empty())) {
        m = m_;
        nb = B;
        nn = N;
        V.clear();
        Z.clear();
        V.resize(m + 1);
        for (auto &v : V) v.alloc(al, N);
        if (flexible) {
            Z.resize(m);
            for (auto &z : Z) z.alloc(al, N);
        }
        w.alloc(al, N);
        r.alloc(al, N);
        t.alloc(al, N);
        H.alloc(al, (size_t)B * (m + 1) * m);
        cs.alloc(al, (size_t)B * m);
        sn.alloc(al, (size_t)B * m);
        g.alloc(al, (size_t)B * (m + 1));
        y.alloc(al, (size_t)B * m);
        hj.alloc(al, (size_t)B * (m + 1));
        scal.alloc(al, (size_t)B * 3);
        ints.alloc(al, (size_t)B * 5);
        std::vector<const double *> hv(m + 1), hz(std::max(m, 1));
        for (int k = 0; k <= m; ++k) hv[k] = V[k].p;
        for (int k = 0; k < (int)Z.size(); ++k) hz[k] = Z[k].p;
        if (Z.empty()) hz.assign(1, nullptr);
        vptr.upload(al, hv, s);
        zptr.upload(al, hz, s);
        if (hint) HIPC(hipHostFree(hint));
        HIPC(hipHostMalloc((void **)&hint, sizeof(int) * 2 * B + sizeof(double) * 2 * B));
    }
    red.ensure(al, sp_, m + 1, s);
}

Gmres::~Gmres() {
    if (hint) (void)hipHostFree(hint);
}

GmDev Gmres::dev(double rtol, double atol, int maxit) {
    GmDev d;
    const int B = nb;
    d.H = H.p; d.cs = cs.p; d.sn = sn.p; d.g = g.p; d.y = y.p; d.hj = hj.p;
    d.tol = scal.p; d.beta = scal.p + B; d.res = scal.p + 2 * B;
    d.active = ints.p; d.conv = ints.p + B; d.kdim = ints.p + 2 * B; d.its = ints.p + 3 * B;
    d.upd = ints.p + 4 * B;
    d.m = m;
    d.maxit = maxit;
    d.rtol = rtol;
    d.atol = atol;
    return d;
}

bool Gmres::any_active(hipStream_t s) {
    HIPC(hipMemcpyAsync(hint, ints.p, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b) if (hint[b]) return true;
    return false;
}

void Gmres::solve(const MatVec &A, const Precond &M, const double *b, double *x, bool x_zero,
                  const GmOpts &o, const int *outer_mask, hipStream_t s) {
    const Space &S = *sp;
    const int nch = (int)S.hchunk.size();
    GmDev st = dev(o.rtol, o.atol, o.maxit);
    const int NB = nblk(S.N, 256);
    // r = b - A x (or b), tol, norms
    const double *r0 = b;
    if (!x_zero) {
        k_gm_tol<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, nch, S.cfirst.p, S.B, b, red.part.p,
                                              red.counter.p, st);
        KCHECK();
        A(x, r.p, b, outer_mask);
        r0 = r.p;
    }
    k_gm_start<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, nch, S.cfirst.p, S.B, r0, red.part.p,
                                            red.counter.p, st, outer_mask, x_zero ? 1 : 0, 1);
    KCHECK();
    const double *const *Vp = vptr.p;
    const bool flex = o.flexible;
    int cycles = 0;
    while (any_active(s)) {
        k_gm_v0<<<NB, 256, 0, s>>>(S.blk.p, S.B, S.N, r0, V[0].p, st);
        KCHECK();
        for (int j = 0; j < m; ++j) {
            double *zj = flex ? Z[j].p : t.p;
            M(V[j].p, zj, st.active);
            A(zj, w.p, nullptr, st.active);
            ProfScope ps("gmres_orth", s);
            for (int pass = 0; pass < 2; ++pass) {
                k_gm_dots<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, nch, S.cfirst.p, S.B, w.p, Vp, j,
                                                      red.part.p, red.counter.p, st, pass == 0);
                KCHECK();
                k_gm_update<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, nch, S.cfirst.p, S.B, w.p, Vp,
                                                        j, red.part.p, red.counter.p, st, pass == 1);
                KCHECK();
            }
            k_gm_next<<<NB, 256, 0, s>>>(S.blk.p, S.B, S.N, w.p, V[j + 1].p, st);
            KCHECK();
            if (j + 1 < m && ((j + 1) % o.check_every == 0) && !any_active(s)) break;
        }
        k_gm_solve_y<<<nblk(S.B, 64), 64, 0, s>>>(S.B, st);
        KCHECK();
        if (flex) {
            k_gm_combine<<<NB, 256, 0, s>>>(S.blk.p, S.B, S.N, zptr.p, x, st, 1);
            KCHECK();
        } else {
            k_gm_combine<<<NB, 256, 0, s>>>(S.blk.p, S.B, S.N, Vp, w.p, st, 0);
            KCHECK();
            M(w.p, t.p, st.upd);
            // x += t on updated blocks
            launch_axpby(S, 1.0, t.p, 1.0, x, st.upd, s);
        }
        ++cycles;
        A(x, r.p, b, nullptr);
        r0 = r.p;
        k_gm_start<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, nch, S.cfirst.p, S.B, r0, red.part.p,
                                                red.counter.p, st, outer_mask, 0, 0);
        KCHECK();
    }
}

void Gmres::stats(std::vector<int> &its, std::vector<double> &res, std::vector<int> &conv,
                  hipStream_t s) {
    const int B = nb;
    std::vector<int> hi(5 * B);
    std::vector<double> hd(3 * B);
    HIPC(hipMemcpyAsync(hi.data(), ints.p, sizeof(int) * 5 * B, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(hd.data(), scal.p, sizeof(double) * 3 * B, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    its.assign(hi.begin() + 3 * B, hi.begin() + 4 * B);
    conv.assign(hi.begin() + B, hi.begin() + 2 * B);
    res.assign(hd.begin() + 2 * B, hd.begin() + 3 * B);
}

}  // namespace nks
