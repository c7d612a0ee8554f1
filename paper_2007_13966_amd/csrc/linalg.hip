// Stencil SpMV, per-reservoir reductions and right-preconditioned
// GMRES / FGMRES(m) (Section 3, the Jacobian system; Remark 2 for the flexible
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
        // at most MAXCH chunks per block, at least CHUNK cells each
        int nch = std::max(1, std::min(MAXCH, (n + CHUNK - 1) / CHUNK));
        const int cs = (n + nch - 1) / nch;
        hcfirst[k] = (int)hchunk.size();
        for (int c = 0; c < n; c += cs) hchunk.push_back({k, N + c, N + std::min(n, c + cs), 0});
        N += n;
    }
    hcfirst[B] = (int)hchunk.size();
    blk.upload(al, hblk, s);
    chunk.upload(al, hchunk, s);
    cfirst.upload(al, hcfirst, s);
}

void Reducer::ensure(Alloc *al, const Space &sp, int cols, hipStream_t s) {
    const size_t need = 2 * (size_t)sp.hchunk.size() * std::max(cols, 1);
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

// y = |A| |x| (the componentwise magnitude of the product)
__global__ void k_spmv_abs(SpmvArgs a) {
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
        s += fabs(a.coef[(size_t)q * a.N + i]) * fabs(a.x[i + dx + k.nx * (dy + k.ny * dz)]);
    }
    a.y[i] = s;
}

// AT = A^T on the same stencil: AT[q][i] = A[opp(q)][i + off_q] (zero where the
// neighbour is outside the reservoir)
__global__ void k_transpose_op(SpmvArgs a, const int *opp, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int bi = find_blk(a.blk, a.B, i);
    const Blk k = a.blk[bi];
    const int l = i - k.off;
    const int x = l % k.nx, y = (l / k.nx) % k.ny, z = l / (k.nx * k.ny);
    for (int q = 0; q < a.K; ++q) {
        const int dx = a.off[3 * q], dy = a.off[3 * q + 1], dz = a.off[3 * q + 2];
        const int xx = x + dx, yy = y + dy, zz = z + dz;
        double v = 0.0;
        if (xx >= 0 && xx < k.nx && yy >= 0 && yy < k.ny && zz >= 0 && zz < k.nz)
            v = a.coef[(size_t)opp[q] * a.N + i + dx + k.nx * (dy + k.ny * dz)];
        out[(size_t)q * a.N + i] = v;
    }
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
    launch_timed("spmv", A.st.K <= 7 ? 0 : 1, k_spmv, dim3(nblk(a.N, 256)), dim3(256), 0, s, a);
    KCHECK();
}

void launch_spmv_abs(const Op &A, const double *x, double *y, hipStream_t s) {
    SpmvArgs a = spmv_args(A, x, y, nullptr, nullptr);
    k_spmv_abs<<<nblk(a.N, 256), 256, 0, s>>>(a);
    KCHECK();
}

void launch_transpose_op(const Op &A, Op &AT, const int *opp, hipStream_t s) {
    SpmvArgs a = spmv_args(A, nullptr, nullptr, nullptr, nullptr);
    k_transpose_op<<<nblk(a.N, 256), 256, 0, s>>>(a, opp, AT.coef.p);
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
// Reductions run in two fixed-order stages with no grid-wide fence: a
// workgroup per chunk writes up to MAXCOL column partials (butterfly
// wavefront sums, then the waves in order); the next kernel's workgroups
// each reduce the partials of their own reservoir in their prologue (chunk q
// to thread q, butterfly, waves in order), so every workgroup of a reservoir
// obtains bitwise the same totals, independent of the other reservoirs.  The
// first chunk of each reservoir commits shared state.
constexpr int MAXCOL = 32;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// column sums of this workgroup's registers into part_row[0..nc)
__device__ __forceinline__ void chunk_columns(const double (&acc)[MAXCOL], int nc, double *part_row) {
    __shared__ double sh[4][MAXCOL];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < MAXCOL; ++c) {
        if (c < nc) {
            const double v = wave_sum(acc[c]);
            if (lane == 0) sh[w][c] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        double t = 0.0;
        const int nw = blockDim.x >> 6;
        for (int k = 0; k < nw; ++k) t += sh[k][threadIdx.x];
        part_row[threadIdx.x] = t;
    }
}

// totals of the nc partial columns of reservoir b (chunks [q0, q1), at most
// blockDim chunks) into out[0..nc) in LDS, visible to the whole workgroup
__device__ __forceinline__ void block_totals(const double *part, int q0, int q1, int nc, double *out) {
    __shared__ double sh[4][MAXCOL];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = q0 + (int)threadIdx.x;
    double v[MAXCOL];
#pragma unroll
    for (int c = 0; c < MAXCOL; ++c) v[c] = (c < nc && q < q1) ? part[(size_t)q * nc + c] : 0.0;
#pragma unroll
    for (int c = 0; c < MAXCOL; ++c) {
        if (c < nc) {
            const double t = wave_sum(v[c]);
            if (lane == 0) sh[w][c] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        double t = 0.0;
        const int nw = blockDim.x >> 6;
        for (int k = 0; k < nw; ++k) t += sh[k][threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// partial dots of x with ncols vectors ys[c] (or ||x||^2 when square)
__global__ void __launch_bounds__(RED_THREADS) k_partials(const Chunk *chunks, const double *x,
                                                          const double *const *ys, int ncols, double *part,
                                                          const int *mask, int square) {
    const Chunk ch = chunks[blockIdx.x];
    const bool on = !mask || mask[ch.blk];
    double acc[MAXCOL];
#pragma unroll
    for (int c = 0; c < MAXCOL; ++c) acc[c] = 0.0;
    if (on) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            const double xi = x[i];
            if (square) {
                acc[0] += xi * xi;
            } else {
#pragma unroll
                for (int c = 0; c < MAXCOL; ++c)
                    if (c < ncols) acc[c] += xi * ys[c][i];
            }
        }
    }
    chunk_columns(acc, ncols, part + (size_t)blockIdx.x * ncols);
}

// one workgroup per reservoir: out[b*ncols + c]
__global__ void __launch_bounds__(RED_THREADS) k_totals(const int *cfirst, const double *part, int ncols,
                                                        double *out) {
    __shared__ double tot[MAXCOL];
    const int b = blockIdx.x;
    block_totals(part, cfirst[b], cfirst[b + 1], ncols, tot);
    if ((int)threadIdx.x < ncols) out[(size_t)b * ncols + threadIdx.x] = tot[threadIdx.x];
}

void launch_block_dots(const Space &sp, Reducer &R, const double *x, const double *const *ys,
                       int ncols, double *out, const int *mask, hipStream_t s) {
    if (ncols > MAXCOL) fail(NKS_EINVAL, "at most %d columns per reduction", MAXCOL);
    k_partials<<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(sp.chunk.p, x, ys, ncols, R.part.p, mask, 0);
    KCHECK();
    k_totals<<<sp.B, RED_THREADS, 0, s>>>(sp.cfirst.p, R.part.p, ncols, out);
    KCHECK();
}

void launch_block_norm2(const Space &sp, Reducer &R, const double *x, double *out, const int *mask,
                        hipStream_t s) {
    k_partials<<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(sp.chunk.p, x, nullptr, 1, R.part.p, mask, 1);
    KCHECK();
    k_totals<<<sp.B, RED_THREADS, 0, s>>>(sp.cfirst.p, R.part.p, 1, out);
    KCHECK();
}

// ---------------------------------------------------------------- GMRES kernels
// Start of a cycle: beta = ||r|| per reservoir (from the norm partials), who
// iterates, and v_0 = r / beta.  set_tol: r == b (x0 = 0), so tol =
// max(rtol ||b||, atol) comes from the same norm.
__global__ void __launch_bounds__(RED_THREADS) k_gm_begin(const Chunk *chunks, const int *cfirst,
                                                          const double *part, const double *r, double *v0,
                                                          GmDev st, const int *outer, int set_tol, int first) {
    __shared__ double tot[MAXCOL];
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk;
    const int q0 = cfirst[b];
    block_totals(part, q0, cfirst[b + 1], 1, tot);
    const double beta = sqrt(tot[0]);
    const bool lead = (int)blockIdx.x == q0;
    const int its = first ? 0 : st.its[b];
    const int conv0 = first ? ((outer && !outer[b]) ? 1 : 0) : st.conv[b];
    const double tol = set_tol ? fmax(st.rtol * beta, st.atol) : st.tol[b];
    int conv = conv0, act = 0;
    if (!conv) {
        if (beta <= tol) conv = 1;
        else if (its < st.maxit) act = 1;
    }
    if (act)
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) v0[i] = r[i] / beta;
    if (lead && threadIdx.x == 0) {
        st.its[b] = its;
        st.conv[b] = conv;
        st.tol[b] = tol;
        st.beta[b] = beta;
        st.res[b] = beta;
        st.kdim[b] = 0;
        for (int k = 0; k <= st.m; ++k) st.g[(size_t)b * (st.m + 1) + k] = 0.0;
        st.g[(size_t)b * (st.m + 1)] = beta;
        st.active[b] = act;
        st.flag[3 * st.nb + b] = act;
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_gm_norm_partials(const Chunk *chunks, const double *r,
                                                                  double *part) {
    const Chunk ch = chunks[blockIdx.x];
    double acc[MAXCOL];
    acc[0] = 0.0;
    for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) acc[0] += r[i] * r[i];
    chunk_columns(acc, 1, part + blockIdx.x);
}

// tol from ||b|| (x0 != 0), lead chunk of each reservoir
__global__ void __launch_bounds__(RED_THREADS) k_gm_tol(const Chunk *chunks, const int *cfirst, const double *part,
                                                        GmDev st) {
    __shared__ double tot[MAXCOL];
    const Chunk ch = chunks[blockIdx.x];
    const int q0 = cfirst[ch.blk];
    if ((int)blockIdx.x != q0) return;
    block_totals(part, q0, cfirst[ch.blk + 1], 1, tot);
    if (threadIdx.x == 0) st.tol[ch.blk] = fmax(st.rtol * sqrt(tot[0]), st.atol);
}

// CGS pass 1 partials: V[0..j]^T w
__global__ void __launch_bounds__(RED_THREADS) k_gm_dots(const Chunk *chunks, const double *w,
                                                         const double *const *V, int j, double *part, GmDev st) {
    const Chunk ch = chunks[blockIdx.x];
    const int nc = j + 1;
    double acc[MAXCOL];
#pragma unroll
    for (int c = 0; c < MAXCOL; ++c) acc[c] = 0.0;
    if (st.active[ch.blk]) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < MAXCOL; ++c)
                if (c < nc) acc[c] += wi * V[c][i];
        }
    }
    chunk_columns(acc, nc, part + (size_t)blockIdx.x * nc);
}

// h1 = totals of pass 1 (lead chunk stores H[:, j] = h1); w -= V h1; pass 2 partials V^T w
__global__ void __launch_bounds__(RED_THREADS) k_gm_update_dots(const Chunk *chunks, const int *cfirst, double *w,
                                                                const double *const *V, int j,
                                                                const double *pin, double *pout, GmDev st) {
    __shared__ double hc[MAXCOL];
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk, nc = j + 1;
    const bool on = st.active[b];
    if (on) block_totals(pin, cfirst[b], cfirst[b + 1], nc, hc);
    if (on && (int)blockIdx.x == cfirst[b] && (int)threadIdx.x < nc)
        st.H[((size_t)b * (st.m + 1) + threadIdx.x) * st.m + j] = hc[threadIdx.x];
    double acc[MAXCOL];
#pragma unroll
    for (int c = 0; c < MAXCOL; ++c) acc[c] = 0.0;
    if (on) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double vv[MAXCOL];
            double t = w[i];
#pragma unroll
            for (int c = 0; c < MAXCOL; ++c)
                if (c < nc) {
                    vv[c] = V[c][i];
                    t -= hc[c] * vv[c];
                }
            w[i] = t;
#pragma unroll
            for (int c = 0; c < MAXCOL; ++c)
                if (c < nc) acc[c] += t * vv[c];
        }
    }
    chunk_columns(acc, nc, pout + (size_t)blockIdx.x * nc);
}

// h2 = totals of pass 2 (lead chunk adds to H[:, j]); w -= V h2; ||w||^2 partials
__global__ void __launch_bounds__(RED_THREADS) k_gm_update_norm(const Chunk *chunks, const int *cfirst, double *w,
                                                                const double *const *V, int j,
                                                                const double *pin, double *pout, GmDev st) {
    __shared__ double hc[MAXCOL];
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk, nc = j + 1;
    const bool on = st.active[b];
    if (on) block_totals(pin, cfirst[b], cfirst[b + 1], nc, hc);
    if (on && (int)blockIdx.x == cfirst[b] && (int)threadIdx.x < nc)
        st.H[((size_t)b * (st.m + 1) + threadIdx.x) * st.m + j] += hc[threadIdx.x];
    double acc[MAXCOL];
    acc[0] = 0.0;
    if (on) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double t = w[i];
#pragma unroll
            for (int c = 0; c < MAXCOL; ++c)
                if (c < nc) t -= hc[c] * V[c][i];
            w[i] = t;
            acc[0] += t * t;
        }
    }
    chunk_columns(acc, 1, pout + blockIdx.x);
}

// h_{j+1,j} = ||w|| from the partials and the Givens step of column j: one
// workgroup per reservoir, thread 0 updates the shared state (single writer).
__global__ void __launch_bounds__(RED_THREADS) k_gm_givens(const int *cfirst, int j, int slot, const double *pin,
                                                           GmDev st) {
    __shared__ double tot[MAXCOL];
    const int b = blockIdx.x;
    if (!st.active[b]) {
        if (threadIdx.x == 0) st.flag[slot * st.nb + b] = 0;
        return;
    }
    block_totals(pin, cfirst[b], cfirst[b + 1], 1, tot);
    if (threadIdx.x != 0) return;
    const double hn = sqrt(tot[0]);
    const int m = st.m;
    double *H = st.H + (size_t)b * (m + 1) * m;
    double *cs = st.cs + (size_t)b * m, *sn = st.sn + (size_t)b * m;
    double *g = st.g + (size_t)b * (m + 1);
    // column j and the previous rotations in registers (independent loads)
    double hc[MAXCOL + 1], cc[MAXCOL], ss[MAXCOL];
#pragma unroll
    for (int k = 0; k < MAXCOL; ++k) {
        hc[k] = k <= j ? H[k * m + j] : 0.0;
        cc[k] = k < j ? cs[k] : 1.0;
        ss[k] = k < j ? sn[k] : 0.0;
    }
    hc[MAXCOL] = 0.0;
#pragma unroll
    for (int k = 0; k < MAXCOL - 1; ++k) {
        if (k < j) {
            const double a0 = hc[k], a1 = hc[k + 1];
            hc[k] = cc[k] * a0 + ss[k] * a1;
            hc[k + 1] = -ss[k] * a0 + cc[k] * a1;
        }
    }
    double a0 = 0.0;
#pragma unroll
    for (int k = 0; k < MAXCOL; ++k)
        if (k == j) a0 = hc[k];
    const double den = sqrt(a0 * a0 + hn * hn);
    const double c = den > 0.0 ? a0 / den : 1.0;
    const double sg = den > 0.0 ? hn / den : 0.0;
#pragma unroll
    for (int k = 0; k < MAXCOL; ++k)
        if (k < j) H[k * m + j] = hc[k];
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    cs[j] = c;
    sn[j] = sg;
    const double gj = g[j];
    g[j + 1] = -sg * gj;
    g[j] = c * gj;
    st.its[b] += 1;
    st.kdim[b] = j + 1;
    st.hj[(size_t)b * (m + 1) + m] = hn;   // normalisation of v_{j+1}
    const double res = fabs(g[j + 1]);
    st.res[b] = res;
    int act = 1;
    if (res <= st.tol[b] || hn == 0.0) {
        st.conv[b] = 1;
        act = 0;
    } else if (st.its[b] >= st.maxit || j + 1 == m) {
        act = 0;   // restart (or stop at maxit)
    }
    st.active[b] = act;
    st.flag[slot * st.nb + b] = act;
}

// v_{j+1} = w / h_{j+1,j} for reservoirs still iterating
__global__ void k_gm_next(const Blk *blk, int B, int N, const double *w, double *vn, GmDev st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    if (!st.active[b]) return;
    vn[i] = w[i] / st.hj[(size_t)b * (st.m + 1) + st.m];
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
        invalidate_graphs();
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
    if (!hflag || flag_b < B) {
        if (hflag) HIPC(hipHostFree((void *)hflag));
        int *h = nullptr;
        HIPC(hipHostMalloc((void **)&h, 4 * sizeof(int) * B, hipHostMallocMapped));
        HIPC(hipHostGetDevicePointer((void **)&dflag, h, 0));
        for (int k = 0; k < 4 * B; ++k) h[k] = 0;
        hflag = h;
        flag_b = B;
        if (!ev[0])
            for (auto &e : ev) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    red.ensure(al, sp_, MAXCOL, s);
}

Gmres::~Gmres() {
    invalidate_graphs();
    if (hint) (void)hipHostFree(hint);
    if (hflag) (void)hipHostFree((void *)hflag);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
}

GmDev Gmres::dev(double rtol, double atol, int maxit) {
    GmDev d;
    const int B = nb;
    d.H = H.p; d.cs = cs.p; d.sn = sn.p; d.g = g.p; d.y = y.p; d.hj = hj.p;
    d.tol = scal.p; d.beta = scal.p + B; d.res = scal.p + 2 * B;
    d.active = ints.p; d.conv = ints.p + B; d.kdim = ints.p + 2 * B; d.its = ints.p + 3 * B;
    d.upd = ints.p + 4 * B;
    d.flag = dflag;
    d.nb = nb;
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
    double *P0 = red.part.p, *P1 = red.part.p + (size_t)nch * MAXCOL;
    auto any_flag = [&](int slot) -> bool {
        HIPC(hipEventSynchronize(ev[slot]));
        for (int k = 0; k < nb; ++k)
            if (hflag[slot * nb + k]) return true;
        return false;
    };
    const double *r0 = b;
    if (!x_zero) {
        k_gm_norm_partials<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, b, P0);
        KCHECK();
        k_gm_tol<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, P0, st);
        KCHECK();
        A(x, r.p, b, outer_mask);
        r0 = r.p;
    }
    k_gm_norm_partials<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, r0, P0);
    KCHECK();
    k_gm_begin<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, P0, r0, V[0].p, st, outer_mask,
                                            x_zero ? 1 : 0, 1);
    KCHECK();
    HIPC(hipEventRecord(ev[3], s));
    const double *const *Vp = vptr.p;
    const bool flex = o.flexible;
    // one GMRES iteration j; its activity flags go to `slot`
    auto iteration = [&](int j, int slot) {
        double *zj = flex ? Z[j].p : t.p;
        M(V[j].p, zj, st.active);
        A(zj, w.p, nullptr, st.active);
        {
            ProfScope ps("gmres_orth", s);
            k_gm_dots<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, w.p, Vp, j, P0, st);
            KCHECK();
            k_gm_update_dots<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, w.p, Vp, j, P0, P1, st);
            KCHECK();
            k_gm_update_norm<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, w.p, Vp, j, P1, P0, st);
            KCHECK();
        }
        k_gm_givens<<<S.B, RED_THREADS, 0, s>>>(S.cfirst.p, j, slot, P0, st);
        KCHECK();
        k_gm_next<<<NB, 256, 0, s>>>(S.blk.p, S.B, S.N, w.p, V[j + 1].p, st);
        KCHECK();
    };
    const int kc = (o.graph_chunk > 0 && graphs_ok && s != nullptr) ? std::min(o.graph_chunk, m) : 0;
    if (kc && kc != gchunk) invalidate_graphs();
    gchunk = kc;
    const int nchunk = kc ? (m + kc - 1) / kc : m;
    if (kc && (int)gexec.size() < nchunk) gexec.resize(nchunk, nullptr);
    auto launch_chunk = [&](int c) {
        const int j0 = kc ? c * kc : c, j1 = kc ? std::min(m, j0 + kc) : c + 1;
        if (!kc) {
            iteration(j0, c % 3);
            return;
        }
        if (!gexec[c]) {
            hipGraph_t gr = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
                (void)hipGetLastError();
                graphs_ok = false;   // e.g. the legacy default stream: plain launches from now on
                for (int j = j0; j < j1; ++j) iteration(j, c % 3);
                return;
            }
            try {
                for (int j = j0; j < j1; ++j) iteration(j, c % 3);
            } catch (...) {
                (void)hipStreamEndCapture(s, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                throw;
            }
            HIPC(hipStreamEndCapture(s, &gr));
            HIPC(hipGraphInstantiate(&gexec[c], gr, nullptr, nullptr, 0));
            HIPC(hipGraphDestroy(gr));
        }
        HIPC(hipGraphLaunch(gexec[c], s));
    };
    while (any_flag(3)) {
        for (int c = 0; c < nchunk; ++c) {
            launch_chunk(c);
            HIPC(hipEventRecord(ev[c % 3], s));
            // look-ahead: stop once an earlier chunk left no reservoir active
            const int back = kc ? 1 : 2;
            if (c >= back && !any_flag((c - back) % 3)) break;
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
            launch_axpby(S, 1.0, t.p, 1.0, x, st.upd, s);   // x += M^{-1} V y
        }
        A(x, r.p, b, nullptr);
        r0 = r.p;
        k_gm_norm_partials<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, r0, P0);
        KCHECK();
        k_gm_begin<<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, P0, r0, V[0].p, st, outer_mask, 0, 0);
        KCHECK();
        HIPC(hipEventRecord(ev[3], s));
    }
}

void Gmres::invalidate_graphs() {
    for (auto &g : gexec)
        if (g) (void)hipGraphExecDestroy(g);
    gexec.clear();
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
