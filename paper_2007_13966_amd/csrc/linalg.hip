// Stencil SpMV, per-reservoir reductions and right-preconditioned
// GMRES / FGMRES(m) (Section 3, the Jacobian system; Remark 2 for the flexible
// variant).  Orthogonalisation is classical Gram-Schmidt with one
// reorthogonalisation pass (CGS2), or a single pass for short solves to a
// loose tolerance, FP64.  Every reduction is deterministic: per-chunk
// partial sums, then a fixed-order sum per reservoir by every workgroup of
// the next kernel.
#include <functional>
#include <type_traits>

#include "krylov.h"
#include "reduce.h"

namespace nks {

static inline int nblk(int n, int t) { return (n + t - 1) / t; }

// ---------------------------------------------------------------- spaces
void Space::build(Alloc *al, const std::vector<Blk> &b, hipStream_t s) {
    hblk = b;
    B = (int)b.size();
    N = 0;
    hchunk.clear();
    hcfirst.assign(B + 1, 0);
    htile.clear();
    for (int k = 0; k < B; ++k) {
        hblk[k].off = N;
        const int n = b[k].nx * b[k].ny * b[k].nz;
        // at most MAXCH chunks per block, at least CHUNK cells each
        int nch = std::max(1, std::min(MAXCH, (n + CHUNK - 1) / CHUNK));
        const int cs = (n + nch - 1) / nch;
        hcfirst[k] = (int)hchunk.size();
        for (int c = 0; c < n; c += cs) hchunk.push_back({k, N + c, N + std::min(n, c + cs), 0});
        for (int c = 0; c < n; c += TILE) htile.push_back({k, N + c, N + std::min(n, c + TILE), 0});
        N += n;
    }
    hcfirst[B] = (int)hchunk.size();
    blk.upload(al, hblk, s);
    chunk.upload(al, hchunk, s);
    cfirst.upload(al, hcfirst, s);
    tile.upload(al, htile, s);
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
    int offp[MAXK];   // the offsets, (dx, dy, dz) packed in the low three bytes of an int
};

// Stencil point batch: a 5- or 7-point stencil in one batch of 8, a 21-point
// one in one batch of 24, wider ones in several.
static inline int stencil_batch(int K) { return K <= 8 ? 8 : 24; }

// sum_q coef[q][i] x[i + off_q] over the neighbours of cell i, q in
// increasing order.  Every operator the library builds (Jacobian, Galerkin
// products, transposes) stores an exact zero for a neighbour outside the
// reservoir, so the neighbour index is only clamped into the reservoir's
// cells and the product is 0 x (a finite value), as if the point were
// skipped.  Loads are issued B points at a time; the linear offsets of the
// points are uniform (scalar) and the coefficient rows are addressed from
// scalar bases.
template <int B, bool ABS = false>
__device__ __forceinline__ double stencil_dot(const int *offp, int K, const double *coef, size_t N,
                                              const double *x, int i, const Blk &k) {
    double s = 0.0;
    const int nx = k.nx, nxy = k.nx * k.ny;
    const int lo = k.off, hi = k.off + nxy * k.nz - 1;
    for (int q0 = 0; q0 < K; q0 += B) {
        double cv[B], xv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int q = min(q0 + u, K - 1);
            const int o = offp[q];
            const int dx = (int)(int8_t)(o & 0xff), dy = (int)(int8_t)((o >> 8) & 0xff),
                      dz = (int)(int8_t)((o >> 16) & 0xff);
            const int j = min(max(i + dx + nx * dy + nxy * dz, lo), hi);
            const double c = coef[(size_t)q * N + i];
            xv[u] = ABS ? fabs(x[j]) : x[j];
            cv[u] = q0 + u < K ? (ABS ? fabs(c) : c) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) s += cv[u] * xv[u];
    }
    return s;
}

// a workgroup per tile (a run of at most TILE cells of one reservoir), so the
// reservoir comes with the tile
template <int BS>
__global__ void __launch_bounds__(256) k_spmv(SpmvArgs a, const Chunk *chunks) {
    const Chunk ch = chunks[blockIdx.x];
    if (a.mask && !a.mask[ch.blk]) return;
    const Blk k = a.blk[ch.blk];
    for (int i = ch.start + (int)threadIdx.x; i < ch.end; i += blockDim.x) {
        const double s = stencil_dot<BS>(a.offp, a.K, a.coef, a.N, a.x, i, k);
        a.y[i] = a.b ? a.b[i] - s : s;
    }
}

// y = |A| |x| (the componentwise magnitude of the product), a workgroup
// per tile; a neighbour outside the reservoir adds |0| |x_j|
template <int BS>
__global__ void __launch_bounds__(256) k_spmv_abs(SpmvArgs a, const Chunk *chunks) {
    const Chunk ch = chunks[blockIdx.x];
    const Blk k = a.blk[ch.blk];
    for (int i = ch.start + (int)threadIdx.x; i < ch.end; i += blockDim.x)
        a.y[i] = stencil_dot<BS, true>(a.offp, a.K, a.coef, a.N, a.x, i, k);
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
    if (A.st.K > MAXK) fail(NKS_EINVAL, "stencil of %d points exceeds %d", A.st.K, MAXK);
    for (int q = 0; q < MAXK; ++q) {
        const int qq = std::min(q, A.st.K - 1);
        a.offp[q] = (A.st.off[3 * qq] & 0xff) | ((A.st.off[3 * qq + 1] & 0xff) << 8) |
                    ((A.st.off[3 * qq + 2] & 0xff) << 16);
    }
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
    const dim3 grid((unsigned)A.sp->htile.size());
    if (stencil_batch(a.K) == 8)
        launch_timed("spmv", A.st.K <= 7 ? 0 : 1, k_spmv<8>, grid, dim3(TILE), 0, s, a, A.sp->tile.p);
    else
        launch_timed("spmv", A.st.K <= 7 ? 0 : 1, k_spmv<24>, grid, dim3(TILE), 0, s, a, A.sp->tile.p);
    KCHECK();
}

void launch_spmv_abs(const Op &A, const double *x, double *y, hipStream_t s) {
    SpmvArgs a = spmv_args(A, x, y, nullptr, nullptr);
    const int nt = (int)A.sp->htile.size();
    if (stencil_batch(a.K) == 8) k_spmv_abs<8><<<nt, TILE, 0, s>>>(a, A.sp->tile.p);
    else k_spmv_abs<24><<<nt, TILE, 0, s>>>(a, A.sp->tile.p);
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
// a workgroup per tile (a run of cells of one reservoir)
__global__ void k_axpby(const Chunk *tiles, double a, const double *x, double b, double *y, const int *mask) {
    const Chunk ch = tiles[blockIdx.x];
    const int i = ch.start + (int)threadIdx.x;
    if (i >= ch.end || (mask && !mask[ch.blk])) return;
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

void launch_axpby(const Space &sp, double a, const double *x, double b, double *y, const int *mask,
                  hipStream_t s) {
    k_axpby<<<(int)sp.htile.size(), TILE, 0, s>>>(sp.tile.p, a, x, b, y, mask);
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
// workgroup per chunk writes up to MAXCOL column partials (column sums over
// the workgroup); the next kernel's workgroups each reduce the partials of
// their own reservoir in their prologue, in a fixed order, so every
// workgroup of a reservoir obtains bitwise the same totals, independent of
// the other reservoirs.  The first chunk of each reservoir commits shared
// state.  The workgroup sums live in reduce.h.
// partial dots of x with ncols <= NC vectors ys[c] (or ||x||^2 when
// square).  NC is a compile-time bound: the column reduction's LDS grows
// with it, and a single column needs none of the wide form's
template <int NC>
__global__ void __launch_bounds__(RED_THREADS) k_partials(const Chunk *chunks, const double *x,
                                                          const double *const *ys, int ncols, double *part,
                                                          const int *mask, int square) {
    const Chunk ch = chunks[blockIdx.x];
    const bool on = !mask || mask[ch.blk];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (on) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            const double xi = x[i];
            if (square) {
                acc[0] += xi * xi;
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (c < ncols) acc[c] += xi * ys[c][i];
            }
        }
    }
    chunk_columns<NC>(acc, ncols, part, gridDim.x);
}

// one workgroup per reservoir: out[b*ncols + c]
template <int NC>
__global__ void __launch_bounds__(RED_THREADS) k_totals(const int *cfirst, const double *part, int ncols,
                                                        double *out, int ns) {
    __shared__ double tot[NC];
    const int b = blockIdx.x;
    block_totals<NC>(part, cfirst[b], cfirst[b + 1], ncols, tot, ns);
    if ((int)threadIdx.x < ncols) out[(size_t)b * ncols + threadIdx.x] = tot[threadIdx.x];
}

void launch_block_dots(const Space &sp, Reducer &R, const double *x, const double *const *ys,
                       int ncols, double *out, const int *mask, hipStream_t s) {
    if (ncols > MAXCOL) fail(NKS_EINVAL, "at most %d columns per reduction", MAXCOL);
    if (ncols == 1)
        k_partials<1><<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(sp.chunk.p, x, ys, 1, R.part.p, mask, 0);
    else
        k_partials<MAXCOL><<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(sp.chunk.p, x, ys, ncols, R.part.p, mask, 0);
    KCHECK();
    if (ncols == 1) k_totals<1><<<sp.B, RED_THREADS, 0, s>>>(sp.cfirst.p, R.part.p, 1, out, (int)sp.hchunk.size());
    else k_totals<MAXCOL><<<sp.B, RED_THREADS, 0, s>>>(sp.cfirst.p, R.part.p, ncols, out, (int)sp.hchunk.size());
    KCHECK();
}

void launch_block_norm2(const Space &sp, Reducer &R, const double *x, double *out, const int *mask,
                        hipStream_t s) {
    k_partials<1><<<(int)sp.hchunk.size(), RED_THREADS, 0, s>>>(sp.chunk.p, x, nullptr, 1, R.part.p, mask, 1);
    KCHECK();
    k_totals<1><<<sp.B, RED_THREADS, 0, s>>>(sp.cfirst.p, R.part.p, 1, out, (int)sp.hchunk.size());
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
    block_totals<1>(part, q0, cfirst[b + 1], 1, tot, gridDim.x);
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
        st.flag[st.m * st.nb + b] = act ? 1 : (conv ? 2 : 0);
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_gm_norm_partials(const Chunk *chunks, const double *r,
                                                                  double *part) {
    const Chunk ch = chunks[blockIdx.x];
    double acc[MAXCOL];
    acc[0] = 0.0;
    for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) acc[0] += r[i] * r[i];
    chunk_columns<1>(acc, 1, part, gridDim.x);
}

// tol from ||b|| (x0 != 0), lead chunk of each reservoir
__global__ void __launch_bounds__(RED_THREADS) k_gm_tol(const Chunk *chunks, const int *cfirst, const double *part,
                                                        GmDev st) {
    __shared__ double tot[MAXCOL];
    const Chunk ch = chunks[blockIdx.x];
    const int q0 = cfirst[ch.blk];
    if ((int)blockIdx.x != q0) return;
    block_totals<1>(part, q0, cfirst[ch.blk + 1], 1, tot, gridDim.x);
    if (threadIdx.x == 0) st.tol[ch.blk] = fmax(st.rtol * sqrt(tot[0]), st.atol);
}


// One Arnoldi step j of classical Gram-Schmidt with one reorthogonalisation
// (CGS2) takes three kernels after the preconditioner:
//   spmv_dots    w = A z_j and the pass-1 partials V[0..j]^T w
//                (or gm_dots when A is not a stencil operator);
//   update_dots  h1 = pass-1 totals (the lead chunk stores H[:, j] = h1),
//                w -= V h1, pass-2 partials V^T w and w.w;
//   finish       h2 = pass-2 totals, h_{j+1,j} = sqrt(w.w - h2.h2) (w is
//                already orthogonal to V to working precision, so h2 is a
//                rounding-size correction and the subtraction loses nothing),
//                v_{j+1} = (w - V h2) / h_{j+1,j}; the lead chunk adds h2 to
//                H[:, j] and applies the Givens rotations.
// The single-pass form (classical Gram-Schmidt without reorthogonalisation,
// for short solves to a loose tolerance) takes two: spmv_dots also sums w.w,
// and finish takes h = pass-1 totals and h_{j+1,j} = sqrt(w.w - h.h).
// Activity flags are double-buffered: iteration j reads act_j and only the
// lead chunk of a reservoir writes act_{j+1}, so no workgroup reads a flag
// that another rewrites in the same kernel.

// pass-1 partials of w = A z with V[0..j] (stencil operator, chunk grid);
// ww: w.w in column j+1 as well
template <int NC, int BS>
__global__ void __launch_bounds__(RED_THREADS) k_gm_spmv_dots(const Chunk *chunks, SpmvArgs a, const double *V, long ld, int j,
                                                              double *part, const int *act, int ww) {
    const Chunk ch = chunks[blockIdx.x];
    // an inactive reservoir's partials are never read
    if (!act[ch.blk]) return;
    const int nc = j + 1;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    {
        const Blk k = a.blk[ch.blk];
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double vv[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) vv[c] = V[(size_t)c * ld + i];
            const double wi = stencil_dot<BS>(a.offp, a.K, a.coef, a.N, a.x, i, k);
            a.y[i] = wi;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) acc[c] += wi * vv[c];
#pragma unroll
            for (int c = 1; c < NC; ++c)
                if (c == nc && ww) acc[c] += wi * wi;
        }
    }
    chunk_columns<NC>(acc, nc + (ww ? 1 : 0), part, gridDim.x);
}

// pass-1 partials V[0..j]^T w (w from a generic operator); ww: w.w in
// column j+1 as well
template <int NC>
__global__ void __launch_bounds__(RED_THREADS) k_gm_dots(const Chunk *chunks, const double *w, const double *V, long ld, int j,
                                                         double *part, const int *act, int ww) {
    const Chunk ch = chunks[blockIdx.x];
    if (!act[ch.blk]) return;   // an inactive reservoir's partials are never read
    const int nc = j + 1;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double vv[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) vv[c] = V[(size_t)c * ld + i];
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) acc[c] += wi * vv[c];
#pragma unroll
            for (int c = 1; c < NC; ++c)
                if (c == nc && ww) acc[c] += wi * wi;
        }
    }
    chunk_columns<NC>(acc, nc + (ww ? 1 : 0), part, gridDim.x);
}

// h1 = pass-1 totals (lead chunk stores H[:, j]); w -= V h1; pass-2 partials
// V^T w in columns 0..j and w.w in column j+1
template <int NC>
__global__ void __launch_bounds__(RED_THREADS) k_gm_update_dots(const Chunk *chunks, const int *cfirst, double *w,
                                                                const double *V, long ld, int j, const double *pin, double *pout,
                                                                GmDev st, const int *act) {
    __shared__ double hc[NC];
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk, nc = j + 1;
    const bool on = act[b];
    if (!on) return;   // an inactive reservoir's partials are never read
    block_totals<NC>(pin, cfirst[b], cfirst[b + 1], nc, hc, gridDim.x);
    if ((int)blockIdx.x == cfirst[b] && (int)threadIdx.x < nc)
        st.H[((size_t)b * (st.m + 1) + threadIdx.x) * st.m + j] = hc[threadIdx.x];
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    if (on) {
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double vv[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) vv[c] = V[(size_t)c * ld + i];
            double t = w[i];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) t -= hc[c] * vv[c];
            w[i] = t;
#pragma unroll
            for (int c = 0; c < NC - 1; ++c)
                if (c < nc) acc[c] += t * vv[c];
#pragma unroll
            for (int c = 1; c < NC; ++c)
                if (c == nc) acc[c] += t * t;
        }
    }
    chunk_columns<NC>(acc, nc + 1, pout, gridDim.x);
}

// h2 and w.w from the pass-2 partials; v_{j+1} = (w - V h2) / h_{j+1,j};
// the lead chunk of each reservoir updates H, the rotations and the
// residual estimate, and decides act_{j+1} and the host flag (single writer).
template <int NC>
__global__ void __launch_bounds__(RED_THREADS) k_gm_finish(const Chunk *chunks, const int *cfirst, const double *w,
                                                           const double *V, long ld, int j, const double *pin, double *vn, GmDev st,
                                                           const int *act, int *act_next, int slot, int single) {
    __shared__ double hc[NC];
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk, nc = j + 1;
    const bool on = act[b];
    const bool lead = (int)blockIdx.x == cfirst[b];
    if (!on) {
        if (lead && threadIdx.x == 0) {
            act_next[b] = 0;
            st.flag[slot * st.nb + b] = st.conv[b] ? 2 : 0;
        }
        return;
    }
    // the lead chunk stages H[:, j] (h1), the previous rotations and g[j]
    // in LDS, one value per thread, while the partial totals load
    __shared__ double gv[3 * NC + 1];
    const int m = st.m;
    double *H = st.H + (size_t)b * (m + 1) * m;
    double *cs = st.cs + (size_t)b * m, *sn = st.sn + (size_t)b * m;
    double *g = st.g + (size_t)b * (m + 1);
    if (lead) {
        const int t = threadIdx.x, jm = max(j - 1, 0);
        if (t < NC) {
            // single pass: column j holds nothing yet (h comes from pin)
            gv[t] = single ? 0.0 : H[(size_t)min(t, j) * m + j];
            gv[NC + t] = cs[min(t, jm)];
            gv[2 * NC + t] = sn[min(t, jm)];
        } else if (t == NC) {
            gv[3 * NC] = g[j];
        }
    }
    // the lead thread's scalars, loaded ahead of the reduction
    int its0 = 0;
    double tol0 = 0.0;
    if (lead && threadIdx.x == 0) {
        its0 = st.its[b];
        tol0 = st.tol[b];
    }
    block_totals<NC>(pin, cfirst[b], cfirst[b + 1], nc + 1, hc, gridDim.x);
    double h2sq = 0.0;
    for (int c = 0; c < nc; ++c) h2sq += hc[c] * hc[c];
    const double hn = sqrt(fmax(hc[nc] - h2sq, 0.0));
    // the lead chunk's first thread applies the rotations before its share
    // of the vector work (the Givens step needs only the totals)
    if (lead && threadIdx.x == 0) {
        // column j (h1 + h2) down the previous rotations, one pair of
        // entries at a time (entry k + 1 is still unrotated when rotation k
        // reaches it), straight from LDS: no register copy of the column
        double a0 = gv[0] + hc[0];
        for (int k = 0; k < j; ++k) {
            const double a1 = gv[k + 1] + hc[k + 1];
            const double ck = gv[NC + k], sk = gv[2 * NC + k];
            H[(size_t)k * m + j] = ck * a0 + sk * a1;
            a0 = -sk * a0 + ck * a1;
        }
        const double gj = gv[3 * NC];
        const double den = sqrt(a0 * a0 + hn * hn);
        const double c = den > 0.0 ? a0 / den : 1.0;
        const double sg = den > 0.0 ? hn / den : 0.0;
        H[(size_t)j * m + j] = den;
        H[(size_t)(j + 1) * m + j] = 0.0;
        cs[j] = c;
        sn[j] = sg;
        g[j + 1] = -sg * gj;
        g[j] = c * gj;
        // an active reservoir has not converged before this iteration
        const int its1 = its0 + 1;
        st.its[b] = its1;
        st.kdim[b] = j + 1;
        const double res = fabs(sg * gj);
        st.res[b] = res;
        int nxt = 1, conv = 0;
        if (res <= tol0 || hn == 0.0) {
            conv = 1;
            st.conv[b] = 1;
            nxt = 0;
        } else if (its1 >= st.maxit || j + 1 == m) {
            nxt = 0;   // restart (or stop at maxit)
        }
        act_next[b] = nxt;
        st.flag[slot * st.nb + b] = nxt ? 1 : (conv ? 2 : 0);
    }
    if (hn > 0.0) {
        const double inv = 1.0 / hn;
        for (int i = ch.start + threadIdx.x; i < ch.end; i += blockDim.x) {
            double vv[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) vv[c] = V[(size_t)c * ld + i];
            double t = w[i];
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c < nc) t -= hc[c] * vv[c];
            vn[i] = t * inv;
        }
    }
}

// Calls f with the smallest compiled column bound (4, 8, 16, MAXCOL) that
// holds `cols` columns: the Arnoldi kernels' register arrays and reductions
// scale with the bound, not with MAXCOL.
template <typename F>
static void with_columns(int cols, F &&f) {
    if (cols <= 4) f(std::integral_constant<int, 4>{});
    else if (cols <= 8) f(std::integral_constant<int, 8>{});
    else if (cols <= 16) f(std::integral_constant<int, 16>{});
    else if (cols <= MAXCOL) f(std::integral_constant<int, MAXCOL>{});
    else fail(NKS_EINVAL, "%d Krylov columns exceed %d", cols, MAXCOL);
}

// back substitution H y = g over the kdim leading columns of each block
// Back substitution R y = g of the rotated Hessenberg matrix, one wavefront
// per reservoir, by columns: lane i holds g_i and column entries H[i][c];
// once y_c is known (lane c), every row above subtracts H[i][c] y_c.
__global__ void __launch_bounds__(64) k_gm_solve_y(int B, GmDev st) {
    constexpr int MR = MAXCOL - 2;   // largest restart
    const int b = blockIdx.x, i = threadIdx.x;
    if (b >= B) return;
    const int m = st.m, k = st.kdim[b];
    const double *H = st.H + (size_t)b * (m + 1) * m;
    double gi = i < k ? st.g[(size_t)b * (m + 1) + i] : 0.0;
    double hr[MR];
#pragma unroll
    for (int c = 0; c < MR; ++c) hr[c] = (i <= c && c < k) ? H[(size_t)i * m + c] : 0.0;
    double yi = 0.0;
#pragma unroll
    for (int c = MR - 1; c >= 0; --c) {
        if (c < k) {
            const double yc = __shfl(gi, c) / __shfl(hr[c], c);
            if (i < c) gi -= hr[c] * yc;
            if (i == c) yi = yc;
        }
    }
    if (i < k) st.y[(size_t)b * m + i] = yi;
    if (i == 0) st.upd[b] = k > 0;
}

// x += sum_{c < kdim} y[c] Zc   (or u = sum y[c] Vc when accumulate == 0),
// a workgroup per tile
__global__ void k_gm_combine(const Chunk *chunks, const double *const *Z, double *x, GmDev st, int accumulate) {
    const Chunk ch = chunks[blockIdx.x];
    const int b = ch.blk;
    const int k = st.kdim[b];
    if (k == 0) return;
    const double *y = st.y + (size_t)b * st.m;
    for (int i = ch.start + (int)threadIdx.x; i < ch.end; i += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += y[c] * Z[c][i];
        x[i] = accumulate ? x[i] + s : s;
    }
}

// ---------------------------------------------------------------- host driver
void Gmres::ensure(Alloc *al_, const Space &sp_, int m_, bool flexible, hipStream_t s) {
    if (m_ < 1 || m_ + 2 > MAXCOL) fail(NKS_EINVAL, "restart %d outside [1, %d]", m_, MAXCOL - 2);
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
        // one allocation for the basis: column k at Vall + k * ld, ld a
        // multiple of 64 doubles, so kernels address it from one pointer
        ld = ((long)N + 63) / 64 * 64;
        Vall.alloc(al, (size_t)(m + 1) * ld);
        V.resize(m + 1);
        for (int k = 0; k <= m; ++k) V[k].p = Vall.p + (size_t)k * ld;
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
        ints.alloc(al, (size_t)B * 6);
        std::vector<const double *> hv(m + 1), hz(std::max(m, 1));
        for (int k = 0; k <= m; ++k) hv[k] = V[k].p;
        for (int k = 0; k < (int)Z.size(); ++k) hz[k] = Z[k].p;
        if (Z.empty()) hz.assign(1, nullptr);
        vptr.upload(al, hv, s);
        zptr.upload(al, hz, s);
        if (hint) HIPC(hipHostFree(hint));
        // pinned staging for stats(): the 6*B ints, then the 3*B doubles
        HIPC(hipHostMalloc((void **)&hint, sizeof(int) * 6 * B + sizeof(double) * 3 * B + 64));
    }
    if (!hflag || flag_b < B || flag_m < m) {
        // one slot of B flags per iteration of a cycle, and slot m for its start
        if (hflag) HIPC(hipHostFree((void *)hflag));
        int *h = nullptr;
        HIPC(hipHostMalloc((void **)&h, (size_t)(m + 1) * sizeof(int) * B, hipHostMallocMapped));
        HIPC(hipHostGetDevicePointer((void **)&dflag, h, 0));
        for (int k = 0; k < (m + 1) * B; ++k) h[k] = 0;
        hflag = h;
        flag_b = B;
        flag_m = m;
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
    d.active2 = ints.p + 5 * B;
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
    count_host_wait();
    for (int b = 0; b < nb; ++b) if (hint[b]) return true;
    return false;
}

void Gmres::solve(const MatVec &A, const Precond &M, const double *b, double *x, bool x_zero,
                  const GmOpts &o, const int *outer_mask, hipStream_t s, const Op *Aop) {
    const Space &S = *sp;
    const int nch = (int)S.hchunk.size();
    GmDev st = dev(o.rtol, o.atol, o.maxit);
    double *P0 = red.part.p, *P1 = red.part.p + (size_t)nch * MAXCOL;
    // host flags per reservoir and iteration slot: 1 iterating, 2 converged,
    // 0 stopped for a restart (or at maxit); slot m: the start of a cycle
    auto any_flag = [&](int slot) -> bool {
        for (int k = 0; k < nb; ++k)
            if (hflag[slot * nb + k] == 1) return true;
        return false;
    };
    auto all_converged = [&](int slot) -> bool {
        for (int k = 0; k < nb; ++k)
            if (hflag[slot * nb + k] != 2) return false;
        return true;
    };
    auto wait = [&](hipEvent_t e) {
        HIPC(hipEventSynchronize(e));
        count_host_wait();
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
    const double *vb = V[0].p;   // the basis: m + 1 columns of stride ld
    const bool flex = o.flexible;
    // one GMRES iteration j; its activity flags go to slot j
    auto iteration = [&](int j) {
        double *zj = flex ? Z[j].p : t.p;
        const int *act = (j & 1) ? st.active2 : st.active;
        int *act_next = (j & 1) ? st.active : st.active2;
        M(V[j].p, zj, act);
        ProfScope ps("gmres_arnoldi", s);
        // pass 2 carries j + 2 columns (V[0..j]^T w and w.w)
        with_columns(j + 2, [&](auto bound) {
            constexpr int NC = decltype(bound)::value;
            const int one = o.single_pass ? 1 : 0;
            if (Aop) {
                SpmvArgs sa = spmv_args(*Aop, zj, w.p, nullptr, nullptr);
                if (stencil_batch(sa.K) == 8)
                    k_gm_spmv_dots<NC, 8><<<nch, RED_THREADS, 0, s>>>(S.chunk.p, sa, vb, ld, j, P0, act, one);
                else
                    k_gm_spmv_dots<NC, 24><<<nch, RED_THREADS, 0, s>>>(S.chunk.p, sa, vb, ld, j, P0, act, one);
                KCHECK();
            } else {
                A(zj, w.p, nullptr, act);
                k_gm_dots<NC><<<nch, RED_THREADS, 0, s>>>(S.chunk.p, w.p, vb, ld, j, P0, act, one);
                KCHECK();
            }
            if (!one) {
                k_gm_update_dots<NC><<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, w.p, vb, ld, j, P0, P1, st,
                                                                 act);
                KCHECK();
            }
            k_gm_finish<NC><<<nch, RED_THREADS, 0, s>>>(S.chunk.p, S.cfirst.p, w.p, vb, ld, j, one ? P0 : P1,
                                                        V[j + 1].p, st, act, act_next, j, one);
            KCHECK();
        });
    };
    const int kc = (o.graph_chunk > 0 && graphs_ok && s != nullptr && !prof_direct()) ? std::min(o.graph_chunk, m) : 0;
    const std::tuple<int, int, int, const void *> key{o.maxit, o.single_pass ? 1 : 0, flex ? 1 : 0, Aop};
    if ((kc && kc != gchunk) || key != gkey) invalidate_graphs();
    gchunk = kc;
    gkey = key;
    // Chunks of iterations [j0, j1): a lead chunk of 2 kc, then chunks of kc,
    // each captured once and replayed (a graph launch costs a boundary of a
    // few microseconds; iterations queued past convergence run as no-ops).
    // Without graphs every chunk is one iteration.
    const int lead = kc ? std::min(m, 2 * kc) : 1, tail = kc ? kc : 1;
    auto chunk_begin = [&](int c) { return c == 0 ? 0 : std::min(m, lead + (c - 1) * tail); };
    const int nchunk = 1 + (m - lead + tail - 1) / tail;
    auto launch_chunk = [&](int c) {
        const int j0 = chunk_begin(c), j1 = chunk_begin(c + 1);
        if (!kc) {
            iteration(j0);
            return;
        }
        hipGraphExec_t &ge = gexec[{j0, j1}];
        if (!ge) {
            hipGraph_t gr = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
                (void)hipGetLastError();
                graphs_ok = false;   // e.g. the legacy default stream: plain launches from now on
                gexec.erase({j0, j1});
                for (int j = j0; j < j1; ++j) iteration(j);
                return;
            }
            try {
                for (int j = j0; j < j1; ++j) iteration(j);
            } catch (...) {
                (void)hipStreamEndCapture(s, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                gexec.erase({j0, j1});
                throw;
            }
            HIPC(hipStreamEndCapture(s, &gr));
            HIPC(hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0));
            HIPC(hipGraphDestroy(gr));
        }
        HIPC(hipGraphLaunch(ge, s));
    };
    for (;;) {
        // The first chunk of a cycle is queued before the cycle's start flag
        // is read (a cycle with nothing to do runs it as no-ops), and each
        // later chunk before the flags of the one ahead of it are read (with
        // graphs one chunk ahead, each graph launch costing a boundary; two
        // without).  The cycle ends when a finished chunk leaves no reservoir
        // iterating; when all of them converged, the solve ends without
        // recomputing the residual.
        bool finished = false;
        for (int c = 0; c < nchunk; ++c) {
            launch_chunk(c);
            HIPC(hipEventRecord(ev[c % 3], s));
            if (c == 0) {
                wait(ev[3]);
                if (!any_flag(m)) {
                    finished = true;
                    break;
                }
            }
            const int back = kc ? 1 : 2;
            if (c >= back) {
                const int cb = c - back, last = chunk_begin(cb + 1) - 1;
                wait(ev[cb % 3]);
                if (!any_flag(last)) {
                    finished = all_converged(last);
                    break;
                }
            }
        }
        k_gm_solve_y<<<S.B, 64, 0, s>>>(S.B, st);
        KCHECK();
        if (flex) {
            k_gm_combine<<<(int)S.htile.size(), TILE, 0, s>>>(S.tile.p, zptr.p, x, st, 1);
            KCHECK();
        } else {
            k_gm_combine<<<(int)S.htile.size(), TILE, 0, s>>>(S.tile.p, Vp, w.p, st, 0);
            KCHECK();
            M(w.p, t.p, st.upd);
            launch_axpby(S, 1.0, t.p, 1.0, x, st.upd, s);   // x += M^{-1} V y
        }
        if (finished) break;
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
        if (g.second) (void)hipGraphExecDestroy(g.second);
    gexec.clear();
}

void Gmres::stats(std::vector<int> &its, std::vector<double> &res, std::vector<int> &conv,
                  hipStream_t s) {
    const int B = nb;
    // through pinned memory: a pageable destination costs a host round trip per copy
    int *hi = hint;
    double *hd = reinterpret_cast<double *>(
        reinterpret_cast<char *>(hint) + ((sizeof(int) * 6 * B + 63) / 64) * 64);
    HIPC(hipMemcpyAsync(hi, ints.p, sizeof(int) * 5 * B, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(hd, scal.p, sizeof(double) * 3 * B, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    count_host_wait();
    its.assign(hi + 3 * B, hi + 4 * B);
    conv.assign(hi + B, hi + 2 * B);
    res.assign(hd + 2 * B, hd + 3 * B);
}

}  // namespace nks
