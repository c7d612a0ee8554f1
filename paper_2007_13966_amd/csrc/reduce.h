// Workgroup reductions of the Krylov kernels: DPP lane-group sums, column
// sums over a workgroup, and the totals of per-chunk partial sums (two-stage,
// fence-free reductions: the partials of one kernel are summed by every
// workgroup of the next).
#pragma once

#include "nks_internal.h"

namespace nks {

constexpr int MAXCOL = 32;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Row sums (16 lanes) by DPP moves: pair swap, quad swap, half-row mirror,
// row mirror.  Every lane of a row ends with the same value, bitwise: each
// step adds the same two operands in either order.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    // every lane has a source for these controls, so no old value is needed
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return v;
}

// Sums over TP consecutive lanes (TP = 8, 16, 32, 64): DPP quad swaps and
// row mirrors inside a row of 16 lanes, then lane shuffles across rows and
// across the two halves of the wavefront.  Each step adds two operands that
// the partner lane adds in the other order, so every lane of a group ends
// with the same value, bitwise.
template <int TP>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(TP == 8 || TP == 16 || TP == 32 || TP == 64, "lane group of 8, 16, 32 or 64");
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    if constexpr (TP >= 16) v += dpp_mov<0x140>(v);
    if constexpr (TP >= 32) v += __shfl_xor(v, 16, 64);
    if constexpr (TP >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

// Sums over the workgroup (RED_THREADS threads) of v[c], c < NC; thread
// (c, s) with s == 0 passes column c < nc to dst(c, total).
// NC <= 2: row sums by DPP, the 16 row sums (4 waves x 4 rows) through LDS,
// added in row order.  NC >= 4: the values go through LDS column-major, TP =
// RED_THREADS / NC consecutive threads add one column's entries in a fixed
// order and finish with a lane-group sum, so the work per thread grows with
// NC, not with NC times the reduction depth.
template <int NC, typename Store>
__device__ __forceinline__ void workgroup_columns(const double (&v)[NC], int nc, Store dst) {
    if constexpr (NC <= 2) {
        __shared__ double sh[16][NC];
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        double r[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) r[c] = row_sum(v[c]);
        if ((lane & 15) == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) sh[w * 4 + (lane >> 4)][c] = r[c];
        }
        __syncthreads();
        if ((int)threadIdx.x < nc) {
            double t = 0.0;
            const int nr = (blockDim.x >> 6) * 4;
            for (int k = 0; k < nr; ++k) t += sh[k][threadIdx.x];
            dst(threadIdx.x, t);
        }
    } else {
        constexpr int TP = RED_THREADS / NC;
        constexpr int LD = RED_THREADS + 2;   // column stride, off the LDS bank period
        __shared__ double sh[NC * LD];
        const int t = threadIdx.x;
#pragma unroll
        for (int c = 0; c < NC; ++c) sh[c * LD + t] = v[c];
        __syncthreads();
        const int c = t / TP, q = t - c * TP;
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k) a += sh[c * LD + q + TP * k];
        a = group_sum<TP>(a);
        if (q == 0 && c < nc) dst(c, a);
    }
}

// column sums of this workgroup's registers into part[c * ns + blockIdx.x]
// (column-major over the ns chunks, so the totals read coalesced)
template <int NC, int M>
__device__ __forceinline__ void chunk_columns(const double (&acc)[M], int nc, double *part, int ns) {
    static_assert(NC <= M, "column bound exceeds the register array");
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = acc[c];
    workgroup_columns<NC>(v, nc, [&](int c, double t) { part[(size_t)c * ns + blockIdx.x] = t; });
}

// totals of the nc partial columns of reservoir b (chunks [q0, q1), at most
// RED_THREADS chunks, column stride ns) into out[0..NC) in LDS (zero past
// nc), visible to the whole workgroup.  Branch-free: every load has a valid
// address (clamped column and chunk) and out-of-range values are zeroed.
// NC >= 4: TP = RED_THREADS / NC consecutive threads share a column, each
// adding every TP-th chunk, then a lane-group sum.
template <int NC>
__device__ __forceinline__ void block_totals(const double *part, int q0, int q1, int nc, double *out, int ns) {
    static_assert(MAXCH <= RED_THREADS, "one reduction thread per chunk");
    if constexpr (NC <= 2) {
        const int q = q0 + (int)threadIdx.x;
        const bool qin = q < q1;
        const int qq = qin ? q : q0;
        double v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double x = part[(size_t)min(c, max(nc - 1, 0)) * ns + qq];
            v[c] = (c < nc && qin) ? x : 0.0;
        }
        workgroup_columns<NC>(v, nc, [&](int c, double t) { out[c] = t; });
        if ((int)threadIdx.x >= nc && (int)threadIdx.x < NC) out[threadIdx.x] = 0.0;
    } else {
        constexpr int TP = RED_THREADS / NC;
        const int c = (int)threadIdx.x / TP, s = (int)threadIdx.x - c * TP;
        const double *col = part + (size_t)min(c, max(nc - 1, 0)) * ns;
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int q = q0 + s + TP * k;
            const double x = col[min(q, q1 - 1)];
            a += q < q1 ? x : 0.0;
        }
        a = group_sum<TP>(a);
        if (s == 0) out[c] = c < nc ? a : 0.0;
    }
    __syncthreads();
}

}  // namespace nks
