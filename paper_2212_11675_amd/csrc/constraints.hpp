// Constraint equations (Section 3: extra equations that make the solution unique; the
// "constraints computation" region that ends Algorithms 1 and 2): n_con sparse rows C given
// by the caller in compressed row form, appended below the observation rows, so that the
// products and solves act on the stacked [A; C].  Row-space vectors then carry the n_con
// constraint entries after the n_rows observation entries.
//
// aprod 1 part (y_c (op)= C x): the entries are split into one contiguous range per block;
// rows are contiguous in entry order, so a block's range spans few rows of a long constraint
// row, or many short rows.  Each thread sums its strided share of the range per row and adds
// the sum into an LDS slot (rows within kConSlots of the block's first row) or, past those,
// straight into the global accumulator; the block then adds its slots to the accumulator
// (one atomic per row it touched).  A one-block finishing kernel applies the operation.
//
// aprod 2 part (x += C^T y_c): over a library-owned copy grouped by column (one group per
// distinct column), one thread per column sums its entries and adds them with a plain
// read-modify-write (each column belongs to exactly one thread); it runs after the other
// aprod 2 kernels, in stream order.
#pragma once

#include "kernels.hpp"

namespace gsr {

constexpr int kConSlots = 64;   // LDS row slots per block of k_con_dot
constexpr int kConBlock = 256;

// acc[row(e)] += val[e] * x[col[e]] over all entries (acc zero before; the finishing kernel
// clears it again).  check_stop: skip once the LSQR stop flag is set; gate: skip when set.
static __global__ __launch_bounds__(kConBlock) void k_con_dot(
    int64_t nnz, int64_t per_block, const int32_t* __restrict__ crow,
    const int64_t* __restrict__ ccol, const double* __restrict__ cval,
    const double* __restrict__ x, double* __restrict__ acc, const LsqrState* __restrict__ st,
    int check_stop, const int32_t* __restrict__ gate) {
    __shared__ double slot[kConSlots];
    if (check_stop && st->stop) return;
    if (gate && *gate) return;
    const int64_t e0 = (int64_t)blockIdx.x * per_block;
    const int64_t e1 = min(nnz, e0 + per_block);
    if (e0 >= e1) return;
    for (int k = threadIdx.x; k < kConSlots; k += blockDim.x) slot[k] = 0.0;
    __syncthreads();
    const int32_t r0 = crow[e0];
    int32_t cur = -1;
    double sum = 0.0;
    auto flush = [&]() {
        if (cur < 0) return;
        if (cur - r0 < kConSlots)
            atomicAdd(slot + (cur - r0), sum);
        else
            atomic_add_f64(acc + cur, sum);
    };
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const int32_t r = crow[e];
        if (r != cur) {
            flush();
            cur = r;
            sum = 0.0;
        }
        sum = fma(cval[e], x[ccol[e]], sum);
    }
    flush();
    __syncthreads();
    const int32_t r_last = crow[e1 - 1];
    for (int k = threadIdx.x; k < kConSlots && r0 + k <= r_last; k += blockDim.x)
        if (slot[k] != 0.0) atomic_add_f64(acc + r0 + k, slot[k]);
}

// What the finishing kernel does with d = (C x)[k]:
//   CON_ADD   : y_c[k] += d
//   CON_RESID : y_c[k] = b_c[k] - d
//   CON_LSQR  : y_c[k] = xs d - ys y_c[k], (xs, ys) = (sv, alpha su) for the forward operator
//               A D or (su, beta sv) for the transposed one (TRANS); partial sum of y_c^2
//               into part[0].  PENDING (transposed operator, row-space iterate): first the
//               pending update z_c += f1 w_c; w_c = sv y_c - f2 w_c with the old y_c, and the
//               partial sums of z^2, z w, w^2 into part[stride], part[2 stride], part[3 stride].
enum { CON_ADD = 0, CON_RESID = 1, CON_LSQR = 2 };

template <int MODE, bool TRANS = false, bool PENDING = false>
static __global__ __launch_bounds__(kConBlock) void k_con_fin(
    int64_t n_con, double* __restrict__ acc, double* __restrict__ yc,
    const double* __restrict__ bc, const LsqrState* __restrict__ st, double* __restrict__ part,
    int stride, double* __restrict__ wc, double* __restrict__ zc,
    const int32_t* __restrict__ gate) {
    __shared__ double sh[kConBlock / kWave];
    if (MODE == CON_LSQR && st->stop) return;
    if (gate && *gate) return;
    double xs = 1.0, ys = 0.0;
    if (MODE == CON_LSQR) {
        xs = TRANS ? st->su : st->sv;
        ys = TRANS ? st->beta * st->sv : st->alpha * st->su;
    }
    const bool pending = PENDING && st->pending;
    const double f1 = st ? st->f1 : 0.0, f2 = st ? st->f2 : 0.0, svo = st ? st->sv : 0.0;
    double ysq = 0.0, zsq = 0.0, zw = 0.0, wsq = 0.0;
    for (int64_t k = threadIdx.x; k < n_con; k += blockDim.x) {
        const double d = acc[k];
        acc[k] = 0.0;
        if (MODE == CON_ADD) {
            yc[k] += d;
        } else if (MODE == CON_RESID) {
            yc[k] = bc[k] - d;
        } else {
            const double yo = yc[k];
            if (PENDING && pending) {
                const double wo = wc[k];
                const double zn = fma(f1, wo, zc[k]);
                const double wn = svo * yo - f2 * wo;
                zc[k] = zn;
                wc[k] = wn;
                zsq = fma(zn, zn, zsq);
                zw = fma(zn, wn, zw);
                wsq = fma(wn, wn, wsq);
            }
            const double yn = (ys != 0.0) ? xs * d - ys * yo : xs * d;
            yc[k] = yn;
            ysq = fma(yn, yn, ysq);
        }
    }
    if (MODE != CON_LSQR) return;
    double t = block_sum<kConBlock>(ysq, sh);
    if (threadIdx.x == 0) part[0] = t;
    if (PENDING) {
        t = block_sum<kConBlock>(zsq, sh);
        if (threadIdx.x == 0) part[stride] = t;
        t = block_sum<kConBlock>(zw, sh);
        if (threadIdx.x == 0) part[2 * stride] = t;
        t = block_sum<kConBlock>(wsq, sh);
        if (threadIdx.x == 0) part[3 * stride] = t;
    }
}

// x[col_j] += sum over the entries of column j of val * y_c[row]  (SQ: val^2, the column
// norms).  One thread per distinct column of C.
template <bool SQ>
static __global__ __launch_bounds__(kConBlock) void k_con_a2(
    int64_t ncols, const int64_t* __restrict__ ucol, const int64_t* __restrict__ uptr,
    const int32_t* __restrict__ urow, const double* __restrict__ uval,
    const double* __restrict__ yc, double* __restrict__ x, const LsqrState* __restrict__ st,
    int check_stop) {
    if (check_stop && st->stop) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ncols; j += stride) {
        double sum = 0.0;
        for (int64_t e = uptr[j]; e < uptr[j + 1]; ++e) {
            const double v = uval[e];
            sum = SQ ? fma(v, v, sum) : fma(v, yc[urow[e]], sum);
        }
        x[ucol[j]] += sum;
    }
}

// Setup of the constraint rows: the row of every entry (binary search in ptr), the
// sequence 0..nnz-1, and checks (bit 0 column out of range).
static __global__ void k_con_rows(int64_t n_con, int64_t nnz, int64_t n_cols,
                                  const int64_t* __restrict__ ptr, const int64_t* __restrict__ col,
                                  int32_t* __restrict__ crow, int32_t* __restrict__ seq,
                                  int* __restrict__ flags) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        int64_t lo = 0, hi = n_con - 1;  // last row k with ptr[k] <= e
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (ptr[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        crow[e] = (int32_t)lo;
        seq[e] = (int32_t)e;
        const int64_t c = col[e];
        if (c < 0 || c >= n_cols) bad |= 1;
    }
    if (bad) atomicOr(flags, bad);
}

// bit 0 of flags: ptr[k+1] < ptr[k] for some k
static __global__ void k_con_check_ptr(int64_t n_con, const int64_t* __restrict__ ptr,
                                       int* __restrict__ flags) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_con; k += stride)
        if (ptr[k + 1] < ptr[k]) bad = 1;
    if (bad) atomicOr(flags, bad);
}

static __global__ void k_fill_i32(int32_t* __restrict__ v, int64_t n, int32_t val) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) v[j] = val;
}

static __global__ void k_widen_i32(int64_t n, const int32_t* __restrict__ src,
                                   int64_t* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        dst[j] = src[j];
}

// The column-grouped copy: entry k of the copy is entry perm[k] of the caller's rows.
static __global__ void k_con_gather(int64_t nnz, const int32_t* __restrict__ perm,
                                    const int32_t* __restrict__ crow,
                                    const double* __restrict__ val, int32_t* __restrict__ urow,
                                    double* __restrict__ uval) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
        const int32_t e = perm[k];
        urow[k] = crow[e];
        uval[k] = val[e];
    }
}

}  // namespace gsr
