// The two products of the hot path (Section 3, Algorithms 1 and 2), written for gfx950.
//
// Lane layout ("quad"): four lanes per row, sixteen rows per wave step.  Lane q of a row
// holds the coefficients in slots 4k + q (k = 0..5), so every vector load instruction of a
// wave reads sixteen 32-byte pieces (four consecutive coefficients of sixteen rows) and
// every attitude access of a quad covers the four consecutive columns t..t+3 of one axis:
//
//   q = 0 : slots 0 4 8 12 16 20   astro 0, astro 4, att j=3 (axes 0,1,2), instr 3
//   q = 1 : slots 1 5 9 13 17 21   astro 1, att j=0 (axes 0,1,2), instr 0, instr 4
//   q = 2 : slots 2 6 10 14 18 22  astro 2, att j=1 (axes 0,1,2), instr 1, instr 5
//   q = 3 : slots 3 7 11 15 19 23  astro 3, att j=2 (axes 0,1,2), instr 2, global
//
// Waves walk contiguous chunks of rows, so runs of equal keys (the star of a row in the
// star-ordered pass, the attitude start t in the attitude pass) are reduced in registers
// with a segmented scan across the 16 row groups plus a carry between steps; a run is
// written once when it ends.
#pragma once

#include "kernels.hpp"

namespace gsr {

constexpr int kQuad = 4;          // lanes per row
constexpr int kStepRows = kWave / kQuad;  // rows per wave step (16)

__device__ __forceinline__ double ld_val(const double* __restrict__ p) {
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ double ld_val(const float* __restrict__ p) {
    return (double)__builtin_nontemporal_load(p);
}

__device__ __forceinline__ double quad_sum(double v) {
    v += __shfl_xor(v, 1, kWave);
    v += __shfl_xor(v, 2, kWave);
    return v;
}

// Inclusive segmented scan over the row groups of a wave (lane = STRIDE * group + q),
// segments given by equal `key` (keys of a segment are contiguous).  NV values per lane.
template <int NV, int STRIDE = kQuad>
__device__ __forceinline__ void seg_scan_rows(int32_t key, double (&v)[NV], int lane) {
#pragma unroll
    for (int off = STRIDE; off < kWave; off <<= 1) {
        const int32_t kk = __shfl_up(key, off, kWave);
        double o[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) o[j] = __shfl_up(v[j], off, kWave);
        if (lane >= off && kk == key) {
#pragma unroll
            for (int j = 0; j < NV; ++j) v[j] += o[j];
        }
    }
}

// ---------------------------------------------------------------------------------------
// aprod 1:  sum_i = sum_k A[i,k] xx[col(i,k)], then
//   A1_ADD   : y[i] += sum_i
//   A1_LSQR  : y[i] = xs sum_i - ys y[i]  with (xs, ys) = (sv, alpha su)   [forward operator]
//   A1_LSQR_T: same with (xs, ys) = (su, beta sv)                           [transposed]
//   A1_RESID : y[i] = b[i] - sum_i
// LSQR modes also write the block partial of sum y[i]^2.  The instrumental part of xx is
// staged in LDS when `lds_instr` is set (dynamic LDS of n_instr doubles).
enum { A1_ADD = 0, A1_LSQR = 1, A1_LSQR_T = 2, A1_RESID = 3 };

template <typename VT, int MODE>
static __global__ __launch_bounds__(512) void k_aprod1(
    Geo g, const VT* __restrict__ vals, const int32_t* __restrict__ star,
    const int32_t* __restrict__ att, const int32_t* __restrict__ instr,
    const double* __restrict__ xx, double* __restrict__ y, const double* __restrict__ b,
    const LsqrState* __restrict__ st, double* __restrict__ partials, int chunk_rows,
    int lds_instr) {
    extern __shared__ double lxi[];
    __shared__ double sh[512 / kWave];
    constexpr bool kLsqr = (MODE == A1_LSQR || MODE == A1_LSQR_T);
    double xs = 1.0, ys = 0.0;
    if (kLsqr) {
        if (st->stop) return;
        if (MODE == A1_LSQR) {
            xs = st->sv;
            ys = st->alpha * st->su;
        } else {
            xs = st->su;
            ys = st->beta * st->sv;
        }
    }
    if (lds_instr) {
        for (int k = threadIdx.x; k < g.I; k += blockDim.x) lxi[k] = xx[g.ins0 + k];
        __syncthreads();
    }
    const double* __restrict__ xi = lds_instr ? lxi : xx + g.ins0;
    const int lane = threadIdx.x % kWave, rg = lane / kQuad, q = lane % kQuad;
    const int wpb = blockDim.x / kWave;
    const int64_t nchunks = (g.m + chunk_rows - 1) / chunk_rows;
    const double xglob = xx[g.glb0];
    const int ia_off = (q == 0) ? 3 : q - 1;  // instrumental index of the lane's first slot
    const int ib_off = (q == 1 || q == 2) ? q + 3 : ia_off;
    const int jatt = (q + 3) & 3;             // attitude column offset of the lane
    double acc = 0.0;
    for (int64_t ch = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; ch < nchunks;
         ch += (int64_t)gridDim.x * wpb) {
        const int64_t r_end = min((ch + 1) * (int64_t)chunk_rows, g.m);
        for (int64_t r0 = ch * (int64_t)chunk_rows; r0 < r_end; r0 += kStepRows) {
            const int64_t r = r0 + rg;
            const bool valid = r < r_end;
            double sum = 0.0;
            if (valid) {
                const VT* __restrict__ row = vals + r * kPar + q;
                double a[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) a[k] = ld_val(row + 4 * k);
                const int32_t s = star[r], t = att[r];
                const int32_t ia = instr[r * kInstr + ia_off];
                const int32_t ib = instr[r * kInstr + ib_off];
                const int64_t ca = (int64_t)kAstro * s;
                sum = a[0] * xx[ca + q];
                if (q == 0) sum = fma(a[1], xx[ca + 4], sum);
                const double* __restrict__ xa = xx + g.att0 + t + jatt;
#pragma unroll
                for (int ax = 0; ax < kAxes; ++ax) {
                    const double c = (q == 0) ? a[ax + 2] : a[ax + 1];
                    sum = fma(c, xa[(int64_t)ax * g.T], sum);
                }
                sum = fma((q == 0) ? a[5] : a[4], xi[ia], sum);
                if (q == 1 || q == 2) sum = fma(a[5], xi[ib], sum);
                if (q == 3) sum = fma(a[5], xglob, sum);
            }
            sum = quad_sum(sum);
            if (valid && q == 0) {
                if (MODE == A1_ADD) {
                    y[r] += sum;
                } else if (MODE == A1_RESID) {
                    y[r] = b[r] - sum;
                } else {
                    const double u = (ys != 0.0) ? xs * sum - ys * y[r] : xs * sum;
                    y[r] = u;
                    acc = fma(u, u, acc);
                }
            }
        }
    }
    if (kLsqr) {
        const double tot = block_sum<512>(acc, sh);
        if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    }
}

// ---------------------------------------------------------------------------------------
// aprod 2, star-ordered pass: astrometric, instrumental and global columns.
//   x[col(i,k)] += A[i,k] yy_i,  yy_i = y[i] (A2_ADD), su y[i] (A2_LSQR), sv y[i]
//   (A2_LSQR_T), or the contribution is A[i,k]^2 (A2_SQ, column norms).
// Astrometric: a star's rows are contiguous; a run is written once by the wave that ends it,
// with a plain read-modify-write when the whole star lies inside the wave's chunk and an
// atomic add when the star continues into a neighbouring chunk.
// Instrumental and global: accumulated in LDS for everything the block visits; the block's
// n_instr + 1 sums go to part[blockIdx] (reduced by k_reduce_partials), or -- when n_instr is
// too large for LDS -- straight to x with atomics.
enum { A2_ADD = 0, A2_LSQR = 1, A2_LSQR_T = 2, A2_SQ = 3 };

template <int MODE>
__device__ __forceinline__ double a2_scale(const LsqrState* __restrict__ st) {
    return MODE == A2_LSQR ? st->su : (MODE == A2_LSQR_T ? st->sv : 1.0);
}

template <int MODE>
__device__ __forceinline__ double contrib(double a, double yy) {
    return MODE == A2_SQ ? a * a : a * yy;
}

template <typename VT, int MODE>
static __global__ __launch_bounds__(512) void k_aprod2_star(
    Geo g, const VT* __restrict__ vals, const int32_t* __restrict__ star,
    const int32_t* __restrict__ instr, const double* __restrict__ y, double* __restrict__ x,
    const LsqrState* __restrict__ st, double* __restrict__ part, int chunk_rows, int lds_instr) {
    extern __shared__ double lds[];  // [n_instr] instrumental, [1] global (lds_instr)
    __shared__ double lglob_nolds;
    if ((MODE == A2_LSQR || MODE == A2_LSQR_T) && st->stop) return;
    const double ysc = a2_scale<MODE>(st);
    const int nI = lds_instr ? g.I : 0;
    double* lglob = lds_instr ? lds + nI : &lglob_nolds;
    for (int k = threadIdx.x; k < nI; k += blockDim.x) lds[k] = 0.0;
    if (threadIdx.x == 0) *lglob = 0.0;
    __syncthreads();

    const int lane = threadIdx.x % kWave, rg = lane / kQuad, q = lane % kQuad;
    const int wpb = blockDim.x / kWave;
    const int64_t nchunks = (g.m + chunk_rows - 1) / chunk_rows;
    double gacc = 0.0;
    for (int64_t ch = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; ch < nchunks;
         ch += (int64_t)gridDim.x * wpb) {
        const int64_t r_beg = ch * (int64_t)chunk_rows;
        const int64_t r_end = min(r_beg + chunk_rows, g.m);
        // stars shared with the neighbouring chunks are written with atomics
        const int32_t shared_first =
            (r_beg > 0 && star[r_beg - 1] == star[r_beg]) ? star[r_beg] : -1;
        const int32_t shared_last =
            (r_end < g.m && star[r_end] == star[r_end - 1]) ? star[r_end - 1] : -1;
        auto flush = [&](int32_t key, double v0, double v1) {
            double* xa = x + (int64_t)kAstro * key;
            if (key == shared_first || key == shared_last) {
                atomic_add_f64(xa + q, v0);
                if (q == 0) atomic_add_f64(xa + 4, v1);
            } else {
                xa[q] += v0;
                if (q == 0) xa[4] += v1;
            }
        };
        double c0 = 0.0, c1 = 0.0;  // carry of the open run (astro q; astro 4 on q = 0)
        int32_t ckey = -1;
        for (int64_t r0 = r_beg; r0 < r_end; r0 += kStepRows) {
            const int64_t r = r0 + rg;
            const bool valid = r < r_end;
            int32_t key = -1;
            double v[2] = {0.0, 0.0};
            if (valid) {
                const VT* __restrict__ row = vals + r * kPar + q;
                const double a0 = ld_val(row);
                const double a1 = (q == 0) ? ld_val(row + 4) : 0.0;
                const double a4 = (q != 0) ? ld_val(row + 16) : 0.0;
                const double a5 = ld_val(row + 20);
                key = star[r];
                const double yy = (MODE == A2_SQ) ? 0.0 : ysc * y[r];
                v[0] = contrib<MODE>(a0, yy);
                v[1] = contrib<MODE>(a1, yy);
                const double p4 = contrib<MODE>(a4, yy), p5 = contrib<MODE>(a5, yy);
                if (q != 0) {
                    const int32_t ia = instr[r * kInstr + q - 1];
                    if (lds_instr) atomicAdd(lds + ia, p4);
                    else atomic_add_f64(x + g.ins0 + ia, p4);
                }
                if (q != 3) {
                    const int32_t ib = instr[r * kInstr + 3 + q];
                    if (lds_instr) atomicAdd(lds + ib, p5);
                    else atomic_add_f64(x + g.ins0 + ib, p5);
                } else {
                    gacc += p5;
                }
            }
            // close or continue the run carried from the previous step
            if (rg == 0 && ckey >= 0) {
                if (key == ckey) {
                    v[0] += c0;
                    v[1] += c1;
                } else {
                    flush(ckey, c0, c1);
                }
            }
            seg_scan_rows<2>(key, v, lane);
            const int32_t knext = __shfl_down(key, kQuad, kWave);
            if (valid && rg < kStepRows - 1 && knext != key) flush(key, v[0], v[1]);
            c0 = __shfl(v[0], kWave - kQuad + q, kWave);
            c1 = __shfl(v[1], kWave - kQuad + q, kWave);
            ckey = __shfl(key, kWave - kQuad, kWave);
        }
        if (rg == 0 && ckey >= 0) flush(ckey, c0, c1);
    }
    const double gs = wave_sum(gacc);
    if (lane == 0) atomicAdd(lglob, gs);
    __syncthreads();
    if (lds_instr) {
        double* dst = part + (int64_t)blockIdx.x * (nI + 1);
        for (int k = threadIdx.x; k <= nI; k += blockDim.x) dst[k] = lds[k];
    } else if (threadIdx.x == 0) {
        atomic_add_f64(x + g.glb0, *lglob);
    }
}

// x[ins0 + c] += sum_b part[b][c] for the n_instr + 1 instrumental and global columns.
static __global__ void k_reduce_partials(int ncols, int nblocks, const double* __restrict__ part,
                                         double* __restrict__ x, const LsqrState* __restrict__ st,
                                         int check_stop) {
    if (check_stop && st->stop) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * ncols + c];
    x[c] += s;
}

// ---------------------------------------------------------------------------------------
// aprod 2, attitude pass over the library-owned copy sorted by attitude start t:
//   attT[k][4 a + j] = A[row_k, 5 + 4 a + j],  rowT[k] = row_k,  tT[k] = att[row_k].
// Lane q takes column t + q of the three axes; runs of equal t are reduced in registers and
// added to x once per run and wave chunk (atomic: chunks meet inside a run).
template <typename VT, int MODE>
static __global__ __launch_bounds__(256) void k_aprod2_att(
    Geo g, const VT* __restrict__ attT, const int32_t* __restrict__ rowT,
    const int32_t* __restrict__ tT, const double* __restrict__ y, double* __restrict__ x,
    const LsqrState* __restrict__ st, int chunk_rows) {
    if ((MODE == A2_LSQR || MODE == A2_LSQR_T) && st->stop) return;
    const double ysc = a2_scale<MODE>(st);
    const int lane = threadIdx.x % kWave, rg = lane / kQuad, q = lane % kQuad;
    const int wpb = blockDim.x / kWave;
    const int64_t nchunks = (g.m + chunk_rows - 1) / chunk_rows;
    double* __restrict__ xatt = x + g.att0 + q;
    auto flush = [&](int32_t key, const double (&v)[3]) {
#pragma unroll
        for (int ax = 0; ax < kAxes; ++ax) atomic_add_f64(xatt + (int64_t)ax * g.T + key, v[ax]);
    };
    for (int64_t ch = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; ch < nchunks;
         ch += (int64_t)gridDim.x * wpb) {
        const int64_t k_end = min((ch + 1) * (int64_t)chunk_rows, g.m);
        double c[3] = {0.0, 0.0, 0.0};
        int32_t ckey = -1;
        for (int64_t k0 = ch * (int64_t)chunk_rows; k0 < k_end; k0 += kStepRows) {
            const int64_t k = k0 + rg;
            const bool valid = k < k_end;
            int32_t key = -1;
            double v[3] = {0.0, 0.0, 0.0};
            if (valid) {
                key = tT[k];
                const double yy = (MODE == A2_SQ) ? 0.0 : ysc * y[rowT[k]];
                const VT* __restrict__ a = attT + k * (kAxes * kParAxis) + q;
#pragma unroll
                for (int ax = 0; ax < kAxes; ++ax)
                    v[ax] = contrib<MODE>(ld_val(a + kParAxis * ax), yy);
            }
            if (rg == 0 && ckey >= 0) {
                if (key == ckey) {
#pragma unroll
                    for (int ax = 0; ax < kAxes; ++ax) v[ax] += c[ax];
                } else {
                    flush(ckey, c);
                }
            }
            seg_scan_rows<3>(key, v, lane);
            const int32_t knext = __shfl_down(key, kQuad, kWave);
            if (valid && rg < kStepRows - 1 && knext != key) flush(key, v);
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax) c[ax] = __shfl(v[ax], kWave - kQuad + q, kWave);
            ckey = __shfl(key, kWave - kQuad, kWave);
        }
        if (rg == 0 && ckey >= 0) flush(ckey, c);
    }
}

// Library-owned attitude copy in t order: attT[k][j] = vals[rowT[k]][5 + j].
template <typename VT>
static __global__ void k_gather_att(int64_t m, const VT* __restrict__ vals,
                                    const int32_t* __restrict__ rowT, VT* __restrict__ attT) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = m * (kAxes * kParAxis);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t k = e / (kAxes * kParAxis);
        const int j = (int)(e % (kAxes * kParAxis));
        attT[e] = vals[(int64_t)rowT[k] * kPar + kAstro + j];
    }
}

static __global__ void k_iota(int64_t m, int32_t* __restrict__ v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
        v[i] = (int32_t)i;
}

}  // namespace gsr
