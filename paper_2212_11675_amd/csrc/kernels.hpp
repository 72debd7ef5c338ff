// Device kernels of the PC-LSQR hot path (arXiv 2212.11675) for gfx950.
//
// Matrix layout (Section 3): row i holds 24 coefficients in the slot order
// [5 astrometric | 3 axes x 4 attitude | 6 instrumental | 1 global]; star[i] selects the
// astrometric block, att[i] the start of the 4-wide block of every attitude axis (axis
// stride n_dfa), instr[6i..6i+5] the instrumental columns.  All sums are binary64; the
// coefficients are read as binary64 or from a binary32 copy (VT = float).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));

constexpr int kPar = 24;     // coefficients per row
constexpr int kAstro = 5;    // astrometric unknowns per star
constexpr int kAxes = 3;     // attitude axes
constexpr int kParAxis = 4;  // attitude coefficients per axis
constexpr int kInstr = 6;    // instrumental coefficients per row
constexpr int kWave = 64;    // gfx950 wavefront
constexpr int kBlock = 256;  // threads per block of the row kernels
constexpr int kInstrLdsMax = 10240;  // instrumental columns privatized in LDS (80 KiB)

// Column geometry of one system.
struct Geo {
    int64_t m;     // rows
    int64_t n;     // columns
    int64_t att0;  // first attitude column  = 5 n_stars
    int64_t ins0;  // first instrumental col = att0 + 3 n_dfa
    int64_t glb0;  // global column          = ins0 + n_instr
    int64_t n_stars;
    int32_t T;     // n_dfa
    int32_t I;     // n_instr
};

// Scalars of one LSQR recurrence, resident in device memory for the whole solve.
// The vectors are stored unnormalized: u = su * u~, v = sv * v~.
struct LsqrState {
    double alpha, beta;   // current alpha_i, beta_i
    double su, sv;        // 1/beta, 1/alpha (0 when the norm is 0)
    double rhobar, phibar;
    double f1, f2;        // pending update z += f1 w; w = sv v~ - f2 w
    double fb;            // extra z += fb w after an exact beta = 0 breakdown
    double anorm2, bnorm, rnorm, arnorm, znorm2;
    double atol, btol;
    double rinv, rinv_b;  // 1/rho of the pending update and of a breakdown step (variances)
    double ddnorm;        // sum ||w_i / rho_i||^2 (condition estimate)
    double ctol;          // 1 / conlim (0: no condition test)
    int32_t itn, itnlim, fixed, istop, stop, pending, pend_b, nonfinite;
};

// State of the residual-correction loop of the precision form, in device memory: once
// `stop` is set, the launches of later correction steps return at once.
struct RefState {
    int32_t stop;       // no further correction step
    int32_t n_refine;   // outer steps taken
    int32_t itn;        // inner iterations summed over the steps taken
    int32_t nonfinite;  // a non-finite value stopped an inner solve
};

// ---------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over a block of NT threads; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NT / kWave; ++k) r += sh[k];
    }
    return r;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v) {
    unsafeAtomicAdd(p, v);  // global_atomic_add_f64 (no CAS loop)
}

__device__ __forceinline__ void load_instr(const int32_t* __restrict__ instr, int64_t i,
                                           int32_t c[kInstr]) {
    const i32x2* r = reinterpret_cast<const i32x2*>(instr + i * kInstr);
#pragma unroll
    for (int k = 0; k < kInstr / 2; ++k) {
        const i32x2 t = __builtin_nontemporal_load(r + k);
        c[2 * k] = t.x;
        c[2 * k + 1] = t.y;
    }
}

// ---------------------------------------------------------------------------------------
// vectors

static __global__ void k_fill(double* __restrict__ v, int64_t n, double val) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        v[j] = val;
}

// p_j = 1/sqrt(ss_j) (0 for an empty column); ss is reset to 0; counts empty columns.
static __global__ void k_recip_sqrt(int64_t n, double* __restrict__ ss, double* __restrict__ p,
                             unsigned long long* __restrict__ n_empty) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long cnt = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        const double s = ss[j];
        ss[j] = 0.0;
        p[j] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        cnt += (s > 0.0) ? 0 : 1;
    }
    if (cnt) atomicAdd(n_empty, cnt);
}

// u = src (o p if PRE); block partial of sum u^2
// (PRE: also xt = p o u, the operand of the next aprod 1)
template <bool PRE>
static __global__ __launch_bounds__(kBlock) void k_copy_norm(int64_t n, const double* __restrict__ src,
                                                      const double* __restrict__ p,
                                                      double* __restrict__ u,
                                                      double* __restrict__ xt,
                                                      double* __restrict__ partials) {
    __shared__ double sh[kBlock / kWave];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        const double v = PRE ? src[j] * p[j] : src[j];
        u[j] = v;
        if (PRE) xt[j] = p[j] * v;
        acc = fma(v, v, acc);
    }
    const double tot = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Forward operator, after aprod 2 accumulated s = A^T (su u~):
//   INIT : v~ = p o s;                 z = 0, w = 0
//   else : apply the pending update  z += f1 w; w = sv v~ - f2 w  (old v~), then
//          v~ = p o s - beta sv v~
// s is reset to 0 and xt = p o v~ (the operand of the next aprod 1) is written.
// Partials (4 rows of G): sum v~^2, sum z^2, sum z w, sum w^2.
// VAR: also the variance estimate var += (w / rho)^2 with the w of the pending update.
template <bool INIT, bool VAR = false>
static __global__ __launch_bounds__(kBlock) void k_vec_v(int64_t n, double* __restrict__ s,
                                                  const double* __restrict__ p,
                                                  double* __restrict__ v, double* __restrict__ w,
                                                  double* __restrict__ z, double* __restrict__ xt,
                                                  const LsqrState* __restrict__ st,
                                                  double* __restrict__ partials,
                                                  double* __restrict__ var = nullptr) {
    __shared__ double sh[kBlock / kWave];
    if (!INIT && st->stop) return;
    const bool pending = !INIT && st->pending;
    const double f1 = st->f1, f2 = st->f2, sv = st->sv;
    const double c1 = INIT ? 0.0 : st->beta * st->sv;
    const double su = st->su;  // s holds A^T u~ unnormalized
    const double rinv = st->rinv;
    double avv = 0.0, azz = 0.0, azw = 0.0, aww = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        const double sj = s[j];
        s[j] = 0.0;
        double vn;
        if (INIT) {
            vn = p[j] * (su * sj);
            z[j] = 0.0;
            w[j] = 0.0;
            if (VAR) var[j] = 0.0;
        } else {
            const double vj = v[j];
            if (pending) {
                const double wj = w[j];
                if (VAR) {
                    const double d = wj * rinv;
                    var[j] = fma(d, d, var[j]);
                }
                const double zj = fma(f1, wj, z[j]);
                const double wn = sv * vj - f2 * wj;
                z[j] = zj;
                w[j] = wn;
                azz = fma(zj, zj, azz);
                azw = fma(zj, wn, azw);
                aww = fma(wn, wn, aww);
            }
            vn = p[j] * (su * sj) - c1 * vj;
        }
        v[j] = vn;
        xt[j] = p[j] * vn;
        avv = fma(vn, vn, avv);
    }
    const int G = gridDim.x;
    double tot = block_sum<kBlock>(avv, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    if (!INIT) {
        tot = block_sum<kBlock>(azz, sh);
        if (threadIdx.x == 0) partials[G + blockIdx.x] = tot;
        tot = block_sum<kBlock>(azw, sh);
        if (threadIdx.x == 0) partials[2 * G + blockIdx.x] = tot;
        tot = block_sum<kBlock>(aww, sh);
        if (threadIdx.x == 0) partials[3 * G + blockIdx.x] = tot;
    }
}

// Transposed operator, u-step after aprod 2 accumulated s = A^T v~ (unnormalized):
//   u~ = p o (sv s) - alpha su u~ ; s = 0 ; xt = p o u~ ; partial sum u~^2.
static __global__ __launch_bounds__(kBlock) void k_vec_tu(int64_t n, double* __restrict__ s,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ u, double* __restrict__ xt,
                                                   const LsqrState* __restrict__ st,
                                                   double* __restrict__ partials) {
    __shared__ double sh[kBlock / kWave];
    if (st->stop) return;
    const double c1 = st->alpha * st->su;
    const double sv = st->sv;  // s holds A^T v~ unnormalized
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        const double sj = s[j];
        s[j] = 0.0;
        const double un = p[j] * (sv * sj) - c1 * u[j];
        u[j] = un;
        xt[j] = p[j] * un;
        acc = fma(un, un, acc);
    }
    const double tot = block_sum<kBlock>(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Transposed operator: pending update in the (row-space) unknowns before v~ is replaced:
//   z += f1 w; w = sv v~ - f2 w.  Partials (3 rows of G): sum z^2, sum z w, sum w^2.
static __global__ __launch_bounds__(kBlock) void k_vec_zw(int64_t n, const double* __restrict__ v,
                                                   double* __restrict__ w,
                                                   double* __restrict__ z,
                                                   const LsqrState* __restrict__ st,
                                                   double* __restrict__ partials) {
    __shared__ double sh[kBlock / kWave];
    if (st->stop) return;
    const bool pending = st->pending;
    const double f1 = st->f1, f2 = st->f2, sv = st->sv;
    double azz = 0.0, azw = 0.0, aww = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    if (pending) {
        for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
            const double wj = w[j];
            const double zj = fma(f1, wj, z[j]);
            const double wn = sv * v[j] - f2 * wj;
            z[j] = zj;
            w[j] = wn;
            azz = fma(zj, zj, azz);
            azw = fma(zj, wn, azw);
            aww = fma(wn, wn, aww);
        }
    }
    const int G = gridDim.x;
    double tot = block_sum<kBlock>(azz, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    tot = block_sum<kBlock>(azw, sh);
    if (threadIdx.x == 0) partials[G + blockIdx.x] = tot;
    tot = block_sum<kBlock>(aww, sh);
    if (threadIdx.x == 0) partials[2 * G + blockIdx.x] = tot;
}

// End of a solve: apply the pending updates, out = p o z (PRE) or z.  VAR: the same for the
// variance estimate, var_out = p^2 o var (PRE) or var.
template <bool PRE, bool VAR = false>
static __global__ void k_final(int64_t n, const double* __restrict__ p, double* __restrict__ z,
                        double* __restrict__ w, const double* __restrict__ v,
                        double* __restrict__ out, const LsqrState* __restrict__ st,
                        double* __restrict__ var = nullptr, double* __restrict__ var_out = nullptr) {
    const bool pending = st->pending, pend_b = st->pend_b;
    const double f1 = st->f1, f2 = st->f2, sv = st->sv, fb = st->fb;
    const double rinv = st->rinv, rinv_b = st->rinv_b;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        double zj = z[j];
        double vr = VAR ? var[j] : 0.0;
        if (pending) {
            const double wj = w[j];
            zj = fma(f1, wj, zj);
            if (VAR) vr = fma(wj * rinv, wj * rinv, vr);
            const double wn = sv * v[j] - f2 * wj;
            if (pend_b) {
                zj = fma(fb, wn, zj);
                if (VAR) vr = fma(wn * rinv_b, wn * rinv_b, vr);
            }
            w[j] = wn;
        }
        z[j] = zj;
        out[j] = PRE ? p[j] * zj : zj;
        if (VAR) {
            var[j] = vr;
            var_out[j] = PRE ? p[j] * p[j] * vr : vr;
        }
    }
}

// ---------------------------------------------------------------------------------------
// scalar steps (one block of kBlock threads)

__device__ __forceinline__ double reduce_partials(const double* __restrict__ part, int G,
                                                  double* sh) {
    double acc = 0.0;
#pragma unroll 4
    for (int k = threadIdx.x; k < G; k += kBlock) acc += part[k];
    return block_sum<kBlock>(acc, sh);  // thread 0
}

// reduce_partials of four arrays at once (p0 of G0 entries; p1, p2, p3 of G1 each): the loads
// of all four are issued together and one shared-memory exchange serves them; the summation
// order of each array is that of reduce_partials.  Results valid in thread 0.
__device__ __forceinline__ void reduce_partials4(const double* __restrict__ p0, int G0,
                                                 const double* __restrict__ p1,
                                                 const double* __restrict__ p2,
                                                 const double* __restrict__ p3, int G1,
                                                 double (&out)[4],
                                                 double (&sh)[4][kBlock / kWave]) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k = threadIdx.x; k < G0; k += kBlock) a[0] += p0[k];
#pragma unroll 4
    for (int k = threadIdx.x; k < G1; k += kBlock) {
        a[1] += p1[k];
        a[2] += p2[k];
        a[3] += p3[k];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = wave_sum(a[q]);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sh[q][w] = a[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double r = 0.0;
#pragma unroll
            for (int k = 0; k < kBlock / kWave; ++k) r += sh[q][k];
            out[q] = r;
        }
    }
}

// The scalar recurrences of one LSQR instance (applied by one thread per instance).

// beta_1 = ||b||, u = b / beta_1.
__device__ __forceinline__ void scal_init1(LsqrState* st, double ss, int32_t itnlim, int32_t fixed,
                                           double atol, double btol, double conlim) {
    const double beta = sqrt(ss);
    LsqrState s = {};
    s.itnlim = itnlim;
    s.fixed = fixed;
    s.atol = atol;
    s.btol = btol;
    s.ctol = conlim > 0.0 ? 1.0 / conlim : 0.0;
    s.beta = beta;
    s.bnorm = beta;
    s.phibar = beta;
    s.rnorm = beta;
    s.su = beta > 0.0 ? 1.0 / beta : 0.0;
    s.nonfinite = !isfinite(beta);
    if (!(beta > 0.0)) {
        s.istop = 4;
        s.stop = 1;
    }
    *st = s;
}

// alpha_1 = ||v~||, v = v~ / alpha_1, w_1 = v_1 (applied by the first vector step).
__device__ __forceinline__ void scal_init2(LsqrState* st, double ss) {
    if (st->stop) return;
    const double alpha = sqrt(ss);
    st->alpha = alpha;
    st->sv = alpha > 0.0 ? 1.0 / alpha : 0.0;
    st->rhobar = alpha;
    st->arnorm = alpha * st->beta;
    st->f1 = 0.0;
    st->f2 = 0.0;
    st->pending = 1;  // w_1 = sv v~_1, z_0 = 0
    if (!isfinite(alpha)) st->nonfinite = 1;
    if (!(alpha > 0.0)) {
        st->istop = 3;
        st->stop = 1;
        st->pending = 0;
    } else if (st->itnlim <= 0) {
        st->stop = 1;
    }
}

// After the u-step: beta_{i+1} = ||u~||.  beta = 0 is an exact breakdown: the last Givens
// step is taken here and the iteration stops.
__device__ __forceinline__ void scal_beta(LsqrState* st, double ss) {
    if (st->stop) return;
    const double beta = sqrt(ss);
    const double alpha = st->alpha;
    st->anorm2 += alpha * alpha + beta * beta;
    st->beta = beta;
    if (!isfinite(beta)) {
        st->nonfinite = 1;
        st->stop = 1;
        return;
    }
    if (beta > 0.0) {
        st->su = 1.0 / beta;
        return;
    }
    // beta = 0: rho = |rhobar|, c = rhobar / rho, s = 0
    const double rhobar = st->rhobar;
    const double rho = sqrt(rhobar * rhobar);
    const double c = rhobar / rho;
    const double phi = c * st->phibar;
    st->fb = phi / rho;
    st->rinv_b = 1.0 / rho;
    st->pend_b = 1;
    st->rhobar = -c * alpha;
    st->phibar = 0.0;
    st->itn += 1;
    st->rnorm = 0.0;
    st->arnorm = 0.0;
    st->istop = 3;
    st->stop = 1;
}

// After the v-step: alpha_{i+1} = ||v~||, Givens rotation, stopping tests.  zz, zw, ww are
// sum z_{i-1}^2, sum z_{i-1} w_i, sum w_i^2, giving ||z_i||^2 without another pass.
__device__ __forceinline__ void scal_alpha(LsqrState* st, double vv, double zz, double zw,
                                           double ww) {
    if (st->stop) return;
    const double alpha = sqrt(vv);
    const double beta = st->beta;
    const double rhobar = st->rhobar, phibar = st->phibar;
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rhobar / rho, s = beta / rho;
    const double theta = s * alpha;
    const double phi = c * phibar;
    st->rhobar = -c * alpha;
    st->phibar = s * phibar;
    st->f1 = phi / rho;
    st->f2 = theta / rho;
    st->rinv = 1.0 / rho;
    st->pending = 1;
    st->alpha = alpha;
    st->sv = alpha > 0.0 ? 1.0 / alpha : 0.0;
    st->itn += 1;
    st->rnorm = st->phibar;
    st->arnorm = st->phibar * alpha * fabs(c);
    const double f1 = st->f1;
    st->znorm2 = fmax(zz + 2.0 * f1 * zw + f1 * f1 * ww, 0.0);
    if (!isfinite(alpha) || !isfinite(st->znorm2)) {
        st->nonfinite = 1;
        st->stop = 1;
        return;
    }
    // d_i = w_i / rho_i: its squared norm adds to the condition estimate
    st->ddnorm += ww * st->rinv * st->rinv;
    const double anorm = sqrt(st->anorm2);
    const double znorm = sqrt(st->znorm2);
    if (!(alpha > 0.0)) {
        st->istop = 3;
        st->stop = 1;
    } else if (!st->fixed) {
        // Paige & Saunders' tests in their order of precedence: the tolerances, the
        // condition estimate against conlim, the three at machine precision
        const double rnorm = st->rnorm, bnorm = st->bnorm;
        const double acond = anorm * sqrt(st->ddnorm);
        const double test2 = st->arnorm / (anorm * rnorm);
        const double test3 = 1.0 / acond;
        const double t1 = (rnorm / bnorm) / (1.0 + anorm * znorm / bnorm);
        int32_t why = 0;
        if (rnorm <= st->btol * bnorm + st->atol * anorm * znorm)
            why = 1;
        else if (st->arnorm <= st->atol * anorm * rnorm)
            why = 2;
        else if (test3 <= st->ctol)
            why = 5;
        else if (1.0 + t1 <= 1.0)
            why = 6;
        else if (1.0 + test2 <= 1.0)
            why = 7;
        else if (1.0 + test3 <= 1.0)
            why = 8;
        if (why) {
            st->istop = why;
            st->stop = 1;
        }
    }
    if (st->itn >= st->itnlim) st->stop = 1;
}

// gate (may be NULL): when *gate is set the solve is not started (st keeps the stopped state
// of the previous solve, so all its launches return at once).
static __global__ __launch_bounds__(kBlock) void k_scal_init1(LsqrState* st, const double* part,
                                                              int G, int32_t itnlim, int32_t fixed,
                                                              double atol, double btol,
                                                              double conlim,
                                                              const int32_t* gate = nullptr) {
    __shared__ double sh[kBlock / kWave];
    if (gate && *gate) return;
    const double ss = reduce_partials(part, G, sh);
    if (threadIdx.x == 0) scal_init1(st, ss, itnlim, fixed, atol, btol, conlim);
}

static __global__ __launch_bounds__(kBlock) void k_scal_init2(LsqrState* st, const double* part,
                                                              int G) {
    __shared__ double sh[kBlock / kWave];
    const double ss = reduce_partials(part, G, sh);
    if (threadIdx.x == 0) scal_init2(st, ss);
}

static __global__ __launch_bounds__(kBlock) void k_scal_beta(LsqrState* st, const double* part,
                                                             int G) {
    __shared__ double sh[kBlock / kWave];
    if (st->stop) return;
    const double ss = reduce_partials(part, G, sh);
    if (threadIdx.x == 0) scal_beta(st, ss);
}

// pz: partial sums of z_{i-1}^2, z_{i-1} w_i, w_i^2 (rows of Gz).
static __global__ __launch_bounds__(kBlock) void k_scal_alpha(LsqrState* st, const double* pv,
                                                              int Gv, const double* pz, int Gz) {
    __shared__ double sh[4][kBlock / kWave];
    if (st->stop) return;
    double r[4];
    reduce_partials4(pv, Gv, pz, pz + Gz, pz + 2 * Gz, Gz, r, sh);
    if (threadIdx.x == 0) scal_alpha(st, r[0], r[1], r[2], r[3]);
}

// ---------------------------------------------------------------------------------------
// precision form and gradient

static __global__ void k_to_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        dst[j] = (float)src[j];  // round to nearest even
}

// x += d; partials (2 rows of G): sum d^2, sum x^2.  Nothing once the loop has stopped.
static __global__ __launch_bounds__(kBlock) void k_axpy_norms(int64_t n, const double* __restrict__ d,
                                                       double* __restrict__ x,
                                                       double* __restrict__ partials,
                                                       const RefState* __restrict__ ref) {
    __shared__ double sh[kBlock / kWave];
    if (ref->stop) return;
    double add = 0.0, axx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        const double dj = d[j];
        const double xj = x[j] + dj;
        x[j] = xj;
        add = fma(dj, dj, add);
        axx = fma(xj, xj, axx);
    }
    double tot = block_sum<kBlock>(add, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    tot = block_sum<kBlock>(axx, sh);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = tot;
}

static __global__ void k_ref_begin(RefState* ref) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ref = RefState{0, 0, 0, 0};
}

// After correction step k (x += d_k done by k_axpy_norms): count the step and its inner
// iterations; the loop ends when ||d_k|| <= tol ||x||, after max_refine steps, or when the
// inner solve met a non-finite value.
static __global__ __launch_bounds__(kBlock) void k_ref_check(RefState* __restrict__ ref,
                                                             const LsqrState* __restrict__ st,
                                                             const double* __restrict__ part,
                                                             int G, double tol,
                                                             int32_t max_refine) {
    __shared__ double sh[kBlock / kWave];
    if (ref->stop) return;
    const double dd = reduce_partials(part, G, sh);
    const double xx = reduce_partials(part + G, G, sh);
    if (threadIdx.x != 0) return;
    RefState r = *ref;
    r.itn += st->itn;
    r.n_refine += 1;
    if (st->nonfinite) {
        r.nonfinite = 1;
        r.stop = 1;
    } else if (sqrt(dd) <= tol * sqrt(xx) || r.n_refine >= max_refine) {
        r.stop = 1;
    }
    *ref = r;
}

static __global__ void k_copy(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        dst[j] = src[j];
}

// dvals[i, k] = r_i lam_c - mu_i x_c  on the stored pattern.
static __global__ __launch_bounds__(kBlock) void k_grad_vals(Geo g, const int32_t* __restrict__ star,
                                                      const int32_t* __restrict__ att,
                                                      const int32_t* __restrict__ instr,
                                                      const double* __restrict__ r,
                                                      const double* __restrict__ mu,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ dvals) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < g.m; i += stride) {
        int32_t c[kInstr];
        load_instr(instr, i, c);
        const int32_t s = star[i], t = att[i];
        const double ri = r[i], mi = mu[i];
        double o[kPar];
        const int64_t ca = (int64_t)kAstro * s;
#pragma unroll
        for (int j = 0; j < kAstro; ++j) o[j] = ri * lam[ca + j] - mi * x[ca + j];
#pragma unroll
        for (int ax = 0; ax < kAxes; ++ax) {
            const int64_t cb = g.att0 + (int64_t)ax * g.T + t;
#pragma unroll
            for (int j = 0; j < kParAxis; ++j)
                o[kAstro + ax * kParAxis + j] = ri * lam[cb + j] - mi * x[cb + j];
        }
#pragma unroll
        for (int j = 0; j < kInstr; ++j) {
            const int64_t cc = g.ins0 + c[j];
            o[17 + j] = ri * lam[cc] - mi * x[cc];
        }
        o[23] = ri * lam[g.glb0] - mi * x[g.glb0];
        f64x2* dst = reinterpret_cast<f64x2*>(dvals + i * kPar);
#pragma unroll
        for (int k = 0; k < kPar / 2; ++k) dst[k] = f64x2{o[2 * k], o[2 * k + 1]};
    }
}

// Index checks: bit 0 star out of range, bit 1 stars not sorted, bit 2 attitude start out
// of range, bit 3 instrumental index out of range.
static __global__ void k_validate(Geo g, const int32_t* __restrict__ star,
                           const int32_t* __restrict__ att, const int32_t* __restrict__ instr,
                           int* __restrict__ flags) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.m; i += stride) {
        const int32_t s = star[i];
        if (s < 0 || s >= g.n_stars) bad |= 1;
        if (i > 0 && star[i - 1] > s) bad |= 2;
        const int32_t t = att[i];
        if (t < 0 || t > g.T - kParAxis) bad |= 4;
        for (int j = 0; j < kInstr; ++j) {
            const int32_t c = instr[i * kInstr + j];
            if (c < 0 || c >= g.I) bad |= 8;
        }
    }
    if (bad) atomicOr(flags, bad);
}

}  // namespace gsr
