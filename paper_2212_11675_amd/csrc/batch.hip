// Batched form: n_sys independent systems stored back to back, K right-hand sides each,
// solved together (declarations and contracts in include/gsr.h).
//
// Every (system, right-hand side) pair runs its own PC-LSQR recurrence (LsqrState per
// pair); the matrix of each system is read once per product for all K right-hand sides
// (sparse matrix times K-column block, RHS-minor storage so the K values of one row or
// column form one contiguous 8K-byte piece).  Lane layout: K lanes per row, lane j = RHS j.
// Work is described by lists of segments that never cross a system boundary:
//   row chunks    (one wave walks a chunk: products, row-space vector steps, partial sums),
//   block chunks  (one block walks a chunk: star-ordered pass of aprod 2, LDS per system),
//   column tiles  (one block: unknown-space vector steps).
// A whole fixed-iteration solve is captured in one hipGraph and launched once.  Chunk
// length and block shape are picked per batch shape by timing candidates (autotuner).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gsr_internal.hpp"
#include "products.hpp"

#include <hipcub/hipcub.hpp>

namespace gsr {

struct SysDesc {
    int64_t row0, m;   // rows [row0, row0 + m) of the concatenated arrays
    int64_t col0, n;   // unknowns [col0, col0 + n) of the batched vector
    int64_t att0, ins0, glb0;  // section bases relative to col0
    int64_t n_stars;
    int32_t T, I;
    int32_t chunk0, nchunk;    // row chunks of the system
    int32_t tile0, ntile;      // column tiles of the system
    int32_t bchunk0, nbchunk;  // block chunks of the system
    int64_t btile0;            // first row tile of the system (rows padded to whole tiles)
};

struct Seg {
    int64_t e0, e1;  // rows or columns (global)
    int32_t sys, pad;
};

constexpr int kBTile = 2048;  // columns per tile

// Block index renumbered so that the blocks of one die are consecutive: contiguous work
// ranges (one or a few systems) then stay on one die and share its L2.
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int per = G / kXcd, rem = G % kXcd;
    const int x = b % kXcd, i = b / kXcd;
    return x * per + min(x, rem) + i;
}

// ---------------------------------------------------------------------------------------
// products

// Y[r, j] (op)= sum_k A[r,k] X[col0 + col(r,k), j]
template <typename VT, int MODE, int K>
static __global__ __launch_bounds__(256) void k_baprod1(
    const SysDesc* __restrict__ sys, const Seg* __restrict__ chunks, int nchunks,
    const VT* __restrict__ vals, const int32_t* __restrict__ star,
    const int32_t* __restrict__ att, const int32_t* __restrict__ instr,
    const double* __restrict__ X, double* __restrict__ Y, const double* __restrict__ B,
    const LsqrState* __restrict__ st, double* __restrict__ partials) {
    constexpr bool kLsqr = (MODE == A1_LSQR);
    constexpr int RS = kWave / K;  // rows per wave step
    const int lane = threadIdx.x % kWave, rr = lane / K, j = lane % K;
    const int wpb = blockDim.x / kWave;
    for (int ch = blockIdx.x * wpb + threadIdx.x / kWave; ch < nchunks; ch += gridDim.x * wpb) {
        const Seg c = chunks[ch];
        const SysDesc d = sys[c.sys];
        bool live = true;
        double xs = 1.0, ys = 0.0;
        if (kLsqr) {
            const LsqrState* p = st + (int64_t)c.sys * K + j;
            live = !p->stop;
            xs = p->sv;
            ys = p->alpha * p->su;
        }
        const double* __restrict__ Xs = X + d.col0 * K + j;
        double acc = 0.0;
        for (int64_t r0 = c.e0; r0 < c.e1; r0 += RS) {
            const int64_t r = r0 + rr;
            if (!(live && r < c.e1)) continue;
            const VT* __restrict__ row = vals + r * kPar;
            double a[kPar];
#pragma unroll
            for (int k = 0; k < kPar; ++k) a[k] = ld_val(row + k);
            const int32_t s = star[r], t = att[r];
            int32_t ins[kInstr];
#pragma unroll
            for (int k = 0; k < kInstr; ++k) ins[k] = instr[r * kInstr + k];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < kAstro; ++k) sum = fma(a[k], Xs[((int64_t)kAstro * s + k) * K], sum);
#pragma unroll
            for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                for (int k = 0; k < kParAxis; ++k)
                    sum = fma(a[kAstro + ax * kParAxis + k],
                              Xs[(d.att0 + (int64_t)ax * d.T + t + k) * K], sum);
#pragma unroll
            for (int k = 0; k < kInstr; ++k) sum = fma(a[17 + k], Xs[(d.ins0 + ins[k]) * K], sum);
            sum = fma(a[23], Xs[d.glb0 * K], sum);
            double* yp = Y + r * K + j;
            if (MODE == A1_ADD) {
                *yp += sum;
            } else if (MODE == A1_RESID) {
                *yp = B[r * K + j] - sum;
            } else {
                const double u = (ys != 0.0) ? xs * sum - ys * *yp : xs * sum;
                *yp = u;
                acc = fma(u, u, acc);
            }
        }
        if (kLsqr) {
#pragma unroll
            for (int off = K; off < kWave; off <<= 1) acc += __shfl_xor(acc, off, kWave);
            if (lane < K) partials[(int64_t)ch * K + j] = acc;
        }
    }
}

// Star-ordered pass of X[c, j] += A[r, c] yy[r, j] (astrometric, instrumental, global).
// Block chunks are walked by whole blocks; each wave takes a contiguous sub-range.  The
// instrumental and global sums of the current system live in LDS and are added to X with
// one atomic per (column, j) when the block moves to another system or finishes.
template <typename VT, int MODE, int K>
static __global__ __launch_bounds__(512) void k_baprod2_star(
    const SysDesc* __restrict__ sys, const Seg* __restrict__ bchunks, int nbchunks,
    const VT* __restrict__ vals, const int32_t* __restrict__ star,
    const int32_t* __restrict__ instr, const double* __restrict__ Y, double* __restrict__ X,
    const LsqrState* __restrict__ st, int max_instr) {
    extern __shared__ double lds[];  // [(max_instr + 1) * K]
    constexpr int RS = kWave / K;
    const int lane = threadIdx.x % kWave, rr = lane / K, j = lane % K;
    const int w = threadIdx.x / kWave, wpb = blockDim.x / kWave;
    const int per = (nbchunks + gridDim.x - 1) / gridDim.x;
    const int bc_beg = xcd_block(blockIdx.x, gridDim.x) * per, bc_end = min(nbchunks, bc_beg + per);
    const int nl = (max_instr + 1) * K;
    for (int e = threadIdx.x; e < nl; e += blockDim.x) lds[e] = 0.0;
    __syncthreads();
    int cur = -1;
    SysDesc d = {};
    double gacc = 0.0;
    auto flush_lds = [&]() {
        const double gs = [&] {
            double v = gacc;
#pragma unroll
            for (int off = K; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
            return v;
        }();
        if (lane < K) atomicAdd(lds + d.I * K + j, gs);
        gacc = 0.0;
        __syncthreads();
        const int ne = (d.I + 1) * K;
        double* xi = X + (d.col0 + d.ins0) * K;  // instrumental then global: contiguous
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            const double v = lds[e];
            if (v != 0.0) atomic_add_f64(xi + e, v);
            lds[e] = 0.0;
        }
        __syncthreads();
    };
    for (int bc = bc_beg; bc < bc_end; ++bc) {
        const Seg c = bchunks[bc];
        if (c.sys != cur) {
            if (cur >= 0) flush_lds();
            cur = c.sys;
            d = sys[cur];
        }
        bool live = true;
        double ysc = 1.0;
        if (MODE == A2_LSQR) {
            const LsqrState* p = st + (int64_t)cur * K + j;
            live = !p->stop;
            ysc = 1.0;  // u~ unnormalized; k_bvec_v applies 1/beta
        }
        // this wave's contiguous sub-range of the block chunk
        const int64_t len = c.e1 - c.e0;
        const int64_t sub = ((len + wpb - 1) / wpb + RS - 1) / RS * RS;
        const int64_t r_beg = min(c.e1, c.e0 + w * sub), r_end = min(c.e1, r_beg + sub);
        const int64_t sys_end = d.row0 + d.m;
        const int32_t shared_first =
            (r_beg < r_end && r_beg > d.row0 && star[r_beg - 1] == star[r_beg]) ? star[r_beg] : -1;
        const int32_t shared_last =
            (r_beg < r_end && r_end < sys_end && star[r_end] == star[r_end - 1]) ? star[r_end - 1]
                                                                                : -1;
        double* __restrict__ Xa = X + d.col0 * K + j;
        // finished star: the lanes of row group 0 write it (S starts at zero in the LSQR and
        // column-norm modes, so an owned star is stored)
        auto flush = [&](int32_t key, const double (&t)[kAstro]) {
            if (rr != 0 || !live) return;
            double* xa = Xa + (int64_t)kAstro * key * K;
            if (key == shared_first || key == shared_last) {
#pragma unroll
                for (int q = 0; q < kAstro; ++q) atomic_add_f64(xa + q * K, t[q]);
            } else if (MODE == A2_ADD) {
#pragma unroll
                for (int q = 0; q < kAstro; ++q) xa[q * K] += t[q];
            } else {
#pragma unroll
                for (int q = 0; q < kAstro; ++q) xa[q * K] = t[q];
            }
        };
        double acc[kAstro] = {0.0, 0.0, 0.0, 0.0, 0.0};
        int32_t ckey = -1;
        for (int64_t r0 = r_beg; r0 < r_end; r0 += RS) {
            const int64_t r = r0 + rr;
            const bool valid = live && r < r_end;
            int32_t key = -1;
            double v[kAstro] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (valid) {
                const VT* __restrict__ row = vals + r * kPar;
                key = star[r];
                const double yy = (MODE == A2_SQ) ? 0.0 : ysc * Y[r * K + j];
#pragma unroll
                for (int q = 0; q < kAstro; ++q) v[q] = contrib<MODE>(ld_val(row + q), yy);
#pragma unroll
                for (int q = 0; q < kInstr; ++q) {
                    const int32_t ic = instr[r * kInstr + q];
                    atomicAdd(lds + ic * K + j, contrib<MODE>(ld_val(row + 17 + q), yy));
                }
                gacc += contrib<MODE>(ld_val(row + 23), yy);
            }
            run_step<kAstro, K>(key, v, acc, ckey, flush);
        }
        run_close<kAstro, K>(acc, ckey, flush);
    }
    if (cur >= 0) flush_lds();
}

// Batched row tiles: per system, kStepRows consecutive rows; every lane of a row needs all
// of the row's coefficients, so a tile is [12 pairs][16 rows][2] (one 256-byte block per
// load instruction) and the index tile [16 rows][8] = (star, att, instr0..5).
constexpr int kBTileVals = kStepRows * kPar;  // 384 doubles
constexpr int kBTileIdx = kStepRows * 8;      // 128 int32

static __global__ void k_make_btiles(int64_t m, int64_t ntiles, const double* __restrict__ vals,
                                     const int32_t* __restrict__ star,
                                     const int32_t* __restrict__ att,
                                     const int32_t* __restrict__ instr, double* __restrict__ vt,
                                     int32_t* __restrict__ it) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ntiles * kBTileVals;
         e += stride) {
        const int64_t tile = e / kBTileVals;
        const int o = (int)(e - tile * kBTileVals);
        const int pair = o / (2 * kStepRows), rg = (o / 2) % kStepRows, h = o % 2;
        const int64_t row = tile * kStepRows + rg;
        vt[e] = row < m ? vals[row * kPar + 2 * pair + h] : 0.0;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ntiles * kBTileIdx;
         e += stride) {
        const int64_t tile = e / kBTileIdx;
        const int o = (int)(e - tile * kBTileIdx);
        const int rg = o / 8, c = o % 8;
        const int64_t row = min(tile * kStepRows + rg, m - 1);
        it[e] = c == 0 ? star[row] : c == 1 ? att[row] : instr[row * kInstr + c - 2];
    }
}

// Attitude tiles of the t-ordered copy, per system as the row tiles: [6 pairs][16 rows][2]
// holding the 12 attitude coefficients of t-ordered rows row0 + 16 tile + rg (global row
// numbers in rowT).
constexpr int kBTileAtt = kStepRows * kAxes * kParAxis;  // 192 doubles

static __global__ void k_make_batt_tiles(int64_t m, int64_t ntiles, int64_t row0,
                                         const double* __restrict__ vals,
                                         const int32_t* __restrict__ rowT,
                                         double* __restrict__ at) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ntiles * kBTileAtt;
         e += stride) {
        const int64_t tile = e / kBTileAtt;
        const int o = (int)(e - tile * kBTileAtt);
        const int pair = o / (2 * kStepRows), rg = (o / 2) % kStepRows, h = o % 2;
        const int64_t lr = tile * kStepRows + rg;
        at[e] = lr < m ? vals[(int64_t)rowT[row0 + lr] * kPar + kAstro + 2 * pair + h] : 0.0;
    }
}

// R consecutive doubles (16-byte pieces when R is even; p then 16-byte aligned).
template <int R>
__device__ __forceinline__ void ld_r(const double* __restrict__ p, double (&o)[R]) {
    if constexpr (R % 2 == 0) {
#pragma unroll
        for (int i = 0; i < R; i += 2) {
            const f64x2 t = *reinterpret_cast<const f64x2*>(p + i);
            o[i] = t.x;
            o[i + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) o[i] = p[i];
    }
}
template <int R>
__device__ __forceinline__ void st_r(double* __restrict__ p, const double (&v)[R]) {
    if constexpr (R % 2 == 0) {
#pragma unroll
        for (int i = 0; i < R; i += 2) *reinterpret_cast<f64x2*>(p + i) = f64x2{v[i], v[i + 1]};
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) p[i] = v[i];
    }
}

// The three coefficient pairs m[] held by quad lane CTRL / 0x55, broadcast to the whole quad
// as six doubles (quad_perm [s,s,s,s] = s * 0x55).
template <int CTRL>
__device__ __forceinline__ void bcast_pairs(const f64x2 (&m)[3], double* __restrict__ out) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        out[2 * i] = dpp_f64<CTRL>(m[i].x);
        out[2 * i + 1] = dpp_f64<CTRL>(m[i].y);
    }
}

// Fused batched row pass: for every (row, rhs j) of a block chunk
//   U[r, j] = sv_j (A XT)[r, j] - alpha_j su_j U[r, j]
// and S += A^T U (astrometric: run accumulators; instrumental/global: LDS of the current
// system), reading each row once.  Sum U^2 per (block chunk, j) -> partials.
// Lane layout: L = min(K, 4) lanes per row, each lane R = K / L right-hand sides, so one row
// costs 16-byte loads: the row's coefficients (with L = 4 each lane reads a quarter and the
// quad exchanges them; otherwise all L lanes read the same 192 bytes), and per column the
// lane's R consecutive values of the K-column block (RHS-minor storage).
// Pairs that have stopped keep their U unchanged and contribute nothing.
template <typename VT, int K>
static __global__ __launch_bounds__(512) void k_baprod12(
    const SysDesc* __restrict__ sys, const Seg* __restrict__ bchunks, int nbchunks,
    const double* __restrict__ vt, const int32_t* __restrict__ it,
    const int32_t* __restrict__ star,
    const double* __restrict__ XT, double* __restrict__ U, double* __restrict__ S,
    const LsqrState* __restrict__ st, double* __restrict__ partials, int max_instr) {
    // [(max_instr + 1) * K] sums, [K] block sum U^2, [max_instr * K] instrumental part of XT
    extern __shared__ double lds[];
    constexpr int L = K >= 4 ? 4 : K;
    constexpr int R = K / L;
    constexpr int RS = kWave / L;
    const int lane = threadIdx.x % kWave, rr = lane / L, j0 = (lane % L) * R;
    const int w = threadIdx.x / kWave, wpb = blockDim.x / kWave;
    // Each XCD takes an eighth of the block chunks (in system order) and deals them to its
    // blocks in turn, so that its blocks move through the systems together and share each
    // system's attitude columns in the XCD's L2 (consecutive blocks go to consecutive XCDs).
    const int ngrp = min((int)gridDim.x, kXcd);
    const int grp = blockIdx.x % ngrp, gi = blockIdx.x / ngrp;
    const int nbg = gridDim.x / ngrp + (grp < (int)gridDim.x % ngrp ? 1 : 0);
    const int bc_beg = (int)((int64_t)nbchunks * grp / ngrp);
    const int bc_end = (int)((int64_t)nbchunks * (grp + 1) / ngrp);
    const int nl = (max_instr + 1) * K;
    double* lusq = lds + nl;
    double* lxi = lusq + K;
    for (int e = threadIdx.x; e < nl + K; e += blockDim.x) lds[e] = 0.0;
    __syncthreads();
    int cur = -1;
    SysDesc d = {};
    double gacc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) gacc[i] = 0.0;
    auto flush_lds = [&]() {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            double gs = gacc[i];
#pragma unroll
            for (int off = L; off < kWave; off <<= 1) gs += __shfl_xor(gs, off, kWave);
            if (lane < L) atomicAdd(lds + d.I * K + j0 + i, gs);
            gacc[i] = 0.0;
        }
        __syncthreads();
        const int ne = (d.I + 1) * K;
        double* xi = S + (d.col0 + d.ins0) * K;  // instrumental then global: contiguous
        for (int e = threadIdx.x; e < ne; e += blockDim.x) {
            const double v = lds[e];
            if (v != 0.0) atomic_add_f64(xi + e, v);
            lds[e] = 0.0;
        }
        __syncthreads();
    };
    for (int bc = bc_beg + gi; bc < bc_end; bc += nbg) {
        const Seg c = bchunks[bc];
        if (c.sys != cur) {
            if (cur >= 0) flush_lds();
            cur = c.sys;
            d = sys[cur];
            // the system's instrumental columns of XT, read from LDS below
            const double* xs_i = XT + (d.col0 + d.ins0) * K;
            for (int e = threadIdx.x; e < d.I * K; e += blockDim.x) lxi[e] = xs_i[e];
            __syncthreads();
        }
        bool live[R];
        double xs[R], ys[R];
        bool any_live = false;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const LsqrState* ps = st + (int64_t)cur * K + j0 + i;
            live[i] = !ps->stop;
            xs[i] = ps->sv;
            ys[i] = ps->alpha * ps->su;
            any_live = any_live || live[i];
        }
        if constexpr (L == 4) {
            // the quad of a row shares its loads: it goes through the row while any pair of
            // the system is live (a lane whose own pairs have stopped adds zeros)
#pragma unroll
            for (int j = 0; j < K; ++j) any_live = any_live || !st[(int64_t)cur * K + j].stop;
        }
        const int64_t len = c.e1 - c.e0;
        const int64_t sub = ((len + wpb - 1) / wpb + RS - 1) / RS * RS;
        const int64_t r_beg = min(c.e1, c.e0 + w * sub), r_end = min(c.e1, r_beg + sub);
        const int64_t sys_end = d.row0 + d.m;
        const int32_t shared_first =
            (r_beg < r_end && r_beg > d.row0 && star[r_beg - 1] == star[r_beg]) ? star[r_beg] : -1;
        const int32_t shared_last =
            (r_beg < r_end && r_end < sys_end && star[r_end] == star[r_end - 1]) ? star[r_end - 1]
                                                                                : -1;
        const double* __restrict__ Xs = XT + d.col0 * K + j0;
        double* __restrict__ Sa = S + d.col0 * K + j0;
        auto flush = [&](int32_t key, const double (&t)[kAstro * R]) {
            if (rr != 0) return;
            double* xa = Sa + (int64_t)kAstro * key * K;
            const bool shared = key == shared_first || key == shared_last;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                if (!live[i]) continue;
#pragma unroll
                for (int q = 0; q < kAstro; ++q) {
                    if (shared)
                        atomic_add_f64(xa + q * K + i, t[i * kAstro + q]);
                    else
                        xa[q * K + i] = t[i * kAstro + q];  // S is zero here
                }
            }
        };
        // the lane's R values of column `col` of XT
        auto xv = [&](int64_t col, double (&o)[R]) { ld_r<R>(Xs + col * K, o); };
        double acc[kAstro * R];
#pragma unroll
        for (int q = 0; q < kAstro * R; ++q) acc[q] = 0.0;
        int32_t ckey = -1;
        double usq[R];
#pragma unroll
        for (int i = 0; i < R; ++i) usq[i] = 0.0;
        for (int64_t r0 = r_beg; r0 < r_end; r0 += RS) {
            const int64_t r = r0 + rr;
            const bool valid = any_live && r < r_end;
            int32_t key = -1;
            double v[kAstro * R];
#pragma unroll
            for (int q = 0; q < kAstro * R; ++q) v[q] = 0.0;
            if (valid) {
                // the row's tile (the system's rows are padded to whole tiles)
                const int64_t lr = r - d.row0;
                const int64_t tile = d.btile0 + lr / kStepRows;
                const int rgl = (int)(lr % kStepRows);
                double a[kPar];
                int32_t sr, tr, ins[kInstr];
                const f64x2* vp = reinterpret_cast<const f64x2*>(vt + tile * kBTileVals) + rgl;
                const int32_t* ip = it + tile * kBTileIdx + rgl * 8;
                if constexpr (L == 4) {
                    // the row's quad splits its loads (lane q: coefficient pairs 3q..3q+2 and
                    // index slots 2q, 2q+1) and exchanges them with DPP quad broadcasts
                    const int q = lane & 3;
                    const f64x2 m[3] = {__builtin_nontemporal_load(vp + (3 * q) * kStepRows),
                                        __builtin_nontemporal_load(vp + (3 * q + 1) * kStepRows),
                                        __builtin_nontemporal_load(vp + (3 * q + 2) * kStepRows)};
                    const i32x2 iv =
                        __builtin_nontemporal_load(reinterpret_cast<const i32x2*>(ip) + q);
                    bcast_pairs<0x00>(m, a + 0);
                    bcast_pairs<0x55>(m, a + 6);
                    bcast_pairs<0xAA>(m, a + 12);
                    bcast_pairs<0xFF>(m, a + 18);
                    sr = __builtin_amdgcn_update_dpp(0, iv.x, 0x00, 0xF, 0xF, false);
                    tr = __builtin_amdgcn_update_dpp(0, iv.y, 0x00, 0xF, 0xF, false);
                    ins[0] = __builtin_amdgcn_update_dpp(0, iv.x, 0x55, 0xF, 0xF, false);
                    ins[1] = __builtin_amdgcn_update_dpp(0, iv.y, 0x55, 0xF, 0xF, false);
                    ins[2] = __builtin_amdgcn_update_dpp(0, iv.x, 0xAA, 0xF, 0xF, false);
                    ins[3] = __builtin_amdgcn_update_dpp(0, iv.y, 0xAA, 0xF, 0xF, false);
                    ins[4] = __builtin_amdgcn_update_dpp(0, iv.x, 0xFF, 0xF, 0xF, false);
                    ins[5] = __builtin_amdgcn_update_dpp(0, iv.y, 0xFF, 0xF, 0xF, false);
                } else {
#pragma unroll
                    for (int k = 0; k < kPar / 2; ++k) {
                        const f64x2 t = __builtin_nontemporal_load(vp + k * kStepRows);
                        a[2 * k] = t.x;
                        a[2 * k + 1] = t.y;
                    }
                    typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
                    const i32x4* ip4 = reinterpret_cast<const i32x4*>(ip);
                    const i32x4 i0 = __builtin_nontemporal_load(ip4);
                    const i32x4 i1 = __builtin_nontemporal_load(ip4 + 1);
                    sr = i0.x;
                    tr = i0.y;
                    ins[0] = i0.z;
                    ins[1] = i0.w;
                    ins[2] = i1.x;
                    ins[3] = i1.y;
                    ins[4] = i1.z;
                    ins[5] = i1.w;
                }
                double sum[R], xv_[R];
#pragma unroll
                for (int i = 0; i < R; ++i) sum[i] = 0.0;
                auto add = [&](double coef, int64_t col) {
                    xv(col, xv_);
#pragma unroll
                    for (int i = 0; i < R; ++i) sum[i] = fma(coef, xv_[i], sum[i]);
                };
#pragma unroll
                for (int k = 0; k < kAstro; ++k) add(a[k], (int64_t)kAstro * sr + k);
#pragma unroll
                for (int ax = 0; ax < kAxes; ++ax)
#pragma unroll
                    for (int k = 0; k < kParAxis; ++k)
                        add(a[kAstro + ax * kParAxis + k], d.att0 + (int64_t)ax * d.T + tr + k);
#pragma unroll
                for (int k = 0; k < kInstr; ++k) {
                    double xl[R];
#pragma unroll
                    for (int i = 0; i < R; ++i) xl[i] = lxi[ins[k] * K + j0 + i];
#pragma unroll
                    for (int i = 0; i < R; ++i) sum[i] = fma(a[17 + k], xl[i], sum[i]);
                }
                add(a[23], d.glb0);
                double* up = U + r * K + j0;
                double uo[R], un[R];
                ld_r<R>(up, uo);
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    un[i] = !live[i]       ? uo[i]
                            : (ys[i] != 0.0) ? xs[i] * sum[i] - ys[i] * uo[i]
                                             : xs[i] * sum[i];
                    const double ul = live[i] ? un[i] : 0.0;
                    usq[i] = fma(ul, ul, usq[i]);
#pragma unroll
                    for (int q = 0; q < kAstro; ++q) v[i * kAstro + q] = a[q] * ul;
                    gacc[i] = fma(a[23], ul, gacc[i]);
                }
                st_r<R>(up, un);
                key = sr;
#pragma unroll
                for (int k = 0; k < kInstr; ++k)
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (live[i]) atomicAdd(lds + ins[k] * K + j0 + i, a[17 + k] * un[i]);
            }
            run_step<kAstro * R, L>(key, v, acc, ckey, flush);
        }
        run_close<kAstro * R, L>(acc, ckey, flush);
        // block sum of U^2 for this block chunk
#pragma unroll
        for (int i = 0; i < R; ++i) {
            double t = usq[i];
#pragma unroll
            for (int off = L; off < kWave; off <<= 1) t += __shfl_xor(t, off, kWave);
            if (lane < L) atomicAdd(lusq + j0 + i, t);
        }
        __syncthreads();
        if (threadIdx.x < K) {
            partials[(int64_t)bc * K + threadIdx.x] = lusq[threadIdx.x];
            lusq[threadIdx.x] = 0.0;
        }
        __syncthreads();
    }
    if (cur >= 0) flush_lds();
}

// Run accumulation as run_step (keys sorted within a wave step, -1 for rows that take no
// part), with the step's values produced on demand by val(j) and each finished run's sum
// passed on as soon as it is reduced, flush1(key, j, sum): neither the step's values nor the
// reduced sums are held as arrays, which keeps the attitude pass at a few waves per SIMD.
template <int NV, int STRIDE, typename V, typename F>
__device__ __forceinline__ void run_step_lean(int32_t key, V&& val, double (&acc)[NV],
                                              int32_t& ckey, F&& flush1) {
    const uint64_t valid = __ballot(key >= 0);
    if (valid == 0) return;
    const int32_t kfirst =
        __builtin_amdgcn_readlane(key, __ffsll((unsigned long long)valid) - 1);
    const int32_t klast = __builtin_amdgcn_readlane(key, 63 - __clzll((unsigned long long)valid));
    if (kfirst == ckey && klast == ckey) {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += val(j);
        return;
    }
    if (ckey >= 0) {  // the open run ends in this step (or ended at its start)
#pragma unroll
        for (int j = 0; j < NV; ++j)
            flush1(ckey, j, group_sum<STRIDE>(acc[j] + (key == ckey ? val(j) : 0.0)));
    }
    auto next_after = [&](int32_t k) {
        const uint64_t gt = __ballot(key > k);
        return (int32_t)__builtin_amdgcn_readlane(key, __ffsll((unsigned long long)gt) - 1);
    };
    int32_t k = (kfirst == ckey) ? next_after(ckey) : kfirst;
    while (k != klast) {  // runs that start and end inside the step
#pragma unroll
        for (int j = 0; j < NV; ++j) flush1(k, j, group_sum<STRIDE>(key == k ? val(j) : 0.0));
        k = next_after(k);
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = (key == klast) ? val(j) : 0.0;
    ckey = klast;
}

template <int NV, int STRIDE, typename F>
__device__ __forceinline__ void run_close_lean(double (&acc)[NV], int32_t& ckey, F&& flush1) {
    if (ckey < 0) return;
#pragma unroll
    for (int j = 0; j < NV; ++j) flush1(ckey, j, group_sum<STRIDE>(acc[j]));
    ckey = -1;
}

// Attitude pass over the t-ordered copy (each system's rows keep their own range).  One lane
// per right-hand side (L = K lanes per row, R = 1): each lane reads the row's 12 attitude
// coefficients (16-byte loads) and its value of Y; with one right-hand side per lane the run
// accumulators stay small enough for four waves per SIMD.
template <typename VT, int MODE, int K>
static __global__ __launch_bounds__(256) void k_baprod2_att(
    const SysDesc* __restrict__ sys, const Seg* __restrict__ chunks, int nchunks,
    const VT* __restrict__ attT, const int32_t* __restrict__ rowT,
    const int32_t* __restrict__ tT, const double* __restrict__ Y, double* __restrict__ X,
    const LsqrState* __restrict__ st) {
    constexpr int L = K;
    constexpr int R = K / L;
    constexpr int RS = kWave / L;
    constexpr int NA = kAxes * kParAxis;
    static_assert(sizeof(VT) == 8, "the batched attitude tiles are binary64");
    const int lane = threadIdx.x % kWave, rr = lane / L, j0 = (lane % L) * R;
    const int wpb = blockDim.x / kWave;
    for (int ch = blockIdx.x * wpb + threadIdx.x / kWave; ch < nchunks; ch += gridDim.x * wpb) {
        const Seg c = chunks[ch];
        const SysDesc d = sys[c.sys];
        bool live[R];
        bool any_live = false;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            live[i] = (MODE == A2_LSQR) ? !st[(int64_t)c.sys * K + j0 + i].stop : true;
            any_live = any_live || live[i];
        }
        // (A2_LSQR: u~ unnormalized; k_bvec_v applies 1/beta)
        double* __restrict__ Xt = X + (d.col0 + d.att0) * K + j0;
        // value j = i * NA + ax * kParAxis + q: right-hand side i, column t + q of axis ax
        auto flush1 = [&](int32_t key, int j, double t) {
            const int i = j / NA, ax = (j % NA) / kParAxis, q = j % kParAxis;
            if (rr == 0 && live[i]) atomic_add_f64(Xt + ((int64_t)ax * d.T + key + q) * K + i, t);
        };
        double acc[NA * R];
#pragma unroll
        for (int q = 0; q < NA * R; ++q) acc[q] = 0.0;
        int32_t ckey = -1;
        for (int64_t k0 = c.e0; k0 < c.e1; k0 += RS) {
            const int64_t k = k0 + rr;
            const bool valid = any_live && k < c.e1;
            int32_t key = -1;
            double yy[R], a[NA];
#pragma unroll
            for (int i = 0; i < R; ++i) yy[i] = 0.0;
#pragma unroll
            for (int q = 0; q < NA; ++q) a[q] = 0.0;
            if (valid) {
                key = tT[k];
                if (MODE == A2_SQ) {
#pragma unroll
                    for (int i = 0; i < R; ++i) yy[i] = 0.0;
                } else {
                    ld_r<R>(Y + (int64_t)rowT[k] * K + j0, yy);
#pragma unroll
                    for (int i = 0; i < R; ++i) yy[i] = live[i] ? yy[i] : 0.0;
                }
                {  // the row's attitude tile
                    const int64_t lr = k - d.row0;
                    const int64_t tile = d.btile0 + lr / kStepRows;
                    const f64x2* ap = reinterpret_cast<const f64x2*>(attT + tile * kBTileAtt) +
                                      (int)(lr % kStepRows);
#pragma unroll
                    for (int q = 0; q < NA / 2; ++q) {
                        const f64x2 t = __builtin_nontemporal_load(ap + q * kStepRows);
                        a[2 * q] = t.x;
                        a[2 * q + 1] = t.y;
                    }
                }
            }
            auto val = [&](int j) { return contrib<MODE>(a[j % NA], yy[j / NA]); };
            run_step_lean<NA * R, L>(key, val, acc, ckey, flush1);
        }
        run_close_lean<NA * R, L>(acc, ckey, flush1);
    }
}

// ---------------------------------------------------------------------------------------
// vectors (one block per segment; elements e = index * K + j)

// Per-segment, per-j block sums of NQ quantities -> part[(q * nseg + seg) * K + j].
template <int K, int NQ>
__device__ __forceinline__ void seg_partials(double (&acc)[NQ], double* sh, double* part,
                                             int nseg, int seg) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    constexpr int W = 256 / kWave;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = K; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
        if (lane < K) sh[(q * W + w) * K + lane] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ * K) {
        const int q = threadIdx.x / K, j = threadIdx.x % K;
        double s = 0.0;
#pragma unroll
        for (int ww = 0; ww < W; ++ww) s += sh[(q * W + ww) * K + j];
        part[((int64_t)q * nseg + seg) * K + j] = s;
    }
    __syncthreads();
}

// u = b per pair (row segments); partial sum u^2
template <int K>
static __global__ __launch_bounds__(256) void k_bcopy_norm(const Seg* __restrict__ segs, int nseg,
                                                           const double* __restrict__ B,
                                                           double* __restrict__ U,
                                                           double* __restrict__ part) {
    __shared__ double sh[4 * K * 1];
    for (int sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const Seg c = segs[sg];
        double acc[1] = {0.0};
        for (int64_t e = c.e0 * K + threadIdx.x; e < c.e1 * K; e += blockDim.x) {
            const double v = B[e];
            U[e] = v;
            acc[0] = fma(v, v, acc[0]);
        }
        seg_partials<K, 1>(acc, sh, part, nseg, sg);
    }
}

// forward v-step over column tiles (see k_vec_v for the single system)
template <bool INIT, int K>
static __global__ __launch_bounds__(256) void k_bvec_v(const Seg* __restrict__ tiles, int ntile,
                                                       double* __restrict__ S,
                                                       const double* __restrict__ p,
                                                       double* __restrict__ V,
                                                       double* __restrict__ Wv,
                                                       double* __restrict__ Z,
                                                       double* __restrict__ XT,
                                                       const LsqrState* __restrict__ st,
                                                       double* __restrict__ part) {
    __shared__ double sh[4 * 4 * K];
    const int j = threadIdx.x % K;
    for (int sg = blockIdx.x; sg < ntile; sg += gridDim.x) {
        const Seg c = tiles[sg];
        const LsqrState* ps = st + (int64_t)c.sys * K + j;
        const bool live = INIT || !ps->stop;
        const bool pending = !INIT && ps->pending;
        const double f1 = ps->f1, f2 = ps->f2, sv = ps->sv;
        const double c1 = INIT ? 0.0 : ps->beta * ps->sv;
        const double su = ps->su;  // S holds A^T u~ unnormalized
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t e = c.e0 * K + threadIdx.x; e < c.e1 * K; e += blockDim.x) {
            const double sj = S[e];
            S[e] = 0.0;
            if (!live) continue;
            const double pj = p[e / K];
            double vn;
            if (INIT) {
                vn = pj * (su * sj);
                Z[e] = 0.0;
                Wv[e] = 0.0;
            } else {
                const double vj = V[e];
                if (pending) {
                    const double wj = Wv[e];
                    const double zj = fma(f1, wj, Z[e]);
                    const double wn = sv * vj - f2 * wj;
                    Z[e] = zj;
                    Wv[e] = wn;
                    acc[1] = fma(zj, zj, acc[1]);
                    acc[2] = fma(zj, wn, acc[2]);
                    acc[3] = fma(wn, wn, acc[3]);
                }
                vn = pj * (su * sj) - c1 * vj;
            }
            V[e] = vn;
            XT[e] = pj * vn;
            acc[0] = fma(vn, vn, acc[0]);
        }
        seg_partials<K, 4>(acc, sh, part, ntile, sg);
    }
}

// X = p o (z + pending updates) per pair
template <int K>
static __global__ __launch_bounds__(256) void k_bfinal(const Seg* __restrict__ tiles, int ntile,
                                                       const double* __restrict__ p,
                                                       double* __restrict__ Z,
                                                       double* __restrict__ Wv,
                                                       const double* __restrict__ V,
                                                       double* __restrict__ Xout,
                                                       const LsqrState* __restrict__ st) {
    const int j = threadIdx.x % K;
    for (int sg = blockIdx.x; sg < ntile; sg += gridDim.x) {
        const Seg c = tiles[sg];
        const LsqrState* ps = st + (int64_t)c.sys * K + j;
        const bool pending = ps->pending, pend_b = ps->pend_b;
        const double f1 = ps->f1, f2 = ps->f2, sv = ps->sv, fb = ps->fb;
        for (int64_t e = c.e0 * K + threadIdx.x; e < c.e1 * K; e += blockDim.x) {
            double zj = Z[e];
            if (pending) {
                const double wj = Wv[e];
                zj = fma(f1, wj, zj);
                const double wn = sv * V[e] - f2 * wj;
                if (pend_b) zj = fma(fb, wn, zj);
                Wv[e] = wn;
            }
            Z[e] = zj;
            Xout[e] = p[e / K] * zj;
        }
    }
}

// p = 1/sqrt(ss), ss reset (K = 1 vectors)
static __global__ void k_brecip_sqrt(int64_t n, double* __restrict__ ss, double* __restrict__ p,
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

// ---------------------------------------------------------------------------------------
// scalars: one wave per (system, rhs) pair

template <int K>
__device__ __forceinline__ double pair_sum(const double* __restrict__ part, int q, int nseg,
                                           int first, int count, int j) {
    const int lane = threadIdx.x % kWave;
    double a = 0.0;
    for (int s = first + lane; s < first + count; s += kWave)
        a += part[((int64_t)q * nseg + s) * K + j];
    return wave_sum(a);
}

enum { BS_INIT1 = 0, BS_INIT2 = 1, BS_BETA = 2, BS_ALPHA = 3 };

template <int STEP, int K>
static __global__ __launch_bounds__(256) void k_bscal(LsqrState* __restrict__ st,
                                                      const SysDesc* __restrict__ sys, int n_sys,
                                                      const double* __restrict__ part, int nseg,
                                                      int32_t itnlim, int32_t fixed, double atol,
                                                      double btol, double conlim, int32_t k_used) {
    const int pair = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (pair >= n_sys * K) return;
    const int sidx = pair / K, j = pair % K;
    const SysDesc d = sys[sidx];
    const bool by_rows = (STEP == BS_INIT1);
    const bool by_bchunks = (STEP == BS_BETA);
    const int first = by_bchunks ? d.bchunk0 : (by_rows ? d.chunk0 : d.tile0);
    const int count = by_bchunks ? d.nbchunk : (by_rows ? d.nchunk : d.ntile);
    LsqrState* ps = st + pair;
    if (STEP == BS_INIT1) {
        const double ss = pair_sum<K>(part, 0, nseg, first, count, j);
        if (threadIdx.x % kWave == 0) {
            scal_init1(ps, ss, itnlim, fixed, atol, btol, conlim);
            if (j >= k_used) {  // padding right-hand side: never iterates
                ps->stop = 1;
                ps->istop = 4;
            }
        }
        return;
    }
    if (ps->stop) return;
    if (STEP == BS_INIT2) {
        const double ss = pair_sum<K>(part, 0, nseg, first, count, j);
        if (threadIdx.x % kWave == 0) scal_init2(ps, ss);
    } else if (STEP == BS_BETA) {
        const double ss = pair_sum<K>(part, 0, nseg, first, count, j);
        if (threadIdx.x % kWave == 0) scal_beta(ps, ss);
    } else {
        const double vv = pair_sum<K>(part, 0, nseg, first, count, j);
        const double zz = pair_sum<K>(part, 1, nseg, first, count, j);
        const double zw = pair_sum<K>(part, 2, nseg, first, count, j);
        const double ww = pair_sum<K>(part, 3, nseg, first, count, j);
        if (threadIdx.x % kWave == 0) scal_alpha(ps, vv, zz, zw, ww);
    }
}

// index checks per system (bits as k_validate)
static __global__ void k_bvalidate(const SysDesc* __restrict__ sys, const Seg* __restrict__ chunks,
                                   int nchunks, const int32_t* __restrict__ star,
                                   const int32_t* __restrict__ att,
                                   const int32_t* __restrict__ instr, int* __restrict__ flags) {
    int bad = 0;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const Seg c = chunks[ch];
        const SysDesc d = sys[c.sys];
        for (int64_t r = c.e0 + threadIdx.x; r < c.e1; r += blockDim.x) {
            const int32_t s = star[r];
            if (s < 0 || s >= d.n_stars) bad |= 1;
            if (r > d.row0 && star[r - 1] > s) bad |= 2;
            const int32_t t = att[r];
            if (t < 0 || t > d.T - kParAxis) bad |= 4;
            for (int q = 0; q < kInstr; ++q) {
                const int32_t ic = instr[r * kInstr + q];
                if (ic < 0 || ic >= d.I) bad |= 8;
            }
        }
    }
    if (bad) atomicOr(flags, bad);
}

// sort keys: (system << tbits) | t
static __global__ void k_bkeys(const SysDesc* __restrict__ sys, const Seg* __restrict__ chunks,
                               int nchunks, const int32_t* __restrict__ att, int tbits,
                               uint64_t* __restrict__ keys, int32_t* __restrict__ iota) {
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const Seg c = chunks[ch];
        for (int64_t r = c.e0 + threadIdx.x; r < c.e1; r += blockDim.x) {
            keys[r] = ((uint64_t)c.sys << tbits) | (uint64_t)(uint32_t)att[r];
            iota[r] = (int32_t)r;
        }
    }
}

static __global__ void k_bkeys_to_t(int64_t m, const uint64_t* __restrict__ keys, int tbits,
                                    int32_t* __restrict__ tT) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint64_t mask = (tbits >= 64) ? ~0ull : ((1ull << tbits) - 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
        tT[i] = (int32_t)(keys[i] & mask);
}

}  // namespace gsr

using namespace gsr;

#define HIP_TRY(call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)
#define GSR_TRY(call)                \
    do {                             \
        gsr_status s_ = (call);      \
        if (s_ != GSR_OK) return s_; \
    } while (0)
#define HIP_TRY_VOID(call) (void)(call)

namespace {

struct Tuning {
    int chunk_rows = 256;  // rows per wave chunk
    int star_block = 512;  // threads of the star-ordered aprod 2 blocks
};

std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int>, Tuning> g_tune_cache;

template <typename T>
gsr_status balloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = device_alloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GSR_E_NOMEM, "hipMalloc of %zu bytes failed", count * sizeof(T));
    }
    return GSR_OK;
}

void bfree(void* p) {
    if (p) (void)hipFree(p);
}

}  // namespace

struct gsr_batch {
    int device = 0, n_cu = 256;
    int n_sys = 0, k = 1;
    int64_t M = 0, N = 0;
    int max_instr = 0;
    std::vector<SysDesc> h_sys;
    std::vector<int64_t> col_off;
    const double* vals = nullptr;
    const int32_t *star = nullptr, *att = nullptr, *instr = nullptr;
    SysDesc* d_sys = nullptr;
    // segment lists (device) and their counts
    Seg *chunks = nullptr, *bchunks = nullptr, *tiles = nullptr;
    int nchunks = 0, nbchunks = 0, ntiles = 0;
    Tuning tune;
    // row tiles (coefficients, indices) of the fused pass
    double* bvt = nullptr;
    int32_t* bit = nullptr;
    int64_t nbtiles = 0;
    // t-ordered attitude copy
    int32_t *rowT = nullptr, *tT = nullptr;
    double* attT = nullptr;
    // preconditioner and LSQR state
    double* p = nullptr;
    LsqrState* st = nullptr;
    std::vector<LsqrState> st_host;
    double *U = nullptr, *V = nullptr, *W = nullptr, *Z = nullptr, *XT = nullptr, *S = nullptr;
    double* part = nullptr;
    size_t part_len = 0;
    int G1 = 1, G2s = 1, G2t = 1;
    hipStream_t cap = nullptr;
    hipGraphExec_t graph = nullptr;  // whole fixed-iteration solve
    int graph_itnlim = -1;
    const double *graph_B = nullptr;
    double* graph_X = nullptr;
    gsr_solve_opts graph_opts = {};
};

namespace {

// (Re)build the row-chunk and block-chunk lists for the tuning `t`; device copies replaced.
gsr_status build_lists(gsr_batch* b, const Tuning& t, hipStream_t s) {
    std::vector<Seg> ch, bch, tl;
    const int wpb = t.star_block / kWave;
    for (int i = 0; i < b->n_sys; ++i) {
        SysDesc& d = b->h_sys[i];
        d.chunk0 = (int)ch.size();
        for (int64_t r = 0; r < d.m; r += t.chunk_rows)
            ch.push_back({d.row0 + r, d.row0 + std::min<int64_t>(d.m, r + t.chunk_rows), i, 0});
        d.nchunk = (int)ch.size() - d.chunk0;
        const int64_t bl = (int64_t)t.chunk_rows * wpb;
        d.bchunk0 = (int)bch.size();
        for (int64_t r = 0; r < d.m; r += bl)
            bch.push_back({d.row0 + r, d.row0 + std::min<int64_t>(d.m, r + bl), i, 0});
        d.nbchunk = (int)bch.size() - d.bchunk0;
        d.tile0 = (int)tl.size();
        for (int64_t c = 0; c < d.n; c += kBTile)
            tl.push_back({d.col0 + c, d.col0 + std::min<int64_t>(d.n, c + kBTile), i, 0});
        d.ntile = (int)tl.size() - d.tile0;
    }
    bfree(b->chunks);
    bfree(b->bchunks);
    bfree(b->tiles);
    b->chunks = b->bchunks = b->tiles = nullptr;
    b->nchunks = (int)ch.size();
    b->nbchunks = (int)bch.size();
    b->ntiles = (int)tl.size();
    GSR_TRY(balloc(&b->chunks, ch.size()));
    GSR_TRY(balloc(&b->bchunks, bch.size()));
    GSR_TRY(balloc(&b->tiles, tl.size()));
    if (!b->d_sys) GSR_TRY(balloc(&b->d_sys, b->n_sys));
    HIP_TRY(hipMemcpyAsync(b->chunks, ch.data(), ch.size() * sizeof(Seg), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->bchunks, bch.data(), bch.size() * sizeof(Seg), hipMemcpyHostToDevice,
                           s));
    HIP_TRY(hipMemcpyAsync(b->tiles, tl.data(), tl.size() * sizeof(Seg), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->d_sys, b->h_sys.data(), b->n_sys * sizeof(SysDesc),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    // persistent grids
    auto cap_grid = [&](int64_t items) {
        return (int)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)b->n_cu * 8));
    };
    b->G1 = cap_grid((b->nchunks + 3) / 4);
    b->G2t = cap_grid((b->nchunks + 3) / 4);
    b->G2s = (int)std::max<int64_t>(1, std::min<int64_t>(b->nbchunks, (int64_t)b->n_cu * 2));
    b->tune = t;
    return GSR_OK;
}

template <typename F>
void with_k(int k, F&& f) {
    switch (k) {
        case 1: f(std::integral_constant<int, 1>()); break;
        case 2: f(std::integral_constant<int, 2>()); break;
        case 4: f(std::integral_constant<int, 4>()); break;
        default: f(std::integral_constant<int, 8>()); break;
    }
}

template <int MODE, int K>
void blaunch_aprod1(gsr_batch* b, const double* X, double* Y, const double* B, hipStream_t s) {
    hipLaunchKernelGGL((k_baprod1<double, MODE, K>), dim3(b->G1), dim3(256), 0, s, b->d_sys,
                       b->chunks, b->nchunks, b->vals, b->star, b->att, b->instr, X, Y, B, b->st,
                       b->part);
}

template <int MODE, int K>
void blaunch_aprod2(gsr_batch* b, const double* Y, double* X, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)(b->max_instr + 1) * K;
    hipLaunchKernelGGL((k_baprod2_star<double, MODE, K>), dim3(b->G2s), dim3(b->tune.star_block),
                       lds, s, b->d_sys, b->bchunks, b->nbchunks, b->vals, b->star, b->instr, Y,
                       X, b->st, b->max_instr);
    hipLaunchKernelGGL((k_baprod2_att<double, MODE, K>), dim3(b->G2t), dim3(256), 0, s, b->d_sys,
                       b->chunks, b->nchunks, b->attT, b->rowT, b->tT, Y, X, b->st);
}

template <int K>
void bscal(gsr_batch* b, int step, int nseg, const gsr_solve_opts& o, hipStream_t s) {
    const int pairs = b->n_sys * K;
    const dim3 grid((pairs + 3) / 4), block(256);
    switch (step) {
        case BS_INIT1:
            hipLaunchKernelGGL((k_bscal<BS_INIT1, K>), grid, block, 0, s, b->st, b->d_sys,
                               b->n_sys, b->part, nseg, o.itnlim, o.fixed_iters, o.atol, o.btol,
                               o.conlim, b->k);
            break;
        case BS_INIT2:
            hipLaunchKernelGGL((k_bscal<BS_INIT2, K>), grid, block, 0, s, b->st, b->d_sys,
                               b->n_sys, b->part, nseg, 0, 0, 0.0, 0.0, 0.0, b->k);
            break;
        case BS_BETA:
            hipLaunchKernelGGL((k_bscal<BS_BETA, K>), grid, block, 0, s, b->st, b->d_sys,
                               b->n_sys, b->part, nseg, 0, 0, 0.0, 0.0, 0.0, b->k);
            break;
        default:
            hipLaunchKernelGGL((k_bscal<BS_ALPHA, K>), grid, block, 0, s, b->st, b->d_sys,
                               b->n_sys, b->part, nseg, 0, 0, 0.0, 0.0, 0.0, b->k);
    }
}

template <int K>
void b_iteration(gsr_batch* b, hipStream_t s) {
    const dim3 tgrid((unsigned)std::min(b->ntiles, b->n_cu * 8));
    // one read of every row: U = sv A XT - alpha su U and S = A^T U (star-ordered part)
    const size_t lds = sizeof(double) * ((size_t)(2 * b->max_instr + 1) * K + K);
    hipLaunchKernelGGL((k_baprod12<double, K>), dim3(b->G2s), dim3(b->tune.star_block), lds, s,
                       b->d_sys, b->bchunks, b->nbchunks, b->bvt, b->bit, b->star, b->XT, b->U,
                       b->S, b->st, b->part, b->max_instr);
    hipLaunchKernelGGL((k_baprod2_att<double, A2_LSQR, K>), dim3(b->G2t), dim3(256), 0, s,
                       b->d_sys, b->chunks, b->nchunks, b->attT, b->rowT, b->tT, b->U, b->S,
                       b->st);
    bscal<K>(b, BS_BETA, b->nbchunks, gsr_solve_opts{}, s);
    hipLaunchKernelGGL((k_bvec_v<false, K>), tgrid, dim3(256), 0, s, b->tiles, b->ntiles, b->S,
                       b->p, b->V, b->W, b->Z, b->XT, b->st, b->part);
    bscal<K>(b, BS_ALPHA, b->ntiles, gsr_solve_opts{}, s);
}

template <int K>
void b_solve_body(gsr_batch* b, const double* B, double* X, const gsr_solve_opts& o,
                  hipStream_t s, int iters) {
    const dim3 tgrid((unsigned)std::min(b->ntiles, b->n_cu * 8));
    const dim3 cgrid((unsigned)std::min(b->nchunks, b->n_cu * 8));
    hipLaunchKernelGGL((k_bcopy_norm<K>), cgrid, dim3(256), 0, s, b->chunks, b->nchunks, B, b->U,
                       b->part);
    bscal<K>(b, BS_INIT1, b->nchunks, o, s);
    hipLaunchKernelGGL(k_fill, dim3(grid_for(b->N * K, 256, 2048)), dim3(256), 0, s, b->S,
                       b->N * K, 0.0);
    blaunch_aprod2<A2_LSQR, K>(b, b->U, b->S, s);
    hipLaunchKernelGGL((k_bvec_v<true, K>), tgrid, dim3(256), 0, s, b->tiles, b->ntiles, b->S,
                       b->p, b->V, b->W, b->Z, b->XT, b->st, b->part);
    bscal<K>(b, BS_INIT2, b->ntiles, o, s);
    for (int it = 0; it < iters; ++it) b_iteration<K>(b, s);
    if (X)
        hipLaunchKernelGGL((k_bfinal<K>), tgrid, dim3(256), 0, s, b->tiles, b->ntiles, b->p, b->Z,
                           b->W, b->V, X, b->st);
}

// Time the two products for each candidate tuning; keep the fastest.  Synchronizes.
gsr_status autotune(gsr_batch* b, hipStream_t s) {
    const auto key = std::make_tuple(b->n_sys, b->M, b->k);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return build_lists(b, it->second, s);
    }
    const Tuning cands[] = {{128, 512}, {256, 512}, {512, 512}, {256, 256}, {1024, 512}};
    Tuning best = cands[1];
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (const Tuning& t : cands) {
        GSR_TRY(build_lists(b, t, s));
        float ms = 0.f;
        with_k(b->k, [&](auto kc) {
            constexpr int K = decltype(kc)::value;
            // the two product passes of one iteration, on scratch contents (every pair's
            // state is still zero here, so the values are zeros)
            HIP_TRY_VOID(hipMemsetAsync(b->XT, 0, sizeof(double) * b->N * K, s));
            HIP_TRY_VOID(hipMemsetAsync(b->U, 0, sizeof(double) * b->M * K, s));
            const size_t lds = sizeof(double) * ((size_t)(2 * b->max_instr + 1) * K + K);
            for (int rep = 0; rep < 3; ++rep) {
                if (rep == 1) (void)hipEventRecord(e0, s);
                hipLaunchKernelGGL((k_baprod12<double, K>), dim3(b->G2s), dim3(t.star_block), lds,
                                   s, b->d_sys, b->bchunks, b->nbchunks, b->bvt, b->bit,
                                   b->star, b->XT, b->U, b->S, b->st, b->part, b->max_instr);
                hipLaunchKernelGGL((k_baprod2_att<double, A2_LSQR, K>), dim3(b->G2t), dim3(256),
                                   0, s, b->d_sys, b->chunks, b->nchunks, b->attT, b->rowT,
                                   b->tT, b->U, b->S, b->st);
            }
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
        });
        HIP_TRY(hipGetLastError());
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    return build_lists(b, best, s);
}

gsr_status b_colnorm(gsr_batch* b, hipStream_t s, unsigned long long* n_empty) {
    // column sums of squares with K = 1 lists (stride-1 vectors)
    const int k_saved = b->k;
    double* ss = b->S;  // N x k >= N doubles
    unsigned long long* d_cnt = nullptr;
    GSR_TRY(balloc(&d_cnt, 1));
    HIP_TRY(hipMemsetAsync(d_cnt, 0, sizeof(*d_cnt), s));
    HIP_TRY(hipMemsetAsync(ss, 0, sizeof(double) * b->N, s));
    b->k = 1;
    blaunch_aprod2<A2_SQ, 1>(b, nullptr, ss, s);
    b->k = k_saved;
    hipLaunchKernelGGL(k_brecip_sqrt, dim3(grid_for(b->N, 256, 2048)), dim3(256), 0, s, b->N, ss,
                       b->p, d_cnt);
    HIP_TRY(hipMemsetAsync(ss, 0, sizeof(double) * b->N * b->k, s));
    hipError_t e = hipMemcpyAsync(n_empty, d_cnt, sizeof(*d_cnt), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    bfree(d_cnt);
    if (e != hipSuccess) return hip_fail(e, "batched column norms");
    return GSR_OK;
}

}  // namespace

extern "C" {

gsr_status gsr_batch_setup(int32_t n_sys, const gsr_dims* dims, const int64_t* row_offset,
                           const double* vals, const int32_t* star, const int32_t* att,
                           const int32_t* instr, int32_t k, const gsr_setup_opts* opts,
                           void* stream, gsr_batch** out) {
    g_last_error.clear();
    if (!out) return fail(GSR_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n_sys < 1 || !dims || !row_offset) return fail(GSR_E_INVAL, "n_sys < 1 or null dims");
    if (k != 1 && k != 2 && k != 4 && k != 8)
        return fail(GSR_E_UNSUPPORTED, "k must be 1, 2, 4 or 8 (got %d)", k);
    if (row_offset[0] != 0) return fail(GSR_E_INVAL, "row_offset[0] must be 0");
    int max_instr = 0;
    for (int i = 0; i < n_sys; ++i) {
        GSR_TRY(check_dims(&dims[i]));
        if (row_offset[i + 1] - row_offset[i] != dims[i].n_rows)
            return fail(GSR_E_INVAL, "row_offset does not match dims[%d].n_rows", i);
        max_instr = std::max(max_instr, dims[i].n_instr);
    }
    const int64_t M = row_offset[n_sys];
    if (M > (int64_t)INT32_MAX) return fail(GSR_E_UNSUPPORTED, "more than 2^31-1 rows");
    if (M > 0 && (!vals || !star || !att || !instr)) return fail(GSR_E_INVAL, "null matrix array");
    if (((uintptr_t)vals & 15) || ((uintptr_t)instr & 7))
        return fail(GSR_E_INVAL, "vals must be 16-byte and instr 8-byte aligned");
    if ((size_t)((2 * max_instr + 1) * k + k) * sizeof(double) > 160 * 1024)
        return fail(GSR_E_UNSUPPORTED, "n_instr * k too large for the batched LDS accumulator");
    gsr_setup_opts so = {0, 1, 0, 0};
    if (opts) so = *opts;
    int dev = 0, n_cu = 0;
    GSR_TRY(check_device(&dev, &n_cu));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    gsr_batch* b = new gsr_batch();
    auto bail = [&](gsr_status st) {
        gsr_batch_destroy(b);
        return st;
    };
    b->device = dev;
    b->n_cu = n_cu;
    b->n_sys = n_sys;
    b->k = k;
    b->M = M;
    b->max_instr = max_instr;
    b->vals = vals;
    b->star = star;
    b->att = att;
    b->instr = instr;
    b->h_sys.resize(n_sys);
    b->col_off.resize(n_sys + 1);
    int64_t col = 0, max_T = 4;
    for (int i = 0; i < n_sys; ++i) {
        const Geo g = make_geo(&dims[i]);
        SysDesc& d = b->h_sys[i];
        d.row0 = row_offset[i];
        d.m = dims[i].n_rows;
        d.col0 = col;
        d.n = g.n;
        d.att0 = g.att0;
        d.ins0 = g.ins0;
        d.glb0 = g.glb0;
        d.n_stars = dims[i].n_stars;
        d.T = g.T;
        d.I = g.I;
        d.btile0 = b->nbtiles;
        b->nbtiles += (d.m + kStepRows - 1) / kStepRows;
        b->col_off[i] = col;
        col += g.n;
        max_T = std::max<int64_t>(max_T, g.T);
    }
    b->col_off[n_sys] = col;
    b->N = col;
    gsr_status st;
    if ((st = build_lists(b, Tuning(), s)) != GSR_OK) return bail(st);
    const size_t NK = (size_t)b->N * k, MK = (size_t)M * k;
    if ((st = balloc(&b->p, b->N)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->S, NK)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->V, NK)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->W, NK)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->Z, NK)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->XT, NK)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->U, MK)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->st, (size_t)n_sys * k)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->bvt, (size_t)b->nbtiles * kBTileVals)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->bit, (size_t)b->nbtiles * kBTileIdx)) != GSR_OK) return bail(st);
    for (int i = 0; i < n_sys; ++i) {
        const SysDesc& d = b->h_sys[i];
        const int64_t nt = (d.m + kStepRows - 1) / kStepRows;
        if (nt == 0) continue;
        hipLaunchKernelGGL(k_make_btiles, dim3(grid_for(nt * kBTileVals, 256, 4096)), dim3(256), 0,
                           s, d.m, nt, vals + d.row0 * kPar, star + d.row0, att + d.row0,
                           instr + d.row0 * kInstr, b->bvt + d.btile0 * kBTileVals,
                           b->bit + d.btile0 * kBTileIdx);
    }
    b->st_host.resize((size_t)n_sys * k);
    {
        hipError_t e = hipMemsetAsync(b->st, 0, sizeof(LsqrState) * n_sys * k, s);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(e, "batch setup"));
    }
    // validation
    if (so.validate && M > 0) {
        int* d_flags = nullptr;
        if ((st = balloc(&d_flags, 1)) != GSR_OK) return bail(st);
        int flags = 0;
        hipError_t e = hipMemsetAsync(d_flags, 0, sizeof(int), s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_bvalidate, dim3(std::min(b->nchunks, 4096)), dim3(256), 0, s,
                               b->d_sys, b->chunks, b->nchunks, star, att, instr, d_flags);
            e = hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        bfree(d_flags);
        if (e != hipSuccess) return bail(hip_fail(e, "batch validation"));
        if (flags)
            return bail(fail(GSR_E_LAYOUT, "index check failed:%s%s%s%s",
                             (flags & 1) ? " star out of range" : "",
                             (flags & 2) ? " stars not sorted" : "",
                             (flags & 4) ? " attitude start out of [0, n_dfa-4]" : "",
                             (flags & 8) ? " instrumental index out of range" : ""));
    }
    // attitude coefficients in (system, t) order
    if ((st = balloc(&b->rowT, M)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->tT, M)) != GSR_OK) return bail(st);
    if ((st = balloc(&b->attT, (size_t)b->nbtiles * kBTileAtt)) != GSR_OK) return bail(st);
    if (M > 0) {
        int tbits = 1;
        while (tbits < 31 && (1LL << tbits) <= max_T) ++tbits;
        int sbits = 1;
        while ((1LL << sbits) < n_sys) ++sbits;
        uint64_t *keys = nullptr, *keys_out = nullptr;
        int32_t* iota = nullptr;
        void* temp = nullptr;
        size_t temp_bytes = 0;
        hipError_t e = hipMalloc(&keys, sizeof(uint64_t) * M);
        if (e == hipSuccess) e = hipMalloc(&keys_out, sizeof(uint64_t) * M);
        if (e == hipSuccess) e = hipMalloc(&iota, sizeof(int32_t) * M);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_bkeys, dim3(std::min(b->nchunks, 4096)), dim3(256), 0, s,
                               b->d_sys, b->chunks, b->nchunks, att, tbits, keys, iota);
            e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys, keys_out, iota,
                                                   b->rowT, (int)M, 0, tbits + sbits, s);
        }
        if (e == hipSuccess) e = hipMalloc(&temp, std::max<size_t>(temp_bytes, 1));
        if (e == hipSuccess)
            e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_out, iota, b->rowT,
                                                   (int)M, 0, tbits + sbits, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_bkeys_to_t, dim3(grid_for(M, 256, 4096)), dim3(256), 0, s, M,
                               keys_out, tbits, b->tT);
            for (int i = 0; i < n_sys; ++i) {
                const SysDesc& d = b->h_sys[i];
                const int64_t nt = (d.m + kStepRows - 1) / kStepRows;
                if (nt == 0) continue;
                hipLaunchKernelGGL(k_make_batt_tiles, dim3(grid_for(nt * kBTileAtt, 256, 4096)),
                                   dim3(256), 0, s, d.m, nt, d.row0, vals, b->rowT,
                                   b->attT + d.btile0 * kBTileAtt);
            }
            e = hipStreamSynchronize(s);
        }
        bfree(keys);
        bfree(keys_out);
        bfree(iota);
        bfree(temp);
        if (e != hipSuccess) return bail(hip_fail(e, "batched attitude ordering"));
    }
    // partial-sum buffer: 4 quantities per (segment, rhs)
    b->part_len = (size_t)4 * std::max(std::max(b->nchunks, b->ntiles), 1) * k * 4;
    if ((st = balloc(&b->part, b->part_len)) != GSR_OK) return bail(st);
    unsigned long long n_empty = 0;
    if ((st = b_colnorm(b, s, &n_empty)) != GSR_OK) return bail(st);
    if (n_empty && !so.allow_empty_cols)
        return bail(fail(GSR_E_LAYOUT, "%llu all-zero column(s); set allow_empty_cols", n_empty));
    if ((st = autotune(b, s)) != GSR_OK) return bail(st);
    // the tuned lists may have more segments than the default ones
    const size_t need = (size_t)4 * std::max(std::max(b->nchunks, b->ntiles), 1) * k;
    if (need > b->part_len) {
        bfree(b->part);
        b->part_len = need;
        if ((st = balloc(&b->part, b->part_len)) != GSR_OK) return bail(st);
    }
    *out = b;
    return GSR_OK;
}

gsr_status gsr_batch_destroy(gsr_batch* b) {
    if (!b) return GSR_OK;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (void* p : {(void*)b->d_sys, (void*)b->chunks, (void*)b->bchunks, (void*)b->tiles,
                    (void*)b->rowT, (void*)b->tT, (void*)b->attT, (void*)b->p, (void*)b->st,
                    (void*)b->U, (void*)b->V, (void*)b->W, (void*)b->Z, (void*)b->XT,
                    (void*)b->S, (void*)b->part, (void*)b->bvt, (void*)b->bit})
        bfree(p);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return GSR_OK;
}

gsr_status gsr_batch_col_offsets(const gsr_batch* b, int64_t* col_offset) {
    if (!b || !col_offset) return fail(GSR_E_INVAL, "null argument");
    std::memcpy(col_offset, b->col_off.data(), sizeof(int64_t) * (b->n_sys + 1));
    return GSR_OK;
}

gsr_status gsr_batch_aprod1(gsr_batch* b, const double* X, double* Y, void* stream) {
    if (!b || !X || !Y) return fail(GSR_E_INVAL, "null argument");
    if (((uintptr_t)X | (uintptr_t)Y) & 15) return fail(GSR_E_INVAL, "X and Y must be 16-byte aligned");
    HIP_TRY(hipSetDevice(b->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    with_k(b->k, [&](auto kc) { blaunch_aprod1<A1_ADD, decltype(kc)::value>(b, X, Y, nullptr, s); });
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_batch_aprod2(gsr_batch* b, const double* Y, double* X, void* stream) {
    if (!b || !X || !Y) return fail(GSR_E_INVAL, "null argument");
    if (((uintptr_t)X | (uintptr_t)Y) & 15) return fail(GSR_E_INVAL, "X and Y must be 16-byte aligned");
    HIP_TRY(hipSetDevice(b->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    with_k(b->k, [&](auto kc) { blaunch_aprod2<A2_ADD, decltype(kc)::value>(b, Y, X, s); });
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_batch_solve(gsr_batch* b, const double* B, double* X, const gsr_solve_opts* opts,
                           gsr_solve_info* info, void* stream) {
    g_last_error.clear();
    if (!b || !X || (!B && b->M > 0)) return fail(GSR_E_INVAL, "null argument");
    gsr_solve_opts o;
    std::memset(&o, 0, sizeof o);
    o.itnlim = 100;
    o.fixed_iters = 1;
    o.atol = o.btol = 1e-14;
    if (opts) o = *opts;
    if (o.itnlim < 0) return fail(GSR_E_INVAL, "itnlim < 0");
    if (!(o.atol >= 0) || !(o.btol >= 0) || !(o.conlim >= 0))
        return fail(GSR_E_INVAL, "atol, btol and conlim must be >= 0");
    if (o.precision != GSR_F64) return fail(GSR_E_UNSUPPORTED, "batched solve is binary64 only");
    HIP_TRY(hipSetDevice(b->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    gsr_status rc = GSR_OK;
    with_k(b->k, [&](auto kc) {
        constexpr int K = decltype(kc)::value;
        if (o.fixed_iters && !o.profile) {
            // the whole solve as one graph, reused while B, X and the options are unchanged
            const bool same = b->graph && b->graph_itnlim == o.itnlim && b->graph_B == B &&
                              b->graph_X == X &&
                              std::memcmp(&b->graph_opts, &o, sizeof o) == 0;
            if (!same) {
                if (b->graph) (void)hipGraphExecDestroy(b->graph);
                b->graph = nullptr;
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    b_solve_body<K>(b, B, X, o, b->cap, o.itnlim);
                    e = hipStreamEndCapture(b->cap, &g);
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
                if (g) (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    b->graph = nullptr;
                    rc = hip_fail(e, "batched solve graph");
                    return;
                }
                b->graph_itnlim = o.itnlim;
                b->graph_B = B;
                b->graph_X = X;
                b->graph_opts = o;
            }
            hipError_t e = hipGraphLaunch(b->graph, s);
            if (e != hipSuccess) rc = hip_fail(e, "hipGraphLaunch");
            return;
        }
        // convergence mode: iterate in launches of 16, checking every pair's stop flag
        b_solve_body<K>(b, B, nullptr, o, s, 0);
        const int every = o.check_every > 0 ? o.check_every : 16;
        for (int done = 0; done < o.itnlim; done += every) {
            for (int it = 0; it < every && done + it < o.itnlim; ++it) b_iteration<K>(b, s);
            hipError_t e = hipMemcpyAsync(b->st_host.data(), b->st,
                                          sizeof(LsqrState) * b->st_host.size(),
                                          hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                rc = hip_fail(e, "batched stop flags");
                return;
            }
            bool all = true;
            for (const LsqrState& t : b->st_host) all = all && t.stop;
            if (all) break;
        }
        const dim3 tgrid((unsigned)std::min(b->ntiles, b->n_cu * 8));
        hipLaunchKernelGGL((k_bfinal<K>), tgrid, dim3(256), 0, s, b->tiles, b->ntiles, b->p, b->Z,
                           b->W, b->V, X, b->st);
    });
    if (rc != GSR_OK) return rc;
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(b->st_host.data(), b->st, sizeof(LsqrState) * b->st_host.size(),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool nonfinite = false;
    for (size_t i = 0; i < b->st_host.size(); ++i) {
        const LsqrState& t = b->st_host[i];
        nonfinite = nonfinite || t.nonfinite;
        if (info) {
            gsr_solve_info& f = info[i];
            std::memset(&f, 0, sizeof f);
            f.itn = t.itn;
            f.istop = t.istop;
            f.n_refine = 1;
            f.nonfinite = t.nonfinite;  // which pair broke down, beside the status returned
            f.fused = 1;                // the batched row pass is always the fused one
            f.rnorm = t.rnorm;
            f.arnorm = t.arnorm;
            f.anorm = std::sqrt(t.anorm2);
            f.znorm = std::sqrt(t.znorm2);
            f.bnorm = t.bnorm;
            f.acond = std::sqrt(t.anorm2) * std::sqrt(t.ddnorm);
        }
    }
    if (nonfinite) return fail(GSR_E_BREAKDOWN, "non-finite value in a batched recurrence");
    return GSR_OK;
}

}  // extern "C"
