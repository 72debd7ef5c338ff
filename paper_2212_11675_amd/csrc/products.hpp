// The two products of the hot path (Section 3, Algorithms 1 and 2), written for gfx950.
//
// Lane layout ("quad"): four lanes per row, sixteen rows per wave step.  Lane q of a row
// holds the coefficients in slots 4k + q (k = 0..5), so every attitude access of a quad
// covers the four consecutive columns t..t+3 of one axis.  Read from the caller's row layout
// a wave load touches sixteen 32-byte pieces; the library's row tiles (below) turn every
// load of a wave step into one contiguous block:
//
//   q = 0 : slots 0 4 8 12 16 20   astro 0, astro 4, att j=3 (axes 0,1,2), instr 3
//   q = 1 : slots 1 5 9 13 17 21   astro 1, att j=0 (axes 0,1,2), instr 0, instr 4
//   q = 2 : slots 2 6 10 14 18 22  astro 2, att j=1 (axes 0,1,2), instr 1, instr 5
//   q = 3 : slots 3 7 11 15 19 23  astro 3, att j=2 (axes 0,1,2), instr 2, global
//
// Waves walk contiguous chunks of rows, so runs of equal keys (the star of a row in the
// star-ordered pass, the attitude start t in the attitude pass) are accumulated in registers
// (run_step) and reduced over the row groups and written once when they end.
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

// ---------------------------------------------------------------------------------------
// Row tiles: a library-owned copy of the coefficients and indices in which every load
// instruction of a wave step reads one contiguous block (the paper's row layout makes each
// lane's coefficients 4 slots apart, so a wave load would touch sixteen separate 32-byte
// pieces).  A tile holds the kStepRows rows of one wave step; lane (rg, q) needs slots
// 4k + q (k = 0..5) of row rg:
//   binary64 : three 1 KiB groups; group h is [rg][q][2] = slots 4(2h) + q, 4(2h+1) + q
//   binary32 : a 1 KiB group [rg][q][4] (k = 0..3), then a 512 B group [rg][q][2] (k = 4, 5)
//   indices  : [rg][q][2] int32 = (star, att), (instr0, instr4), (instr1, instr5),
//              (instr2, instr3) for q = 0..3
// The index tile follows the coefficients of the same tile (one stream per wave).  Padding
// rows of the last tile carry zero coefficients and the last row's indices.
constexpr int kTileVals = kStepRows * kPar;  // 384 coefficients per tile
constexpr int kTileIdx = kStepRows * 8;      // 128 int32 per tile
template <typename VT>
constexpr int64_t tile_elems() {  // coefficients, then the index tile, in units of VT
    return kTileVals + kTileIdx * 4 / (int64_t)sizeof(VT);
}

__device__ __forceinline__ void ld_tile(const double* __restrict__ tiles, int64_t tile, int lane,
                                        double (&a)[6]) {
    const f64x2* __restrict__ p =
        reinterpret_cast<const f64x2*>(tiles + tile * tile_elems<double>()) + lane;
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        const f64x2 v = __builtin_nontemporal_load(p + h * kWave);
        a[2 * h] = v.x;
        a[2 * h + 1] = v.y;
    }
}
__device__ __forceinline__ void ld_tile(const float* __restrict__ tiles, int64_t tile, int lane,
                                        double (&a)[6]) {
    const float* __restrict__ t = tiles + tile * tile_elems<float>();
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(t) + lane);
    const f32x2 w = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(t + 4 * kWave) + lane);
    a[0] = v.x;
    a[1] = v.y;
    a[2] = v.z;
    a[3] = v.w;
    a[4] = w.x;
    a[5] = w.y;
}

// Index tile of a wave step: star, attitude start and the lane's instrumental indices
// (ia: the instrumental slot among k = 0..5 of lane q; ib: the second one of lanes 1 and 2).
template <typename VT>
__device__ __forceinline__ void ld_tile_idx(const VT* __restrict__ tiles, int64_t tile, int lane,
                                            int32_t& sr, int32_t& tr, int32_t& ia, int32_t& ib) {
    const int32_t* itile =
        reinterpret_cast<const int32_t*>(tiles + tile * tile_elems<VT>() + kTileVals);
    const i32x2 v = __builtin_nontemporal_load(reinterpret_cast<const i32x2*>(itile) + lane);
    sr = __builtin_amdgcn_update_dpp(0, v.x, 0x00, 0xF, 0xF, false);   // quad_perm [0,0,0,0]
    tr = __builtin_amdgcn_update_dpp(0, v.y, 0x00, 0xF, 0xF, false);
    const int32_t i3 = __builtin_amdgcn_update_dpp(0, v.y, 0xFF, 0xF, 0xF, false);  // [3,3,3,3]
    ia = ((lane & 3) == 0) ? i3 : v.x;
    ib = v.y;
}

// Setup: row tiles from the paper's row layout (one thread per tile element).
template <typename VT>
static __global__ void k_make_tiles(int64_t m, int64_t ntiles, const double* __restrict__ vals,
                                    VT* __restrict__ tiles) {
    const int64_t total = ntiles * kTileVals;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t tile = e / kTileVals;
        const int o = (int)(e - tile * kTileVals);
        VT* __restrict__ dst = tiles + tile * tile_elems<VT>() + o;
        int lane, k;
        if (sizeof(VT) == 8) {
            lane = (o % (2 * kWave)) / 2;
            k = 2 * (o / (2 * kWave)) + o % 2;
        } else if (o < 4 * kWave) {
            lane = o / 4;
            k = o % 4;
        } else {
            lane = (o - 4 * kWave) / 2;
            k = 4 + (o - 4 * kWave) % 2;
        }
        const int64_t row = tile * kStepRows + lane / kQuad;
        const int slot = 4 * k + lane % kQuad;
        *dst = row < m ? (VT)vals[row * kPar + slot] : (VT)0;  // binary32: round to nearest
    }
}

template <typename VT>
static __global__ void k_make_itiles(int64_t m, int64_t ntiles, const int32_t* __restrict__ star,
                                     const int32_t* __restrict__ att,
                                     const int32_t* __restrict__ instr, VT* __restrict__ tiles) {
    const int64_t total = ntiles * kTileIdx;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t tile = e / kTileIdx;
        const int o = (int)(e - tile * kTileIdx);
        const int lane = o / 2, h = o % 2, q = lane % kQuad;
        const int64_t row = min(tile * kStepRows + lane / kQuad, m - 1);
        int32_t v;
        if (q == 0) {
            v = h ? att[row] : star[row];
        } else {
            const int k = (q == 1) ? (h ? 4 : 0) : (q == 2) ? (h ? 5 : 1) : (h ? 3 : 2);
            v = instr[row * kInstr + k];
        }
        reinterpret_cast<int32_t*>(tiles + tile * tile_elems<VT>() + kTileVals)[o] = v;
    }
}

// Attitude tiles (the attitude copy): kStepRows rows of 12 attitude coefficients; lane
// (rg, q) needs column t + q of the three axes of row rg: a group [rg][q][2] (axes 0, 1)
// followed by a group [rg][q] (axis 2).  Padding rows are zero.
constexpr int kTileAtt = kStepRows * kAxes * kParAxis;  // 192 coefficients per tile

__device__ __forceinline__ void ld_att_tile(const double* __restrict__ t, int64_t tile, int lane,
                                            double (&va)[kAxes]) {
    const double* __restrict__ b = t + tile * kTileAtt;
    const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(b) + lane);
    va[0] = v.x;
    va[1] = v.y;
    va[2] = __builtin_nontemporal_load(b + 2 * kWave + lane);
}
__device__ __forceinline__ void ld_att_tile(const float* __restrict__ t, int64_t tile, int lane,
                                            double (&va)[kAxes]) {
    const float* __restrict__ b = t + tile * kTileAtt;
    const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(b) + lane);
    va[0] = v.x;
    va[1] = v.y;
    va[2] = __builtin_nontemporal_load(b + 2 * kWave + lane);
}

// Cross-lane moves of a double with a DPP control (both 32-bit halves).
// quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E; row_ror:4 = 0x124, row_ror:8 = 0x128.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi2, lo2);
}

// Sum over the four lanes of a quad, result in all four.
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    return v;
}

// v[l] + v[l ^ 16] (PAIR = 16) or v[l] + v[l ^ 32] (PAIR = 32) in every lane, with the gfx950
// row swaps (no LDS crossbar): swapping a register with itself yields, in every lane, the
// value of the lower and of the upper partner, added in that order (the same in both lanes).
template <int PAIR>
__device__ __forceinline__ double pair_sum(double v) {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    unsigned l0, l1, h0, h1;
    if (PAIR == 16) {
        const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
    } else {
        const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
    }
    return __hiloint2double((int)h0, (int)l0) + __hiloint2double((int)h1, (int)l1);
}

// Sum over the lanes with the same lane % STRIDE (STRIDE = 1, 2, 4 or 8), result in all of
// them: DPP within each 16-lane row, then the two row swaps across rows.
template <int STRIDE>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(STRIDE == 1 || STRIDE == 2 || STRIDE == 4 || STRIDE == 8, "stride");
    if (STRIDE <= 1) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    if (STRIDE <= 2) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if (STRIDE <= 4) v += dpp_f64<0x124>(v);  // row_ror:4
    v += dpp_f64<0x128>(v);                   // row_ror:8
    v = pair_sum<16>(v);
    return pair_sum<32>(v);
}

// Runs of equal keys over the row groups of a wave (lane = STRIDE * group + q; keys sorted
// within the step, -1 for rows that take no part).  acc[] holds each lane's share of the
// open run `ckey`.  A step whose rows all continue the open run only adds; when runs end,
// their sums are reduced over the row groups and passed to flush(key, sums) -- called by
// every lane, with the totals valid in all of them -- and the step's last run stays open.
template <int NV, int STRIDE, typename F>
__device__ __forceinline__ void run_step(int32_t key, const double (&v)[NV], double (&acc)[NV],
                                         int32_t& ckey, F&& flush) {
    const uint64_t valid = __ballot(key >= 0);
    if (valid == 0) return;
    // lane indices below are wave-uniform: read the key with v_readlane (no LDS round trip)
    const int32_t kfirst =
        __builtin_amdgcn_readlane(key, __ffsll((unsigned long long)valid) - 1);
    const int32_t klast = __builtin_amdgcn_readlane(key, 63 - __clzll((unsigned long long)valid));
    if (kfirst == ckey && klast == ckey) {
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] += v[j];
        return;
    }
    double red[NV];
    if (ckey >= 0) {  // the open run ends in this step (or ended at its start)
#pragma unroll
        for (int j = 0; j < NV; ++j) red[j] = group_sum<STRIDE>(acc[j] + (key == ckey ? v[j] : 0.0));
        flush(ckey, red);
    }
    auto next_after = [&](int32_t k) {
        const uint64_t gt = __ballot(key > k);
        return (int32_t)__builtin_amdgcn_readlane(key, __ffsll((unsigned long long)gt) - 1);
    };
    int32_t k = (kfirst == ckey) ? next_after(ckey) : kfirst;
    while (k != klast) {  // runs that start and end inside the step
#pragma unroll
        for (int j = 0; j < NV; ++j) red[j] = group_sum<STRIDE>(key == k ? v[j] : 0.0);
        flush(k, red);
        k = next_after(k);
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = (key == klast) ? v[j] : 0.0;
    ckey = klast;
}

// Close the open run at the end of a chunk.
template <int NV, int STRIDE, typename F>
__device__ __forceinline__ void run_close(double (&acc)[NV], int32_t& ckey, F&& flush) {
    if (ckey < 0) return;
    double red[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) red[j] = group_sum<STRIDE>(acc[j]);
    flush(ckey, red);
    ckey = -1;
}

// ---------------------------------------------------------------------------------------
// aprod 1:  sum_i = sum_k A[i,k] xx[col(i,k)], then
//   A1_ADD   : y[i] += sum_i
//   A1_LSQR  : y[i] = xs sum_i - ys y[i]  with (xs, ys) = (sv, alpha su)   [forward operator]
//   A1_LSQR_T: same with (xs, ys) = (su, beta sv)                           [transposed]
//   A1_RESID : y[i] = b[i] - sum_i
// LSQR modes also write the block partial of sum y[i]^2.  LDSI: the instrumental part of xx
// is staged in LDS (dynamic LDS of n_instr doubles).  TILED: coefficients and indices come
// from the row tiles (vals, star, att, instr then unused).  gate (may be NULL): nothing is
// done when *gate is set (a residual of a correction step that will not be taken).
enum { A1_ADD = 0, A1_LSQR = 1, A1_LSQR_T = 2, A1_RESID = 3 };

template <typename VT, int MODE, bool TILED, bool LDSI>
static __global__ __launch_bounds__(512) void k_aprod1(
    Geo g, const VT* __restrict__ vals, const int32_t* __restrict__ star,
    const int32_t* __restrict__ att, const int32_t* __restrict__ instr,
    const VT* __restrict__ tiles, const double* __restrict__ xx, double* __restrict__ y,
    const double* __restrict__ b,
    const LsqrState* __restrict__ st, double* __restrict__ partials, int chunk_rows,
    const int32_t* __restrict__ gate) {
    extern __shared__ double lxi[];
    __shared__ double sh[512 / kWave];
    if (gate && *gate) return;
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
    if (LDSI) {
        for (int k = threadIdx.x; k < g.I; k += blockDim.x) lxi[k] = xx[g.ins0 + k];
        __syncthreads();
    }
    const double* __restrict__ xi = LDSI ? lxi : xx + g.ins0;
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
            double a[6];
            int32_t s, t, ia, ib;
            // the row's old y (or b) is loaded with the coefficients, not after the gathers
            // (one memory round trip fewer per step)
            const int64_t rr = valid ? r : r_end - 1;  // in-bounds stand-in row
            double yo = 0.0;
            if (MODE == A1_RESID)
                yo = b[rr];
            else if (MODE == A1_ADD || (kLsqr && ys != 0.0))
                yo = y[rr];
            if (TILED) {  // the whole step's tile (rows past m are padding inside it)
                ld_tile(tiles, r0 / kStepRows, lane, a);
                ld_tile_idx(tiles, r0 / kStepRows, lane, s, t, ia, ib);
            } else if (valid) {
                const VT* __restrict__ row = vals + r * kPar + q;
#pragma unroll
                for (int k = 0; k < 6; ++k) a[k] = ld_val(row + 4 * k);
                s = star[r];
                t = att[r];
                ia = instr[r * kInstr + ia_off];
                ib = instr[r * kInstr + ib_off];
            }
            if (valid) {
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
                    y[r] = yo + sum;
                } else if (MODE == A1_RESID) {
                    y[r] = yo - sum;
                } else {
                    const double u = (ys != 0.0) ? xs * sum - ys * yo : xs * sum;
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
//   x[col(i,k)] += A[i,k] y[i]  (A2_ADD; A2_LSQR / A2_LSQR_T, where y is the unnormalized
//   u~ or v~ and the following vector step applies 1/beta or 1/alpha), or the contribution is
//   A[i,k]^2 (A2_SQ, column norms).  LSQR modes return at once when the stop flag is set.
// Astrometric: a star's rows are contiguous; a run is written once by the wave that ends it,
// with a plain read-modify-write when the whole star lies inside the wave's chunk and an
// atomic add when the star continues into a neighbouring chunk.
// Instrumental and global: accumulated in LDS for everything the block visits; the block's
// n_instr + 1 sums go to part[blockIdx] (reduced by k_reduce_partials), or -- when n_instr is
// too large for LDS -- straight to x with atomics.
enum { A2_ADD = 0, A2_LSQR = 1, A2_LSQR_T = 2, A2_SQ = 3 };

template <int MODE>
__device__ __forceinline__ double a2_scale(const LsqrState* __restrict__ st) {
    return 1.0;  // LSQR modes accumulate unnormalized (the vector step applies 1/beta, 1/alpha)
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
        // finished star: row group 0 writes it (astro q; astro 4 from q = 0).  In the LSQR and
        // column-norm modes the target starts at zero, so an owned star is simply stored.
        auto flush = [&](int32_t key, const double (&t)[2]) {
            if (rg != 0) return;
            double* xa = x + (int64_t)kAstro * key;
            if (key == shared_first || key == shared_last) {
                atomic_add_f64(xa + q, t[0]);
                if (q == 0) atomic_add_f64(xa + 4, t[1]);
            } else if (MODE == A2_ADD) {
                xa[q] += t[0];
                if (q == 0) xa[4] += t[1];
            } else {
                xa[q] = t[0];
                if (q == 0) xa[4] = t[1];
            }
        };
        double acc[2] = {0.0, 0.0};  // this lane's share of the open run
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
            run_step<2, kQuad>(key, v, acc, ckey, flush);
        }
        run_close<2, kQuad>(acc, ckey, flush);
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
// blockIdx.y takes a slice of the blocks; slices meet in one atomic add per column.
static __global__ void k_reduce_partials(int ncols, int nblocks, const double* __restrict__ part,
                                         double* __restrict__ x, const LsqrState* __restrict__ st,
                                         int check_stop) {
    if (check_stop && st->stop) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    const int per = (nblocks + gridDim.y - 1) / gridDim.y;
    const int b0 = blockIdx.y * per, b1 = min(nblocks, b0 + per);
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += part[(int64_t)b * ncols + c];
    if (gridDim.y == 1) {
        x[c] += s;
    } else if (b0 < b1) {
        atomic_add_f64(x + c, s);
    }
}

// ---------------------------------------------------------------------------------------
// Fused LSQR u-step and star-ordered part of the following v-step (one read of each row):
//   u~[r] = sv (A xt)[r] - alpha su u~[r]            (xt = p o v~, the previous v-step)
//   s[c] += A[r,c] u~[r]   for the astrometric, instrumental and global columns
// s is accumulated unnormalized (1/beta is applied by the vector step once beta is known);
// the attitude columns of s come from k_aprod2_att on the attitude copy.  Block partials:
// sum u~^2 -> partials[block], instrumental/global sums -> part[block][n_instr + 1].
// U row steps are loaded before any of them is reduced.
//
// TRANS: the same pass for the transposed operator D A^T (the adjoint solve), where the
// row-space vector is v~:  v~[r] = su (A xt)[r] - beta sv v~[r]  (xt = p o u~), preceded on
// the same rows by the pending update z += f1 w; w = sv v~ - f2 w of the row-space z, w.
// Partials then are 4 rows (pstride apart; entries past gridDim belong to the constraint
// rows): sum v~^2, sum z^2, sum z w, sum w^2.
//
// INIT: the initial aprod 2 of a solve: u~ is left as it is (no dot products) and only
// s += A^T u~ is scattered (star-ordered columns; the attitude pass follows as usual).
template <typename VT, int U, bool TRANS = false, bool INIT = false>
static __global__ __launch_bounds__(1024) void k_aprod12(
    Geo g, const VT* __restrict__ tiles, const int32_t* __restrict__ star,
    const double* __restrict__ xx, double* __restrict__ uu, double* __restrict__ s,
    const LsqrState* __restrict__ st, double* __restrict__ partials,
    double* __restrict__ part, int chunk_rows, int pstride, double* __restrict__ ww_vec = nullptr,
    double* __restrict__ zz_vec = nullptr) {
    extern __shared__ double lds[];  // [n_instr + 1] sums, then [n_instr] staged xt
    __shared__ double sh[1024 / kWave];
    if (st->stop) return;
    const double xs = TRANS ? st->su : st->sv;
    const double ys = TRANS ? st->beta * st->sv : st->alpha * st->su;
    const bool pending = TRANS && st->pending;
    const double f1 = st->f1, f2 = st->f2, svo = st->sv;
    double zsq = 0.0, zw = 0.0, wsq = 0.0;
    double* lsum = lds;  // instrumental and global sums of the block
    double* lxi = lds + g.I + 1;
    for (int k = threadIdx.x; k <= g.I; k += blockDim.x) lsum[k] = 0.0;
    if (!INIT)
        for (int k = threadIdx.x; k < g.I; k += blockDim.x) lxi[k] = xx[g.ins0 + k];
    __syncthreads();
    const double* __restrict__ xi = lxi;  // LDS reads (not flat loads tied to vmcnt)
    const int lane = threadIdx.x % kWave, rg = lane / kQuad, q = lane % kQuad;
    const int wpb = blockDim.x / kWave;
    const int64_t nchunks = (g.m + chunk_rows - 1) / chunk_rows;
    const double xglob = INIT ? 0.0 : xx[g.glb0];
    const int jatt = (q + 3) & 3;
    double usq = 0.0, gacc = 0.0;
    for (int64_t ch = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; ch < nchunks;
         ch += (int64_t)gridDim.x * wpb) {
        const int64_t r_beg = ch * (int64_t)chunk_rows;
        const int64_t r_end = min(r_beg + chunk_rows, g.m);
        const int32_t shared_first =
            (r_beg > 0 && star[r_beg - 1] == star[r_beg]) ? star[r_beg] : -1;
        const int32_t shared_last =
            (r_end < g.m && star[r_end] == star[r_end - 1]) ? star[r_end - 1] : -1;
        // finished star (s is zero before this pass: owned stars are stored)
        auto flush = [&](int32_t key, const double (&t)[2]) {
            if (rg != 0) return;
            double* xa = s + (int64_t)kAstro * key;
            if (key == shared_first || key == shared_last) {
                atomic_add_f64(xa + q, t[0]);
                if (q == 0) atomic_add_f64(xa + 4, t[1]);
            } else {
                xa[q] = t[0];
                if (q == 0) xa[4] = t[1];
            }
        };
        double acc[2] = {0.0, 0.0};
        int32_t ckey = -1;
        for (int64_t r0 = r_beg; r0 < r_end; r0 += kStepRows * U) {
            double a[U][6], uo[U];
            int32_t sr[U], tr[U], ia[U], ib[U];
            bool valid[U];
#pragma unroll
            for (int w = 0; w < U; ++w) {
                const int64_t r = r0 + w * kStepRows + rg;
                valid[w] = r < r_end;
                const int64_t rr = valid[w] ? r : r_beg;  // in-bounds stand-in row
                // tiles past the chunk are replaced by its first one (rows of the system's
                // last tile past m are padding inside the allocation)
                const int64_t tile = (r0 + w * kStepRows < r_end) ? r0 / kStepRows + w
                                                                  : r_beg / kStepRows;
                ld_tile(tiles, tile, lane, a[w]);
                ld_tile_idx(tiles, tile, lane, sr[w], tr[w], ia[w], ib[w]);
                uo[w] = uu[rr];
            }
#pragma unroll
            for (int w = 0; w < U; ++w) {
                const int64_t r = r0 + w * kStepRows + rg;
                const double regA = (q == 0) ? a[w][5] : a[w][4];
                double un = uo[w];
                if (!INIT) {
                    // aprod 1 part: the row's dot product, spread over the quad
                    const int64_t ca = (int64_t)kAstro * sr[w];
                    double sum = a[w][0] * xx[ca + q];
                    if (q == 0) sum = fma(a[w][1], xx[ca + 4], sum);
                    const double* __restrict__ xa = xx + g.att0 + tr[w] + jatt;
#pragma unroll
                    for (int ax = 0; ax < kAxes; ++ax) {
                        const double c = (q == 0) ? a[w][ax + 2] : a[w][ax + 1];
                        sum = fma(c, xa[(int64_t)ax * g.T], sum);
                    }
                    sum = fma(regA, xi[ia[w]], sum);
                    if (q == 1 || q == 2) sum = fma(a[w][5], xi[ib[w]], sum);
                    if (q == 3) sum = fma(a[w][5], xglob, sum);
                    sum = quad_sum(sum);
                    un = (ys != 0.0) ? xs * sum - ys * uo[w] : xs * sum;
                }
                int32_t key = -1;
                double v[2] = {0.0, 0.0};
                if (valid[w]) {
                    if (q == 0 && !INIT) {
                        if (TRANS && pending) {  // z, w updated with the old v~ of this row
                            const double wo = ww_vec[r];
                            const double zn = fma(f1, wo, zz_vec[r]);
                            const double wn = svo * uo[w] - f2 * wo;
                            zz_vec[r] = zn;
                            ww_vec[r] = wn;
                            zsq = fma(zn, zn, zsq);
                            zw = fma(zn, wn, zw);
                            wsq = fma(wn, wn, wsq);
                        }
                        uu[r] = un;
                        usq = fma(un, un, usq);
                    }
                    key = sr[w];
                    v[0] = a[w][0] * un;
                    v[1] = (q == 0) ? a[w][1] * un : 0.0;
                    atomicAdd(lsum + ia[w], regA * un);
                    if (q == 1 || q == 2) atomicAdd(lsum + ib[w], a[w][5] * un);
                    if (q == 3) gacc = fma(a[w][5], un, gacc);
                }
                // aprod 2 part, astrometric columns: runs of equal star
                run_step<2, kQuad>(key, v, acc, ckey, flush);
            }
        }
        run_close<2, kQuad>(acc, ckey, flush);
    }
    const double gs = wave_sum(gacc);
    if (lane == 0) atomicAdd(lsum + g.I, gs);
    const double tot = block_sum<1024>(usq, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    if (TRANS) {
        const int G = pstride;
        double t2 = block_sum<1024>(zsq, sh);
        if (threadIdx.x == 0) partials[G + blockIdx.x] = t2;
        t2 = block_sum<1024>(zw, sh);
        if (threadIdx.x == 0) partials[2 * G + blockIdx.x] = t2;
        t2 = block_sum<1024>(wsq, sh);
        if (threadIdx.x == 0) partials[3 * G + blockIdx.x] = t2;
    }
    __syncthreads();
    double* dst = part + (int64_t)blockIdx.x * (g.I + 1);
    for (int k = threadIdx.x; k <= g.I; k += blockDim.x) dst[k] = lsum[k];
}

// ---------------------------------------------------------------------------------------
// aprod 2, attitude columns, over the library-owned copy of the attitude coefficients in
// the order (group, row slice, t).  The attitude starts are cut into nb buckets of W knots
// and the rows into slices of consecutive rows, dealt round-robin to the dies; group
// G = b kXcd + x holds the rows of bucket b in the slices of die x.  Block G (placed by the
// dispatcher on die G % kXcd) takes group G and sums the columns t + q of its bucket, three
// axes, in LDS; its waves move through the die's slices in step with the die's other blocks,
// so the u~ values they gather at any time come from one slice, which the die's L2 holds.
// The block's sums go to part[G] (kAxes rows of lw = W + kParAxis - 1 columns), added to x by
// k_att_reduce.  Row k of the copy (tile k / kStepRows): attT = A[row_k, 5 + 4 a + j],
// rowT[k] = row_k, tL[k] = att[row_k] - b W; group G is rows seg[G] .. seg[G + 1] - 1.
constexpr int kXcd = 8;  // accelerator dies; the dispatcher places block i on die i % 8
constexpr int kBlockAtt = 512;
constexpr int kAttChunkTiles = 2;  // wave steps per chunk (chunks dealt to the waves in turn)

template <typename VT, int MODE>
static __global__ __launch_bounds__(kBlockAtt) void k_aprod2_att(
    Geo g, const VT* __restrict__ attT, const int32_t* __restrict__ rowT,
    const int32_t* __restrict__ tL, const int64_t* __restrict__ seg, int lw,
    const double* __restrict__ y, double* __restrict__ part, const LsqrState* __restrict__ st) {
    if ((MODE == A2_LSQR || MODE == A2_LSQR_T) && st->stop) return;
    extern __shared__ double acc[];  // [kAxes][lw]
    for (int i = threadIdx.x; i < kAxes * lw; i += blockDim.x) acc[i] = 0.0;
    __syncthreads();
    const double ysc = a2_scale<MODE>(st);
    const int lane = threadIdx.x % kWave, rg = lane / kQuad, q = lane % kQuad;
    const int wave = threadIdx.x / kWave, wpb = blockDim.x / kWave;
    const int64_t lo = seg[blockIdx.x], hi = seg[blockIdx.x + 1];
    if (lo < hi) {
        const int64_t t_beg = lo / kStepRows, t_end = (hi + kStepRows - 1) / kStepRows;
        for (int64_t c0 = t_beg + (int64_t)wave * kAttChunkTiles; c0 < t_end;
             c0 += (int64_t)wpb * kAttChunkTiles) {
            const int64_t c1 = min(c0 + kAttChunkTiles, t_end);
            constexpr int U = 2;  // wave steps loaded before any is added
            for (int64_t tl = c0; tl < c1; tl += U) {
                int32_t col[U];
                double va[U][kAxes], yy[U];
                bool valid[U];
#pragma unroll
                for (int w = 0; w < U; ++w) {
                    const int64_t tile = (tl + w < c1) ? tl + w : c0;
                    const int64_t k = tile * kStepRows + rg;
                    valid[w] = tl + w < c1 && k >= lo && k < hi;
                    const int64_t kk = valid[w] ? k : lo;  // in-bounds stand-in
                    col[w] = tL[kk] + q;
                    yy[w] = (MODE == A2_SQ) ? 0.0 : ysc * y[rowT[kk]];
                    ld_att_tile(attT, tile, lane, va[w]);
                }
#pragma unroll
                for (int w = 0; w < U; ++w) {
                    if (!valid[w]) continue;
#pragma unroll
                    for (int ax = 0; ax < kAxes; ++ax)
                        atomicAdd(acc + ax * lw + col[w], contrib<MODE>(va[w][ax], yy[w]));
                }
            }
        }
    }
    __syncthreads();
    double* __restrict__ dst = part + (int64_t)blockIdx.x * kAxes * lw;
    for (int i = threadIdx.x; i < kAxes * lw; i += blockDim.x) dst[i] = acc[i];
}

// x[att0 + a T + c] += the sums of column c over the groups whose bucket covers it: bucket
// c / W of every die and the buckets before it whose columns reach c (the previous one for
// the first kParAxis - 1 columns of a bucket when W >= kParAxis - 1, more when W is smaller).
// check_stop: nothing is done once the LSQR stop flag is set.
static __global__ void k_att_reduce(Geo g, int w, int lw, const double* __restrict__ part,
                                    double* __restrict__ x, const LsqrState* __restrict__ st,
                                    int check_stop) {
    if (check_stop && st->stop) return;
    const int64_t n = (int64_t)kAxes * g.T;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const int64_t ax = e / g.T, c = e - ax * g.T;
        double sum = 0.0;
        for (int64_t b = c / w; b >= 0 && c - b * w < lw; --b) {
            const double* __restrict__ p = part + (b * kXcd * kAxes + ax) * lw + (c - b * w);
#pragma unroll
            for (int d = 0; d < kXcd; ++d) sum += p[(int64_t)d * kAxes * lw];
        }
        x[g.att0 + e] += sum;
    }
}

// Library-owned attitude copy (the order of k_aprod2_att), as attitude tiles: row k of the
// copy is row rowT[k] of the system; ntiles * kTileAtt elements.
template <typename VT>
static __global__ void k_gather_att(int64_t m, int64_t ntiles, const VT* __restrict__ vals,
                                    const int32_t* __restrict__ rowT, VT* __restrict__ attT) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = ntiles * kTileAtt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t tile = e / kTileAtt;
        const int o = (int)(e - tile * kTileAtt);
        const int lane = (o < 2 * kWave) ? o / 2 : o - 2 * kWave;
        const int ax = (o < 2 * kWave) ? o % 2 : 2;
        const int64_t k = tile * kStepRows + lane / kQuad;
        const int j = kParAxis * ax + lane % kQuad;
        attT[e] = k < m ? vals[(int64_t)rowT[k] * kPar + kAstro + j] : (VT)0;
    }
}

static __global__ void k_iota(int64_t m, int32_t* __restrict__ v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
        v[i] = (int32_t)i;
}

// Sort key of row i for the attitude copy: group G = (t / w) kXcd + (slice % kXcd) above the
// slice's number on its die (sbits wide) above t - (t / w) w (tbits wide); slice = i >> shift.
static __global__ void k_att_keys(int64_t m, int shift, int w, int sbits, int tbits,
                                  const int32_t* __restrict__ att, uint64_t* __restrict__ key) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const int64_t slice = i >> shift, t = att[i], b = t / w;
        const uint64_t grp = (uint64_t)(b * kXcd + slice % kXcd);
        key[i] = (((grp << sbits) | (uint64_t)(slice / kXcd)) << tbits) | (uint64_t)(t - b * w);
    }
}

// seg[G] = first position of group G in the sorted keys (G = 0 .. ng; seg[ng] = m).
static __global__ void k_att_seg(int64_t m, int ng, int low_bits, const uint64_t* __restrict__ key,
                                 int64_t* __restrict__ seg) {
    const int grp = blockIdx.x * blockDim.x + threadIdx.x;
    if (grp > ng) return;
    const uint64_t target = (uint64_t)grp << low_bits;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (key[mid] < target)
            lo = mid + 1;
        else
            hi = mid;
    }
    seg[grp] = lo;
}

// The column offset in the bucket, t - b w, from each sorted key.
static __global__ void k_att_tl(int64_t m, uint64_t mask, const uint64_t* __restrict__ key,
                                int32_t* __restrict__ tl) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
        tl[i] = (int32_t)(key[i] & mask);
}

}  // namespace gsr
