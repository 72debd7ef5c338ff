// C ABI of the PC-LSQR hot path (declarations and contracts in include/gsr.h).
//
// One handle = one system whose coefficient and index arrays stay in the caller's device
// buffers.  The handle owns the preconditioner, the optional binary32 coefficient copy and
// the LSQR work vectors; every LSQR scalar lives in device memory (LsqrState), so an
// iteration is a fixed sequence of kernels that is captured once in a hipGraph and
// replayed; the host only reads the stop flag between replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gsr.h"
#include "gsr_internal.hpp"
#include "kernels.hpp"
#include "products.hpp"
#include "constraints.hpp"

#include <hipcub/hipcub.hpp>

using namespace gsr;

namespace gsr {

thread_local std::string g_last_error;

gsr_status fail(gsr_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

gsr_status hip_fail(hipError_t e, const char* what) {
    return fail(GSR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

gsr_status check_device(int* dev, int* n_cu) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(GSR_E_NODEVICE, "no HIP device visible");
    e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, *dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(GSR_E_NODEVICE, "device %d is %s; this library is built for gfx950", *dev,
                    prop.gcnArchName);
    *n_cu = prop.multiProcessorCount;
    return GSR_OK;
}

gsr_status check_dims(const gsr_dims* d) {
    if (!d) return fail(GSR_E_INVAL, "dims is NULL");
    if (d->n_rows < 0) return fail(GSR_E_INVAL, "n_rows < 0");
    if (d->n_stars < 1) return fail(GSR_E_INVAL, "n_stars < 1");
    if (d->n_dfa < kParAxis) return fail(GSR_E_INVAL, "n_dfa < 4");
    if (d->n_instr < kInstr) return fail(GSR_E_INVAL, "n_instr < 6");
    if (d->n_glob != 1) return fail(GSR_E_UNSUPPORTED, "n_glob must be 1");
    if (d->n_stars > (int64_t)INT32_MAX / kAstro)
        return fail(GSR_E_UNSUPPORTED, "n_stars too large for int32 star indices");
    return GSR_OK;
}

Geo make_geo(const gsr_dims* d) {
    Geo g;
    g.m = d->n_rows;
    g.n_stars = d->n_stars;
    g.T = d->n_dfa;
    g.I = d->n_instr;
    g.att0 = (int64_t)kAstro * d->n_stars;
    g.ins0 = g.att0 + (int64_t)kAxes * d->n_dfa;
    g.glb0 = g.ins0 + d->n_instr;
    g.n = g.glb0 + d->n_glob;
    return g;
}

int grid_for(int64_t items, int per_block, int max_blocks) {
    const int64_t b = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, max_blocks));
}

// Arrays of 1 GiB and more are asked for as physically contiguous memory first, plain
// hipMalloc when that fails.  Measured: with ordinary allocations the fused row pass over
// tens of GB of row tiles ran up to 10% slower in a process started right after another one
// had used and freed most of the device memory, and at full speed with contiguous ones.
hipError_t device_alloc(void** p, size_t bytes) {
    if (bytes >= (size_t(1) << 30)) {
        if (hipExtMallocWithFlags(p, bytes, hipDeviceMallocContiguous) == hipSuccess)
            return hipSuccess;
        (void)hipGetLastError();
    }
    return hipMalloc(p, bytes);
}

}  // namespace gsr

#define HIP_TRY(call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)

#define GSR_TRY(call)                     \
    do {                                  \
        gsr_status s_ = (call);           \
        if (s_ != GSR_OK) return s_;      \
    } while (0)

namespace {

// Workspace of one LSQR recurrence over an operator with `rows` x `cols`.
struct LsqrWork {
    int64_t rows = 0, cols = 0;
    double *u = nullptr, *v = nullptr, *w = nullptr, *z = nullptr;
    double* var = nullptr;  // [cols] variance estimate (solves that return it)
    hipGraphExec_t graph = nullptr;
    int graph_iters = 0;
};

}  // namespace

struct gsr_handle {
    int device = 0;
    int n_cu = 256;
    Geo g;
    const double* vals = nullptr;
    const int32_t *star = nullptr, *att = nullptr, *instr = nullptr;
    float* vals32 = nullptr;
    double *p64 = nullptr, *p32 = nullptr;
    double* s = nullptr;       // [n] aprod 2 accumulator (kept zero between uses)
    double* xt = nullptr;      // [n] operand of the next aprod 1 (p o v)
    // attitude coefficients in (bucket and die, row slice, attitude start) order (built at
    // setup): row of each entry, its column offset in the bucket, group boundaries
    int32_t *rowT = nullptr, *tT = nullptr;
    double* attT64 = nullptr;
    float* attT32 = nullptr;
    int64_t* att_seg = nullptr;   // [att_ng + 1]
    double* att_part = nullptr;   // [att_ng][kAxes][att_lw] group sums of the attitude pass
    int att_ng = 1, att_w = 1, att_lw = kParAxis;
    double* part_ig = nullptr;  // [G2s][n_instr + 1] block sums of the star-ordered pass
    double *partA = nullptr, *partB = nullptr;
    LsqrState* st = nullptr;   // device scalars
    LsqrState* st_host = nullptr;  // pinned mirror
    int G1 = 1, G2s = 1, Gn = 1, Gm = 1;
    int chunk1 = 16, chunk2s = 16;
    int lds1 = 0, lds2 = 0;           // instrumental columns staged / privatized in LDS
    size_t lds1_bytes = 0, lds2_bytes = 0;
    // fused row pass (aprod 1 + star-ordered part of aprod 2), used when n_instr fits LDS
    int fused = 0, G12 = 1, chunk12 = 16;
    int allow_empty = 0;           // setup option: all-zero columns accepted
    size_t lds12_bytes = 0;
    // row tiles of the fused pass (coefficients per precision, packed indices)
    int64_t ntiles = 0;
    double* tiles64 = nullptr;
    float* tiles32 = nullptr;
    LsqrWork fwd64, fwd32, trans;  // forward (per precision) and transposed recurrences
    LsqrWork fwd64v;               // forward recurrence with the variance estimate
    // residual correction of the precision form (allocated at setup with the binary32 copy)
    double *dx = nullptr, *r = nullptr;  // [n] correction, [m] residual
    double* ref_part = nullptr;          // [2 Gn] partial norms of a correction step
    RefState* ref = nullptr;             // loop state (device)
    RefState* ref_host = nullptr;        // pinned mirror
    hipStream_t cap = nullptr;     // capture stream
    // constraint rows below the observation rows (gsr_set_constraints)
    int64_t n_con = 0, nnz_c = 0;
    const int64_t *cptr = nullptr, *ccol = nullptr;  // caller's rows (device)
    const double* cval = nullptr;
    int32_t* crow = nullptr;     // [nnz_c] row of each entry
    double* cacc = nullptr;      // [n_con] dot products (kept zero between uses)
    int64_t ncu = 0;             // distinct columns of C
    int64_t *cu_col = nullptr, *cu_ptr = nullptr;  // [ncu], [ncu + 1]
    int32_t* cu_row = nullptr;   // [nnz_c] entries grouped by column: row, value
    double* cu_val = nullptr;
    int Gcon = 1;
    int64_t con_per_block = 0;
    int nc1 = 0;                 // 1 when constraint rows exist (one more partial-sum slot)
    int64_t rows() const { return g.m + n_con; }  // rows of the stacked operator
};

namespace {

constexpr int kVecBlocksMax = 2048;
constexpr int kGraphIters = 16;

template <typename T>
gsr_status dalloc(T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = device_alloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(GSR_E_NOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    return GSR_OK;
}

void dfree(void* p) {
    if (p) (void)hipFree(p);
}

void free_work(LsqrWork& w) {
    if (w.graph) (void)hipGraphExecDestroy(w.graph);
    dfree(w.u);
    dfree(w.v);
    dfree(w.w);
    dfree(w.z);
    dfree(w.var);
    w = LsqrWork();
}

gsr_status ensure_work(LsqrWork& w, int64_t rows, int64_t cols, bool with_var = false) {
    if (w.u) return GSR_OK;
    w.rows = rows;
    w.cols = cols;
    GSR_TRY(dalloc(&w.u, rows));
    GSR_TRY(dalloc(&w.v, cols));
    GSR_TRY(dalloc(&w.w, cols));
    GSR_TRY(dalloc(&w.z, cols));
    if (with_var) GSR_TRY(dalloc(&w.var, cols));
    return GSR_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

void fill(double* v, int64_t n, double val, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock, kVecBlocksMax)), dim3(kBlock), 0, s, v,
                       n, val);
}

// ---- launches of the products --------------------------------------------------------

constexpr int kBlock1 = 512;   // aprod 1
constexpr int kBlock2s = 512;  // aprod 2, star-ordered pass

const double* tiles_of(const gsr_handle* h, const double*) { return h->tiles64; }
const float* tiles_of(const gsr_handle* h, const float*) { return h->tiles32; }

// Constraint rows.  y_c (op)= C x with the operation of k_con_fin (LSQR modes write their
// partial sums to part[0] (and part[stride], ... with PENDING)).
template <int MODE, bool TRANS = false, bool PENDING = false>
void launch_con_a1(const gsr_handle* h, const double* x, double* yc, const double* bc,
                   double* part, int stride, double* wc, double* zc, hipStream_t s,
                   const int32_t* gate = nullptr) {
    if (!h->n_con) return;
    if (h->nnz_c > 0)
        hipLaunchKernelGGL(k_con_dot, dim3(h->Gcon), dim3(kConBlock), 0, s, h->nnz_c,
                           h->con_per_block, h->crow, h->ccol, h->cval, x, h->cacc, h->st,
                           (int)(MODE == CON_LSQR), gate);
    hipLaunchKernelGGL((k_con_fin<MODE, TRANS, PENDING>), dim3(1), dim3(kConBlock), 0, s,
                       h->n_con, h->cacc, yc, bc, h->st, part, stride, wc, zc, gate);
}

// x += C^T y_c (SQ: the squared coefficients, for the column norms; y_c unused)
template <bool SQ>
void launch_con_a2(const gsr_handle* h, const double* yc, double* x, int check_stop,
                   hipStream_t s) {
    if (!h->n_con || !h->ncu) return;
    hipLaunchKernelGGL((k_con_a2<SQ>), dim3(grid_for(h->ncu, kConBlock, kVecBlocksMax)),
                       dim3(kConBlock), 0, s, h->ncu, h->cu_col, h->cu_ptr, h->cu_row, h->cu_val,
                       yc, x, h->st, check_stop);
}

// y (op)= A xx, from the row tiles when the library built them for this precision; then the
// constraint rows of y (binary64 coefficients in every precision)
template <typename VT, int MODE>
void launch_aprod1(const gsr_handle* h, const VT* vals, const double* xx, double* y,
                   const double* b, hipStream_t s, const int32_t* gate = nullptr) {
    const VT* tiles = tiles_of(h, vals);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(h->G1), dim3(kBlock1), h->lds1_bytes, s, h->g, vals,
                           h->star, h->att, h->instr, tiles, xx, y, b, h->st,
                           h->partA, h->chunk1, gate);
    };
    if (tiles && h->lds1)
        go(k_aprod1<VT, MODE, true, true>);
    else if (tiles)
        go(k_aprod1<VT, MODE, true, false>);
    else if (h->lds1)
        go(k_aprod1<VT, MODE, false, true>);
    else
        go(k_aprod1<VT, MODE, false, false>);
    const int64_t m = h->g.m;
    if (MODE == A1_ADD)
        launch_con_a1<CON_ADD>(h, xx, y + m, nullptr, nullptr, 0, nullptr, nullptr, s);
    else if (MODE == A1_RESID)
        launch_con_a1<CON_RESID>(h, xx, y + m, b + m, nullptr, 0, nullptr, nullptr, s, gate);
    else  // the u-step's (or transposed v-step's) sum of squares continues in slot G1
        launch_con_a1<CON_LSQR, MODE == A1_LSQR_T>(h, xx, y + m, nullptr, h->partA + h->G1, 0,
                                                   nullptr, nullptr, s);
}

// x[ins0 .. glb0] += the blocks' instrumental/global sums in part_ig
void launch_reduce(const gsr_handle* h, int nblocks, double* x, int check_stop, hipStream_t s) {
    const int ncols = h->g.I + 1;
    const int slices = std::max(1, std::min(32, nblocks / 8));
    hipLaunchKernelGGL(k_reduce_partials, dim3((ncols + 255) / 256, slices), dim3(256), 0, s,
                       ncols, nblocks, h->part_ig, x + h->g.ins0, h->st, check_stop);
}

// x += A^T y over the attitude columns: the attitude pass over the library's copy, then the
// sums of its groups added to x.
template <typename VT, int MODE>
void launch_att(const gsr_handle* h, const VT* attT, const double* y, double* x, hipStream_t s) {
    const Geo& g = h->g;
    if (g.m == 0) return;
    hipLaunchKernelGGL((k_aprod2_att<VT, MODE>), dim3(h->att_ng), dim3(kBlockAtt),
                       sizeof(double) * kAxes * h->att_lw, s, g, attT, h->rowT, h->tT,
                       h->att_seg, h->att_lw, y, h->att_part, h->st);
    const int64_t n = (int64_t)kAxes * g.T;
    hipLaunchKernelGGL(k_att_reduce, dim3(grid_for(n, kBlock, kVecBlocksMax)), dim3(kBlock), 0,
                       s, g, h->att_w, h->att_lw, h->att_part, x, h->st,
                       (int)(MODE == A2_LSQR || MODE == A2_LSQR_T));
}

// x += A^T y: star-ordered pass (astrometric, instrumental, global), reduction of the
// instrumental/global block sums, attitude pass over the library's copy.
template <typename VT, int MODE>
void launch_aprod2(const gsr_handle* h, const VT* vals, const VT* attT, const double* y,
                   double* x, hipStream_t s) {
    const Geo& g = h->g;
    hipLaunchKernelGGL((k_aprod2_star<VT, MODE>), dim3(h->G2s), dim3(kBlock2s), h->lds2_bytes, s,
                       g, vals, h->star, h->instr, y, x, h->st, h->part_ig, h->chunk2s, h->lds2);
    if (h->lds2) launch_reduce(h, h->G2s, x, (int)(MODE == A2_LSQR || MODE == A2_LSQR_T), s);
    launch_att<VT, MODE>(h, attT, y, x, s);
    launch_con_a2<MODE == A2_SQ>(h, MODE == A2_SQ ? nullptr : y + g.m, x,
                                 (int)(MODE == A2_LSQR || MODE == A2_LSQR_T), s);
}

// p = 1 / column norms of `vals`.  Synchronizes.
template <typename VT>
gsr_status colnorm(gsr_handle* h, const VT* vals, const VT* attT, double* p, hipStream_t s,
                   unsigned long long* n_empty) {
    unsigned long long* d_cnt = nullptr;
    GSR_TRY(dalloc(&d_cnt, 1));
    HIP_TRY(hipMemsetAsync(d_cnt, 0, sizeof(*d_cnt), s));
    fill(h->s, h->g.n, 0.0, s);
    launch_aprod2<VT, A2_SQ>(h, vals, attT, nullptr, h->s, s);
    hipLaunchKernelGGL(k_recip_sqrt, dim3(grid_for(h->g.n, kBlock, kVecBlocksMax)), dim3(kBlock),
                       0, s, h->g.n, h->s, p, d_cnt);
    hipError_t e = hipMemcpyAsync(n_empty, d_cnt, sizeof(*d_cnt), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(d_cnt);
    if (e != hipSuccess) return hip_fail(e, "column norms");
    return GSR_OK;
}

// The attitude copy (see k_aprod2_att): rows sorted by (group, slice on its die, t - b W)
// with a stable radix sort, the group boundaries, and the attitude coefficients gathered in
// that order.  Buckets: kAttBuckets per die (512 blocks of kBlockAtt threads on 256 compute
// units, 16 waves per unit: measured faster than 8, whose loads in flight do not fill the
// memory pipe, and than 32, whose gathers and streamed lines crowd the slice out of L2), fewer
// when T is small, more when a bucket's sums would outgrow kAttLdsBytes.  Slices: 2^16 rows
// (512 KiB of binary64 u~, well inside a die's 4 MiB L2 beside the streamed coefficients),
// shorter for small systems so that every die gets slices.  Synchronizes.
constexpr int kAttBuckets = 64;
constexpr size_t kAttLdsBytes = 40 * 1024;

gsr_status build_att_order(gsr_handle* h, hipStream_t s) {
    const Geo& g = h->g;
    const int64_t m = g.m;
    GSR_TRY(dalloc(&h->rowT, m));
    GSR_TRY(dalloc(&h->tT, m));
    const int64_t ntiles_att = (m + kStepRows - 1) / kStepRows;
    GSR_TRY(dalloc(&h->attT64, ntiles_att * kTileAtt));
    if (m > (int64_t)INT32_MAX) return fail(GSR_E_UNSUPPORTED, "more than 2^31-1 rows");
    auto bits_for = [](int64_t v) {  // bits that hold 0 .. v
        int b = 0;
        while (b < 63 && (v >> b) != 0) ++b;
        return b;
    };
    const int64_t T = std::max<int64_t>(g.T, 1);
    const int64_t w_max = (int64_t)(kAttLdsBytes / (sizeof(double) * kAxes)) - (kParAxis - 1);
    int64_t nb = std::min<int64_t>(kAttBuckets, T);
    int64_t w = (T + nb - 1) / nb;
    if (w > w_max) {
        nb = (T + w_max - 1) / w_max;
        w = (T + nb - 1) / nb;
    }
    if (nb * kXcd > INT32_MAX / 2) return fail(GSR_E_UNSUPPORTED, "too many attitude knots");
    h->att_w = (int)w;
    h->att_lw = (int)w + kParAxis - 1;
    h->att_ng = (int)(nb * kXcd);
    GSR_TRY(dalloc(&h->att_seg, (size_t)h->att_ng + 1));
    GSR_TRY(dalloc(&h->att_part, (size_t)h->att_ng * kAxes * h->att_lw));
    if (m == 0) return GSR_OK;
    int shift = 16;
    while (shift > 8 && (m >> shift) < 64) --shift;
    const int sbits = bits_for(((m - 1) >> shift) / kXcd);
    const int tbits = bits_for(w - 1);
    const int low_bits = sbits + tbits;
    const int end_bit = bits_for(h->att_ng - 1) + low_bits;
    int32_t* iota = nullptr;
    uint64_t *keys = nullptr, *keys_out = nullptr;
    gsr_status st = dalloc(&iota, m);
    if (st == GSR_OK) st = dalloc(&keys, m);
    if (st == GSR_OK) st = dalloc(&keys_out, m);
    if (st != GSR_OK) {
        dfree(iota);
        dfree(keys);
        return st;
    }
    const dim3 vgrid(grid_for(m, kBlock, kVecBlocksMax));
    hipLaunchKernelGGL(k_iota, vgrid, dim3(kBlock), 0, s, m, iota);
    hipLaunchKernelGGL(k_att_keys, vgrid, dim3(kBlock), 0, s, m, shift, (int)w, sbits, tbits,
                       h->att, keys);
    size_t temp_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys, keys_out, iota,
                                                      h->rowT, (int)m, 0, end_bit, s);
    void* temp = nullptr;
    if (e == hipSuccess) e = hipMalloc(&temp, std::max<size_t>(temp_bytes, 1));
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys, keys_out, iota, h->rowT,
                                               (int)m, 0, end_bit, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_att_seg, dim3((h->att_ng + 1 + 255) / 256), dim3(256), 0, s, m,
                           h->att_ng, low_bits, keys_out, h->att_seg);
        hipLaunchKernelGGL(k_att_tl, vgrid, dim3(kBlock), 0, s, m, (1ull << tbits) - 1, keys_out,
                           h->tT);
        const int64_t total = ntiles_att * kTileAtt;
        hipLaunchKernelGGL(k_gather_att<double>, dim3(grid_for(total, kBlock, 8192)),
                           dim3(kBlock), 0, s, m, ntiles_att, h->vals, h->rowT, h->attT64);
        e = hipStreamSynchronize(s);
    }
    dfree(temp);
    dfree(keys_out);
    dfree(keys);
    dfree(iota);
    if (e != hipSuccess) return hip_fail(e, "attitude ordering");
    return GSR_OK;
}

// ---- one forward PC-LSQR iteration: u- and v-steps, Givens, vector updates -------------

// Events bracketing the two products of one iteration (profile mode only).
struct IterEvents {
    hipEvent_t a1_begin, a1_end, a2_begin, a2_end;
};

void mark(hipEvent_t e, hipStream_t s) {
    if (e) (void)hipEventRecord(e, s);
}

// Fused row pass: u~ = sv A xt - alpha su u~ and s += A^T u~ (astrometric, instrumental,
// global), then the instrumental/global reduction and the attitude pass (s += A_att^T u~).
// The fused row pass (u-step of the forward solve, or with TRANS the v-step of the adjoint
// solve with its pending z/w update in ww/zz), then the instrumental/global block sums and
// the attitude columns of s from the attitude copy.  Sum-of-squares partials go to `parts`.
constexpr int kU12 = 1;  // row steps per load batch of the fused pass (measured best)
template <typename VT, bool TRANS = false, bool INIT = false>
void launch_fused(const gsr_handle* h, const VT* vals, const VT* attT, double* u, double* s_acc,
                  double* parts, hipStream_t s, const IterEvents* ev, double* ww = nullptr,
                  double* zz = nullptr) {
    const Geo& g = h->g;
    const int pstride = h->G12 + h->nc1;  // partial sums: G12 blocks, then the constraint rows
    if (ev) mark(TRANS ? ev->a2_begin : ev->a1_begin, s);
    if (!INIT)  // constraint rows of the same step (with the transposed operator, their
                // pending z/w update too)
        launch_con_a1<CON_LSQR, TRANS, TRANS>(h, h->xt, u + g.m, nullptr, parts + h->G12,
                                              pstride, TRANS ? ww + g.m : nullptr,
                                              TRANS ? zz + g.m : nullptr, s);
    hipLaunchKernelGGL((k_aprod12<VT, kU12, TRANS, INIT>), dim3(h->G12), dim3(1024),
                       h->lds12_bytes, s,
                       g, tiles_of(h, vals), h->star, h->xt, u, s_acc, h->st, parts,
                       h->part_ig, h->chunk12, pstride, ww, zz);
    if (ev) mark(TRANS ? ev->a2_end : ev->a1_end, s);
    if (ev) mark(TRANS ? ev->a1_begin : ev->a2_begin, s);
    launch_reduce(h, h->G12, s_acc, 1, s);
    launch_att<VT, A2_LSQR>(h, attT, u, s_acc, s);
    launch_con_a2<false>(h, u + g.m, s_acc, 1, s);
    if (ev) mark(TRANS ? ev->a1_end : ev->a2_end, s);
}

template <typename VT, bool VAR = false>
void fwd_iteration(const gsr_handle* h, LsqrWork& w, const VT* vals, const VT* attT,
                   const double* p, hipStream_t s, const IterEvents* ev = nullptr) {
    const Geo& g = h->g;
    if (h->fused) {
        // one read of every row: beta u = A (p o v) - alpha u and s = A^T u~ (unnormalized)
        launch_fused<VT>(h, vals, attT, w.u, h->s, h->partA, s, ev);
        hipLaunchKernelGGL(k_scal_beta, dim3(1), dim3(kBlock), 0, s, h->st, h->partA,
                           h->G12 + h->nc1);
    } else {
        // beta u = A (p o v) - alpha u        (xt = p o v~ from the previous vector step)
        if (ev) mark(ev->a1_begin, s);
        launch_aprod1<VT, A1_LSQR>(h, vals, h->xt, w.u, nullptr, s);
        if (ev) mark(ev->a1_end, s);
        hipLaunchKernelGGL(k_scal_beta, dim3(1), dim3(kBlock), 0, s, h->st, h->partA,
                           h->G1 + h->nc1);
        // s = A^T u~ (unnormalized)
        if (ev) mark(ev->a2_begin, s);
        launch_aprod2<VT, A2_LSQR>(h, vals, attT, w.u, h->s, s);
        if (ev) mark(ev->a2_end, s);
    }
    // alpha v = p o (s / beta) - beta v, with the pending z/w update of the previous iteration
    hipLaunchKernelGGL((k_vec_v<false, VAR>), dim3(h->Gn), dim3(kBlock), 0, s, g.n, h->s, p, w.v,
                       w.w, w.z, h->xt, h->st, h->partB, w.var);
    hipLaunchKernelGGL(k_scal_alpha, dim3(1), dim3(kBlock), 0, s, h->st, h->partB, h->Gn,
                       h->partB + h->Gn, h->Gn);
}

// Transposed operator B = D A^T (rows = n_cols, cols = n_rows): u lives in the unknowns'
// space, v / w / z in the observations' space.
void trans_iteration(const gsr_handle* h, LsqrWork& w, hipStream_t s,
                     const IterEvents* ev = nullptr) {
    const Geo& g = h->g;
    if (h->fused) {
        // beta u = D A^T v - alpha u  (s = A^T v~ left by the previous row pass)
        hipLaunchKernelGGL(k_vec_tu, dim3(h->Gn), dim3(kBlock), 0, s, g.n, h->s, h->p64, w.u,
                           h->xt, h->st, h->partA);
        hipLaunchKernelGGL(k_scal_beta, dim3(1), dim3(kBlock), 0, s, h->st, h->partA, h->Gn);
        // one read of every row: pending z/w update, alpha v = A D u - beta v, s = A^T v~
        launch_fused<double, true>(h, h->vals, h->attT64, w.v, h->s, h->partB, s, ev, w.w, w.z);
        const int P = h->G12 + h->nc1;
        hipLaunchKernelGGL(k_scal_alpha, dim3(1), dim3(kBlock), 0, s, h->st, h->partB, P,
                           h->partB + P, P);
        return;
    }
    // beta u = D A^T v - alpha u
    if (ev) mark(ev->a2_begin, s);
    launch_aprod2<double, A2_LSQR_T>(h, h->vals, h->attT64, w.v, h->s, s);
    if (ev) mark(ev->a2_end, s);
    hipLaunchKernelGGL(k_vec_tu, dim3(h->Gn), dim3(kBlock), 0, s, g.n, h->s, h->p64, w.u, h->xt,
                       h->st, h->partA);
    hipLaunchKernelGGL(k_scal_beta, dim3(1), dim3(kBlock), 0, s, h->st, h->partA, h->Gn);
    // pending z/w update, then alpha v = A D u - beta v
    hipLaunchKernelGGL(k_vec_zw, dim3(h->Gm), dim3(kBlock), 0, s, h->rows(), w.v, w.w, w.z,
                       h->st, h->partB);
    if (ev) mark(ev->a1_begin, s);
    launch_aprod1<double, A1_LSQR_T>(h, h->vals, h->xt, w.v, nullptr, s);
    if (ev) mark(ev->a1_end, s);
    hipLaunchKernelGGL(k_scal_alpha, dim3(1), dim3(kBlock), 0, s, h->st, h->partA,
                       h->G1 + h->nc1, h->partB, h->Gm);
}

// Profile mode: the iterations are launched one by one with events around the products;
// mean durations over the iterations actually performed go to `info`.  Synchronizes.
template <typename F>
gsr_status run_profiled(gsr_handle* h, const gsr_solve_opts& o, hipStream_t s, F&& iteration,
                        double* ms1, double* ms2, int* n_done) {
    std::vector<IterEvents> ev((size_t)o.itnlim);
    for (auto& e : ev) {
        HIP_TRY(hipEventCreate(&e.a1_begin));
        HIP_TRY(hipEventCreate(&e.a1_end));
        HIP_TRY(hipEventCreate(&e.a2_begin));
        HIP_TRY(hipEventCreate(&e.a2_end));
    }
    const int every = o.check_every > 0 ? o.check_every : 16;
    int launched = 0;
    gsr_status rc = GSR_OK;
    for (int it = 0; it < o.itnlim; ++it) {
        iteration(s, &ev[(size_t)it]);
        ++launched;
        if (!o.fixed_iters && (it + 1) % every == 0) {
            hipError_t e = hipMemcpyAsync(&h->st_host->stop, &h->st->stop, sizeof(int32_t),
                                          hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                rc = hip_fail(e, "stop flag");
                break;
            }
            if (h->st_host->stop) break;
        }
    }
    hipError_t e = hipMemcpyAsync(h->st_host, h->st, sizeof(LsqrState), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess && rc == GSR_OK) rc = hip_fail(e, "profile sync");
    const int done = std::min(launched, (int)h->st_host->itn);
    double t1 = 0.0, t2 = 0.0;
    for (int it = 0; rc == GSR_OK && it < done; ++it) {
        float a = 0.f, b = 0.f;
        (void)hipEventElapsedTime(&a, ev[(size_t)it].a1_begin, ev[(size_t)it].a1_end);
        (void)hipEventElapsedTime(&b, ev[(size_t)it].a2_begin, ev[(size_t)it].a2_end);
        t1 += a;
        t2 += b;
    }
    for (auto& x : ev) {
        (void)hipEventDestroy(x.a1_begin);
        (void)hipEventDestroy(x.a1_end);
        (void)hipEventDestroy(x.a2_begin);
        (void)hipEventDestroy(x.a2_end);
    }
    *n_done = done;
    *ms1 = done ? t1 / done : 0.0;
    *ms2 = done ? t2 / done : 0.0;
    return rc;
}

template <typename F>
gsr_status capture_graph(gsr_handle* h, LsqrWork& w, F&& body) {
    if (w.graph) return GSR_OK;
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kGraphIters; ++k) body(h->cap);
    hipError_t e = hipStreamEndCapture(h->cap, &graph);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&w.graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        w.graph = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    w.graph_iters = kGraphIters;
    return GSR_OK;
}

// Replays the iteration graph until the device stop flag is set (or itnlim is reached).
gsr_status run_iterations(gsr_handle* h, LsqrWork& w, const gsr_solve_opts& o, hipStream_t s) {
    const int per_check = std::max(1, (o.check_every > 0 ? o.check_every : 16) / w.graph_iters);
    int done = 0;
    while (done < o.itnlim) {
        for (int k = 0; k < per_check && done < o.itnlim; ++k) {
            HIP_TRY(hipGraphLaunch(w.graph, s));
            done += w.graph_iters;
        }
        if (o.fixed_iters || done >= o.itnlim) continue;
        HIP_TRY(hipMemcpyAsync(&h->st_host->stop, &h->st->stop, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h->st_host->stop) break;
    }
    return GSR_OK;
}

struct ProfileOut {
    double ms1 = 0.0, ms2 = 0.0;
    int n = 0;
};

gsr_status read_info(gsr_handle* h, gsr_solve_info* info, hipStream_t s,
                     const ProfileOut& prof) {
    HIP_TRY(hipMemcpyAsync(h->st_host, h->st, sizeof(LsqrState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const LsqrState& t = *h->st_host;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->ms_pass1 = prof.ms1;
        info->ms_pass2 = prof.ms2;
        info->n_pass = prof.n;
        info->fused = h->fused;
        info->itn = t.itn;
        info->istop = t.istop;
        info->n_refine = 1;
        info->nonfinite = t.nonfinite;
        info->rnorm = t.rnorm;
        info->arnorm = t.arnorm;
        info->anorm = std::sqrt(t.anorm2);
        info->znorm = std::sqrt(t.znorm2);
        info->bnorm = t.bnorm;
        info->acond = std::sqrt(t.anorm2) * std::sqrt(t.ddnorm);
    }
    if (t.nonfinite) return fail(GSR_E_BREAKDOWN, "non-finite value in the LSQR recurrence");
    return GSR_OK;
}

// PC-LSQR on A (binary64 or binary32 coefficients): x = p o z; VAR: also the variance
// estimate var_out = p^2 o sum (w_i / rho_i)^2.  Synchronizes.
template <typename VT, bool VAR = false>
gsr_status fwd_solve(gsr_handle* h, LsqrWork& w, const VT* vals, const VT* attT,
                     const double* p, const double* b, double* x, const gsr_solve_opts& o,
                     gsr_solve_info* info, hipStream_t s, double* var_out = nullptr) {
    const Geo& g = h->g;
    GSR_TRY(ensure_work(w, h->rows(), g.n, VAR));
    GSR_TRY(capture_graph(
        h, w, [&](hipStream_t cs) { fwd_iteration<VT, VAR>(h, w, vals, attT, p, cs); }));
    // beta_1 u_1 = b
    hipLaunchKernelGGL(k_copy_norm<false>, dim3(h->Gm), dim3(kBlock), 0, s, h->rows(), b, nullptr,
                       w.u, nullptr, h->partA);
    hipLaunchKernelGGL(k_scal_init1, dim3(1), dim3(kBlock), 0, s, h->st, h->partA, h->Gm,
                       o.itnlim, o.fixed_iters, o.atol, o.btol, o.conlim);
    // alpha_1 v_1 = p o A^T u_1  (the initial aprod 2)
    fill(h->s, g.n, 0.0, s);
    if (h->fused)
        launch_fused<VT, false, true>(h, vals, attT, w.u, h->s, h->partB, s, nullptr);
    else
        launch_aprod2<VT, A2_LSQR>(h, vals, attT, w.u, h->s, s);
    hipLaunchKernelGGL((k_vec_v<true, VAR>), dim3(h->Gn), dim3(kBlock), 0, s, g.n, h->s, p, w.v,
                       w.w, w.z, h->xt, h->st, h->partB, w.var);
    hipLaunchKernelGGL(k_scal_init2, dim3(1), dim3(kBlock), 0, s, h->st, h->partB, h->Gn);
    ProfileOut prof;
    if (o.profile)
        GSR_TRY(run_profiled(
            h, o, s,
            [&](hipStream_t cs, const IterEvents* ev) {
                fwd_iteration<VT, VAR>(h, w, vals, attT, p, cs, ev);
            },
            &prof.ms1, &prof.ms2, &prof.n));
    else
        GSR_TRY(run_iterations(h, w, o, s));
    hipLaunchKernelGGL((k_final<true, VAR>), dim3(h->Gn), dim3(kBlock), 0, s, g.n, p, w.z, w.w,
                       w.v, x, h->st, w.var, var_out);
    HIP_TRY(hipGetLastError());
    return read_info(h, info, s, prof);
}

// Solve information from the device state, written on the device (stream-ordered solve).
// ref (may be NULL): the precision form's loop state, which gives the iteration count summed
// over the correction steps and the number of steps.
static __global__ void k_write_info(const LsqrState* __restrict__ st, gsr_solve_info* info,
                                    int32_t fused, const RefState* __restrict__ ref) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    gsr_solve_info f = {};
    f.itn = st->itn;
    f.istop = st->istop;
    f.n_refine = 1;
    f.nonfinite = st->nonfinite;
    f.rnorm = st->rnorm;
    f.arnorm = st->arnorm;
    f.anorm = sqrt(st->anorm2);
    f.znorm = sqrt(st->znorm2);
    f.bnorm = st->bnorm;
    f.fused = fused;
    f.acond = sqrt(st->anorm2) * sqrt(st->ddnorm);
    if (ref) {
        f.itn = ref->itn;
        f.n_refine = ref->n_refine;
        f.nonfinite = ref->nonfinite | st->nonfinite;
    }
    *info = f;
}

// One PC-LSQR solve with every iteration launched on `s` (no graph of its own, no host
// synchronization, no allocation): capturable into the caller's graph.  All o.itnlim
// iterations are enqueued; once the device stop flag is set the rest return at once.
// gate (may be NULL): when *gate is set at the time the solve would start, it is not started.
template <typename VT>
void fwd_enqueue(const gsr_handle* h, LsqrWork& w, const VT* vals, const VT* attT,
                 const double* p, const double* b, double* x, const gsr_solve_opts& o,
                 hipStream_t s, const int32_t* gate) {
    const Geo& g = h->g;
    hipLaunchKernelGGL(k_copy_norm<false>, dim3(h->Gm), dim3(kBlock), 0, s, h->rows(), b, nullptr,
                       w.u, nullptr, h->partA);
    hipLaunchKernelGGL(k_scal_init1, dim3(1), dim3(kBlock), 0, s, h->st, h->partA, h->Gm,
                       o.itnlim, o.fixed_iters, o.atol, o.btol, o.conlim, gate);
    fill(h->s, g.n, 0.0, s);
    if (h->fused)
        launch_fused<VT, false, true>(h, vals, attT, w.u, h->s, h->partB, s, nullptr);
    else
        launch_aprod2<VT, A2_LSQR>(h, vals, attT, w.u, h->s, s);
    hipLaunchKernelGGL((k_vec_v<true>), dim3(h->Gn), dim3(kBlock), 0, s, g.n, h->s, p, w.v,
                       w.w, w.z, h->xt, h->st, h->partB, nullptr);
    hipLaunchKernelGGL(k_scal_init2, dim3(1), dim3(kBlock), 0, s, h->st, h->partB, h->Gn);
    for (int it = 0; it < o.itnlim; ++it) fwd_iteration<VT>(h, w, vals, attT, p, s);
    hipLaunchKernelGGL((k_final<true>), dim3(h->Gn), dim3(kBlock), 0, s, g.n, p, w.z, w.w, w.v,
                       x, h->st);
}

// Options of inner solve k of the precision form: the correction solves after the first may
// have their own iteration limit, the first its own tolerance.
gsr_solve_opts inner_opts(const gsr_solve_opts& o, int k) {
    gsr_solve_opts ok = o;
    if (k > 0 && o.refine_itnlim > 0) ok.itnlim = o.refine_itnlim;
    if (k == 0 && o.refine_first_tol > 0.0) ok.atol = ok.btol = o.refine_first_tol;
    return ok;
}

const int32_t* ref_stop_flag(const gsr_handle* h) {
    return reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(h->ref) +
                                            offsetof(RefState, stop));
}

// x += d_k, then the device-side test of the correction step (k_ref_check).
void ref_step(const gsr_handle* h, double* x, const gsr_solve_opts& o, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_norms, dim3(h->Gn), dim3(kBlock), 0, s, h->g.n, h->dx, x,
                       h->ref_part, h->ref);
    hipLaunchKernelGGL(k_ref_check, dim3(1), dim3(kBlock), 0, s, h->ref, h->st, h->ref_part,
                       h->Gn, o.refine_tol, o.max_refine);
}

// The binary64 PC-LSQR, stream-ordered.
gsr_status fwd_solve_async(gsr_handle* h, const double* b, double* x, const gsr_solve_opts& o,
                           gsr_solve_info* info_dev, hipStream_t s) {
    fwd_enqueue<double>(h, h->fwd64, h->vals, h->attT64, h->p64, b, x, o, s, nullptr);
    hipLaunchKernelGGL(k_write_info, dim3(1), dim3(64), 0, s, h->st, info_dev, (int32_t)h->fused,
                       nullptr);
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

// The precision form, stream-ordered: all max_refine correction steps are enqueued; the
// test of each step runs on the device and, once it stops the loop, gates the launches of
// the remaining steps (their residual, inner solve and update return at once).
gsr_status f32v_solve_async(gsr_handle* h, const double* b, double* x, const gsr_solve_opts& o,
                            gsr_solve_info* info_dev, hipStream_t s) {
    const Geo& g = h->g;
    const int32_t* gate = ref_stop_flag(h);
    hipLaunchKernelGGL(k_ref_begin, dim3(1), dim3(64), 0, s, h->ref);
    hipLaunchKernelGGL(k_copy, dim3(grid_for(g.m, kBlock, kVecBlocksMax)), dim3(kBlock), 0, s,
                       h->rows(), b, h->r);
    fill(x, g.n, 0.0, s);
    for (int k = 0; k < o.max_refine; ++k) {
        fwd_enqueue<float>(h, h->fwd32, h->vals32, h->attT32, h->p32, h->r, h->dx,
                           inner_opts(o, k), s, gate);
        ref_step(h, x, o, s);
        if (k + 1 < o.max_refine)
            launch_aprod1<double, A1_RESID>(h, h->vals, x, h->r, b, s, gate);
    }
    hipLaunchKernelGGL(k_write_info, dim3(1), dim3(64), 0, s, h->st, info_dev, (int32_t)h->fused,
                       h->ref);
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status trans_solve(gsr_handle* h, const double* gvec, double* mu, const gsr_solve_opts& o,
                       gsr_solve_info* info, hipStream_t s) {
    const Geo& g = h->g;
    LsqrWork& w = h->trans;
    GSR_TRY(ensure_work(w, g.n, h->rows()));
    GSR_TRY(capture_graph(h, w, [&](hipStream_t cs) { trans_iteration(h, w, cs); }));
    // beta_1 u_1 = D g
    hipLaunchKernelGGL(k_copy_norm<true>, dim3(h->Gn), dim3(kBlock), 0, s, g.n, gvec, h->p64,
                       w.u, h->xt, h->partA);
    hipLaunchKernelGGL(k_scal_init1, dim3(1), dim3(kBlock), 0, s, h->st, h->partA, h->Gn,
                       o.itnlim, o.fixed_iters, o.atol, o.btol, o.conlim);
    fill(w.w, h->rows(), 0.0, s);
    fill(w.z, h->rows(), 0.0, s);
    // alpha_1 v_1 = A D u_1 (and, fused, s = A^T v~_1 for the first u-step)
    if (h->fused) {
        fill(h->s, g.n, 0.0, s);
        launch_fused<double, true>(h, h->vals, h->attT64, w.v, h->s, h->partB, s, nullptr, w.w,
                                   w.z);
        hipLaunchKernelGGL(k_scal_init2, dim3(1), dim3(kBlock), 0, s, h->st, h->partB,
                           h->G12 + h->nc1);
    } else {
        launch_aprod1<double, A1_LSQR_T>(h, h->vals, h->xt, w.v, nullptr, s);
        hipLaunchKernelGGL(k_scal_init2, dim3(1), dim3(kBlock), 0, s, h->st, h->partA,
                           h->G1 + h->nc1);
    }
    ProfileOut prof;
    if (o.profile)
        GSR_TRY(run_profiled(
            h, o, s, [&](hipStream_t cs, const IterEvents* ev) { trans_iteration(h, w, cs, ev); },
            &prof.ms1, &prof.ms2, &prof.n));
    else
        GSR_TRY(run_iterations(h, w, o, s));
    hipLaunchKernelGGL(k_final<false>, dim3(h->Gm), dim3(kBlock), 0, s, h->rows(), nullptr, w.z, w.w,
                       w.v, mu, h->st);
    HIP_TRY(hipGetLastError());
    return read_info(h, info, s, prof);
}

void release_constraints(gsr_handle* h) {
    dfree(h->crow);
    dfree(h->cacc);
    dfree(h->cu_col);
    dfree(h->cu_ptr);
    dfree(h->cu_row);
    dfree(h->cu_val);
    h->crow = h->cu_row = nullptr;
    h->cacc = h->cu_val = nullptr;
    h->cu_col = h->cu_ptr = nullptr;
    h->cptr = h->ccol = nullptr;
    h->cval = nullptr;
    h->n_con = h->nnz_c = h->ncu = 0;
    h->nc1 = 0;
}

// Library-side arrays of the constraint rows: the row of every entry, and a copy of the
// entries grouped by column (radix sort by column, run-length encoding into the distinct
// columns, offsets by a scan).  Synchronizes.
gsr_status build_constraints(gsr_handle* h, int64_t n_con, int64_t nnz, const int64_t* ptr,
                             const int64_t* col, const double* val, hipStream_t s) {
    if (n_con == 0) return GSR_OK;
    h->n_con = n_con;
    h->nnz_c = nnz;
    h->cptr = ptr;
    h->ccol = col;
    h->cval = val;
    h->nc1 = 1;
    GSR_TRY(dalloc(&h->cacc, n_con));
    fill(h->cacc, n_con, 0.0, s);
    {  // row pointer non-decreasing
        int* d_flags = nullptr;
        GSR_TRY(dalloc(&d_flags, 1));
        int flags = 0;
        hipError_t e = hipMemsetAsync(d_flags, 0, sizeof(int), s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_con_check_ptr, dim3(grid_for(n_con, kBlock, kVecBlocksMax)),
                               dim3(kBlock), 0, s, n_con, ptr, d_flags);
            e = hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dfree(d_flags);
        if (e != hipSuccess) return hip_fail(e, "constraint rows");
        if (flags) return fail(GSR_E_LAYOUT, "constraint ptr decreases");
    }
    if (nnz == 0) return GSR_OK;
    h->Gcon = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nnz + 4095) / 4096));
    h->con_per_block = (nnz + h->Gcon - 1) / h->Gcon;
    GSR_TRY(dalloc(&h->crow, nnz));
    GSR_TRY(dalloc(&h->cu_row, nnz));
    GSR_TRY(dalloc(&h->cu_val, nnz));
    GSR_TRY(dalloc(&h->cu_col, nnz));
    int32_t *seq = nullptr, *perm = nullptr, *counts = nullptr;
    int64_t* ksorted = nullptr;
    int* d_misc = nullptr;  // [0] check flags, [1] number of distinct columns
    void* temp = nullptr;
    gsr_status rc = GSR_OK;
    auto cleanup = [&]() {
        dfree(seq);
        dfree(perm);
        dfree(counts);
        dfree(ksorted);
        dfree(d_misc);
        dfree(temp);
    };
    if ((rc = dalloc(&seq, nnz)) != GSR_OK || (rc = dalloc(&perm, nnz)) != GSR_OK ||
        (rc = dalloc(&counts, nnz + 1)) != GSR_OK || (rc = dalloc(&ksorted, nnz)) != GSR_OK ||
        (rc = dalloc(&d_misc, 2)) != GSR_OK) {
        cleanup();
        return rc;
    }
    int misc[2] = {0, 0};
    hipError_t e = hipMemsetAsync(d_misc, 0, 2 * sizeof(int), s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_con_rows, dim3(grid_for(nnz, kBlock, kVecBlocksMax)), dim3(kBlock),
                           0, s, n_con, nnz, h->g.n, ptr, col, h->crow, seq, d_misc);
        e = hipMemcpyAsync(misc, d_misc, sizeof(int), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "constraint rows");
    }
    if (misc[0]) {
        cleanup();
        return fail(GSR_E_LAYOUT, "constraint column out of [0, n_cols)");
    }
    int end_bit = 1;
    while (end_bit < 63 && (1LL << end_bit) <= h->g.n) ++end_bit;
    const int n = (int)nnz;
    size_t b1 = 0, b2 = 0, b3 = 0;
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, b1, col, ksorted, seq, perm, n, 0, end_bit, s);
    if (e == hipSuccess)
        e = hipcub::DeviceRunLengthEncode::Encode(nullptr, b2, ksorted, h->cu_col, counts,
                                                  d_misc + 1, n, s);
    if (e == hipSuccess)
        e = hipcub::DeviceScan::ExclusiveSum(nullptr, b3, counts, counts, n + 1, s);
    if (e == hipSuccess) e = hipMalloc(&temp, std::max(std::max(b1, b2), std::max<size_t>(b3, 1)));
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairs(temp, b1, col, ksorted, seq, perm, n, 0, end_bit,
                                               s);
    if (e == hipSuccess)
        e = hipcub::DeviceRunLengthEncode::Encode(temp, b2, ksorted, h->cu_col, counts, d_misc + 1,
                                                  n, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&misc[1], d_misc + 1, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        cleanup();
        return hip_fail(e, "constraint columns");
    }
    h->ncu = misc[1];
    // offsets of the column groups: exclusive scan of the counts with a zero appended
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, counts + h->ncu, (int64_t)1, 0);
    rc = dalloc(&h->cu_ptr, h->ncu + 1);
    int32_t* offs = seq;  // seq is no longer needed: the offsets as int32 (nnz < 2^31)
    if (rc == GSR_OK) {
        e = hipcub::DeviceScan::ExclusiveSum(temp, b3, counts, offs, (int)h->ncu + 1, s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_widen_i32, dim3(grid_for(h->ncu + 1, kBlock, kVecBlocksMax)),
                               dim3(kBlock), 0, s, h->ncu + 1, offs, h->cu_ptr);
            hipLaunchKernelGGL(k_con_gather, dim3(grid_for(nnz, kBlock, kVecBlocksMax)),
                               dim3(kBlock), 0, s, nnz, perm, h->crow, val, h->cu_row, h->cu_val);
            e = hipStreamSynchronize(s);
        }
        if (e != hipSuccess) rc = hip_fail(e, "constraint columns");
    }
    cleanup();
    return rc;
}

gsr_solve_opts default_opts() {
    gsr_solve_opts o;
    std::memset(&o, 0, sizeof o);
    o.itnlim = 100;
    o.fixed_iters = 1;
    o.atol = 1e-14;
    o.btol = 1e-14;
    o.precision = GSR_F64;
    o.max_refine = 4;
    o.refine_tol = 1e-10;
    return o;
}

gsr_status check_opts(const gsr_solve_opts& o) {
    if (o.itnlim < 0) return fail(GSR_E_INVAL, "itnlim < 0");
    if (!(o.atol >= 0) || !(o.btol >= 0)) return fail(GSR_E_INVAL, "atol/btol must be >= 0");
    if (!(o.conlim >= 0)) return fail(GSR_E_INVAL, "conlim must be >= 0");
    if (o.refine_itnlim < 0) return fail(GSR_E_INVAL, "refine_itnlim < 0");
    if (!(o.refine_first_tol >= 0)) return fail(GSR_E_INVAL, "refine_first_tol must be >= 0");
    if (o.precision != GSR_F64 && o.precision != GSR_F32V)
        return fail(GSR_E_INVAL, "unknown precision %d", o.precision);
    if (o.precision == GSR_F32V && o.max_refine < 1) return fail(GSR_E_INVAL, "max_refine < 1");
    return GSR_OK;
}

gsr_status set_device(const gsr_handle* h) {
    HIP_TRY(hipSetDevice(h->device));
    return GSR_OK;
}

}  // namespace

// =======================================================================================
// C ABI

extern "C" {

int32_t gsr_abi_version(void) { return GSR_ABI_VERSION; }

const char* gsr_status_string(gsr_status s) {
    switch (s) {
        case GSR_OK: return "ok";
        case GSR_E_INVAL: return "invalid argument";
        case GSR_E_LAYOUT: return "matrix layout violated";
        case GSR_E_NOMEM: return "device allocation failed";
        case GSR_E_HIP: return "HIP runtime error";
        case GSR_E_BREAKDOWN: return "non-finite value in the iteration";
        case GSR_E_UNSUPPORTED: return "unsupported";
        case GSR_E_NODEVICE: return "no gfx950 device";
    }
    return "unknown status";
}

const char* gsr_last_error(void) { return g_last_error.c_str(); }

gsr_status gsr_lsqr_setup(const gsr_dims* dims, const double* vals, const int32_t* star,
                          const int32_t* att, const int32_t* instr, const gsr_setup_opts* opts,
                          void* stream, gsr_handle** out) {
    g_last_error.clear();
    if (!out) return fail(GSR_E_INVAL, "out is NULL");
    *out = nullptr;
    GSR_TRY(check_dims(dims));
    if (dims->n_rows > 0 && (!vals || !star || !att || !instr))
        return fail(GSR_E_INVAL, "null matrix array");
    if (((uintptr_t)vals & 15) || ((uintptr_t)instr & 7))
        return fail(GSR_E_INVAL, "vals must be 16-byte and instr 8-byte aligned");
    gsr_setup_opts so = {0, 1, 0, 0};
    if (opts) so = *opts;

    int dev = 0, n_cu = 0;
    GSR_TRY(check_device(&dev, &n_cu));
    hipStream_t s = as_stream(stream);

    gsr_handle* h = new gsr_handle();
    h->device = dev;
    h->n_cu = n_cu;
    h->g = make_geo(dims);
    h->vals = vals;
    h->star = star;
    h->att = att;
    h->instr = instr;
    const Geo& g = h->g;
    auto bail = [&](gsr_status st) {
        gsr_destroy(h);
        return st;
    };

    // launch shapes: persistent grids sized by occupancy; row chunks of 16..1024 rows
    // so that every wave slot of the GPU gets several chunks
    h->Gn = grid_for(g.n, kBlock, kVecBlocksMax);
    h->Gm = grid_for(g.m, kBlock, kVecBlocksMax);
    h->lds1 = g.I <= kInstrLdsMax;
    h->lds2 = g.I <= kInstrLdsMax;
    h->lds1_bytes = h->lds1 ? sizeof(double) * g.I : 0;
    h->lds2_bytes = h->lds2 ? sizeof(double) * (g.I + 1) : 0;
    {
        auto occ = [&](const void* fn, int threads, size_t lds) {
            int per_cu = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
            return (e != hipSuccess || per_cu < 1) ? 1 : per_cu;
        };
        // rows per wave chunk: at most 1024, and sized so that every wave of the persistent
        // grid gets (nearly) the same number of chunks (small systems: at least 4 per wave)
        // rows per wave chunk: about `cap`, the same number of chunks for every wave, at
        // least four chunks per wave for small systems
        auto chunk_for = [&](int waves, int64_t cap = 1024) {
            const int64_t w = std::max(waves, 1);
            int64_t c;
            if (g.m >= 4 * cap * w) {
                const int64_t per = (g.m + cap * w - 1) / (cap * w);  // chunks per wave
                c = (g.m + w * per - 1) / (w * per);
            } else {
                c = g.m / (4 * w);
            }
            c = std::max<int64_t>(kStepRows, std::min<int64_t>(cap, c));
            return (int)((c + kStepRows - 1) / kStepRows * kStepRows);
        };
        auto grid = [&](int per_cu, int threads, int chunk) {
            const int64_t chunks = (g.m + chunk - 1) / chunk;
            const int64_t need = (chunks + threads / kWave - 1) / (threads / kWave);
            return (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * n_cu));
        };
        const int o1 = occ((const void*)k_aprod1<double, A1_LSQR, false, true>, kBlock1, h->lds1_bytes);
        const int o2s = occ((const void*)k_aprod2_star<double, A2_LSQR>, kBlock2s, h->lds2_bytes);
        h->chunk1 = chunk_for(o1 * n_cu * kBlock1 / kWave);
        h->chunk2s = chunk_for(o2s * n_cu * kBlock2s / kWave);
        h->G1 = grid(o1, kBlock1, h->chunk1);
        h->G2s = grid(o2s, kBlock2s, h->chunk2s);
        // the fused pass keeps the block's instrumental sums and the instrumental part of xt
        // in LDS (160 KiB per CU)
        h->lds12_bytes = sizeof(double) * (2 * (size_t)g.I + 1);
        h->fused = h->lds2 && h->lds12_bytes <= 160 * 1024;
        if (h->fused) {
            const int o12 = occ((const void*)k_aprod12<double, kU12>, 1024, h->lds12_bytes);
            // about 3,072-row chunks: measured 3.5 % faster than 1,024 at 2e8 rows (fewer
            // chunk switches, each a fresh stream start)
            h->chunk12 = chunk_for(o12 * n_cu * 1024 / kWave, 3072);
            h->G12 = grid(o12, 1024, h->chunk12);
        }
    }
    gsr_status st;
    if ((st = dalloc(&h->p64, g.n)) != GSR_OK) return bail(st);
    if ((st = dalloc(&h->s, g.n)) != GSR_OK) return bail(st);
    if ((st = dalloc(&h->xt, g.n)) != GSR_OK) return bail(st);
    // one more slot than the largest grid: the constraint rows' partial sum
    const int part_len = std::max(std::max(std::max(h->G1, h->Gm), h->Gn), h->G12) + 1;
    if ((st = dalloc(&h->partA, part_len)) != GSR_OK) return bail(st);
    if ((st = dalloc(&h->partB, 4 * (size_t)part_len)) != GSR_OK) return bail(st);
    if (h->lds2 && (st = dalloc(&h->part_ig, (size_t)std::max(h->G2s, h->G12) * (g.I + 1))) !=
                       GSR_OK)
        return bail(st);
    if ((st = dalloc(&h->st, 1)) != GSR_OK) return bail(st);
    // the binary64 solve's vectors: allocated here so that a stream-ordered solve allocates
    // nothing
    if ((st = ensure_work(h->fwd64, g.m, g.n)) != GSR_OK) return bail(st);
    {
        hipError_t e = hipMemsetAsync(h->st, 0, sizeof(LsqrState), s);
        if (e != hipSuccess) return bail(hip_fail(e, "hipMemsetAsync"));
        e = hipHostMalloc((void**)&h->st_host, sizeof(LsqrState), hipHostMallocDefault);
        if (e != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
        e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(hip_fail(e, "hipStreamCreate"));
    }

    if (so.validate && g.m > 0) {
        int* d_flags = nullptr;
        if ((st = dalloc(&d_flags, 1)) != GSR_OK) return bail(st);
        int flags = 0;
        hipError_t e = hipMemsetAsync(d_flags, 0, sizeof(int), s);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_validate, dim3(grid_for(g.m, kBlock, kVecBlocksMax)),
                               dim3(kBlock), 0, s, g, star, att, instr, d_flags);
            e = hipMemcpyAsync(&flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dfree(d_flags);
        if (e != hipSuccess) return bail(hip_fail(e, "validation"));
        if (flags)
            return bail(fail(GSR_E_LAYOUT,
                             "index check failed:%s%s%s%s", (flags & 1) ? " star out of range" : "",
                             (flags & 2) ? " stars not sorted" : "",
                             (flags & 4) ? " attitude start out of [0, n_dfa-4]" : "",
                             (flags & 8) ? " instrumental index out of range" : ""));
    }
    if ((st = build_att_order(h, s)) != GSR_OK) return bail(st);
    unsigned long long n_empty = 0;
    if ((st = colnorm<double>(h, vals, h->attT64, h->p64, s, &n_empty)) != GSR_OK)
        return bail(st);
    h->allow_empty = so.allow_empty_cols;
    if (n_empty && !so.allow_empty_cols)
        return bail(fail(GSR_E_LAYOUT, "%llu all-zero column(s); set allow_empty_cols", n_empty));
    if (h->fused && g.m > 0) {
        h->ntiles = (g.m + kStepRows - 1) / kStepRows;
        const int64_t nv = h->ntiles * kTileVals, ni = h->ntiles * kTileIdx;
        if ((st = dalloc(&h->tiles64, h->ntiles * tile_elems<double>())) != GSR_OK)
            return bail(st);
        hipLaunchKernelGGL(k_make_tiles<double>, dim3(grid_for(nv, kBlock, 8192)), dim3(kBlock), 0,
                           s, g.m, h->ntiles, vals, h->tiles64);
        hipLaunchKernelGGL(k_make_itiles<double>, dim3(grid_for(ni, kBlock, 8192)), dim3(kBlock),
                           0, s, g.m, h->ntiles, h->star, h->att, h->instr, h->tiles64);
        if (so.build_f32) {
            if ((st = dalloc(&h->tiles32, h->ntiles * tile_elems<float>())) != GSR_OK)
                return bail(st);
            hipLaunchKernelGGL(k_make_tiles<float>, dim3(grid_for(nv, kBlock, 8192)),
                               dim3(kBlock), 0, s, g.m, h->ntiles, vals, h->tiles32);
            hipLaunchKernelGGL(k_make_itiles<float>, dim3(grid_for(ni, kBlock, 8192)),
                               dim3(kBlock), 0, s, g.m, h->ntiles, h->star, h->att, h->instr,
                               h->tiles32);
        }
    }
    if (so.build_f32) {
        const int64_t nnz = (int64_t)g.m * kPar,
                      natt = (g.m + kStepRows - 1) / kStepRows * kTileAtt;
        if ((st = dalloc(&h->vals32, nnz)) != GSR_OK) return bail(st);
        if ((st = dalloc(&h->attT32, natt)) != GSR_OK) return bail(st);
        if ((st = dalloc(&h->p32, g.n)) != GSR_OK) return bail(st);
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nnz, kBlock, 8192)), dim3(kBlock), 0, s, nnz,
                           vals, h->vals32);
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(natt, kBlock, 8192)), dim3(kBlock), 0, s,
                           natt, h->attT64, h->attT32);
        unsigned long long n_empty32 = 0;
        if ((st = colnorm<float>(h, h->vals32, h->attT32, h->p32, s, &n_empty32)) != GSR_OK)
            return bail(st);
        // the precision form's workspaces, so that its stream-ordered solve allocates nothing
        if ((st = ensure_work(h->fwd32, g.m, g.n)) != GSR_OK) return bail(st);
        if ((st = dalloc(&h->dx, g.n)) != GSR_OK) return bail(st);
        if ((st = dalloc(&h->r, g.m)) != GSR_OK) return bail(st);
        if ((st = dalloc(&h->ref_part, 2 * (size_t)h->Gn)) != GSR_OK) return bail(st);
        if ((st = dalloc(&h->ref, 1)) != GSR_OK) return bail(st);
        hipError_t e = hipHostMalloc((void**)&h->ref_host, sizeof(RefState), hipHostMallocDefault);
        if (e != hipSuccess) return bail(hip_fail(e, "hipHostMalloc"));
    }
    *out = h;
    return GSR_OK;
}

gsr_status gsr_destroy(gsr_handle* h) {
    if (!h) return GSR_OK;
    (void)hipSetDevice(h->device);
    if (h->cap) (void)hipStreamSynchronize(h->cap);
    (void)hipDeviceSynchronize();
    free_work(h->fwd64);
    free_work(h->fwd64v);
    free_work(h->fwd32);
    free_work(h->trans);
    dfree(h->vals32);
    dfree(h->tiles64);
    dfree(h->tiles32);
    dfree(h->attT32);
    dfree(h->attT64);
    dfree(h->rowT);
    dfree(h->tT);
    dfree(h->att_seg);
    dfree(h->att_part);
    dfree(h->xt);
    dfree(h->part_ig);
    dfree(h->p64);
    dfree(h->p32);
    dfree(h->s);
    dfree(h->partA);
    dfree(h->partB);
    dfree(h->st);
    dfree(h->dx);
    dfree(h->r);
    dfree(h->ref_part);
    dfree(h->ref);
    release_constraints(h);
    if (h->ref_host) (void)hipHostFree(h->ref_host);
    if (h->st_host) (void)hipHostFree(h->st_host);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
    return GSR_OK;
}

gsr_status gsr_get_size(const gsr_handle* h, int64_t* n_rows, int64_t* n_cols) {
    if (!h) return fail(GSR_E_INVAL, "handle is NULL");
    if (n_rows) *n_rows = h->rows();
    if (n_cols) *n_cols = h->g.n;
    return GSR_OK;
}

gsr_status gsr_update_values(gsr_handle* h, const double* vals, void* stream) {
    g_last_error.clear();
    if (!h) return fail(GSR_E_INVAL, "handle is NULL");
    const Geo& g = h->g;
    if (g.m > 0 && !vals) return fail(GSR_E_INVAL, "vals is NULL");
    if ((uintptr_t)vals & 15) return fail(GSR_E_INVAL, "vals must be 16-byte aligned");
    GSR_TRY(set_device(h));
    hipStream_t s = as_stream(stream);
    // the captured iterations of the unfused path read the coefficients from `vals`
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamSynchronize(h->cap));
    for (LsqrWork* w : {&h->fwd64, &h->fwd64v, &h->fwd32, &h->trans}) {
        if (w->graph) (void)hipGraphExecDestroy(w->graph);
        w->graph = nullptr;
    }
    h->vals = vals;
    if (g.m > 0) {
        const int64_t ntiles_att = (g.m + kStepRows - 1) / kStepRows;
        const int64_t natt = ntiles_att * kTileAtt;
        hipLaunchKernelGGL(k_gather_att<double>, dim3(grid_for(natt, kBlock, 8192)), dim3(kBlock),
                           0, s, g.m, ntiles_att, vals, h->rowT, h->attT64);
        const int64_t nv = h->ntiles * kTileVals;
        if (h->tiles64)
            hipLaunchKernelGGL(k_make_tiles<double>, dim3(grid_for(nv, kBlock, 8192)),
                               dim3(kBlock), 0, s, g.m, h->ntiles, vals, h->tiles64);
        if (h->tiles32)
            hipLaunchKernelGGL(k_make_tiles<float>, dim3(grid_for(nv, kBlock, 8192)),
                               dim3(kBlock), 0, s, g.m, h->ntiles, vals, h->tiles32);
        if (h->vals32) {
            const int64_t nnz = g.m * kPar;
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nnz, kBlock, 8192)), dim3(kBlock), 0, s,
                               nnz, vals, h->vals32);
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(natt, kBlock, 8192)), dim3(kBlock), 0, s,
                               natt, h->attT64, h->attT32);
        }
        HIP_TRY(hipGetLastError());
    }
    unsigned long long n_empty = 0, n_empty32 = 0;
    GSR_TRY(colnorm<double>(h, vals, h->attT64, h->p64, s, &n_empty));
    if (h->vals32) GSR_TRY(colnorm<float>(h, h->vals32, h->attT32, h->p32, s, &n_empty32));
    if (n_empty && !h->allow_empty)
        return fail(GSR_E_LAYOUT, "%llu all-zero column(s) in the new values; set "
                                  "allow_empty_cols at setup", n_empty);
    return GSR_OK;
}

gsr_status gsr_set_constraints(gsr_handle* h, int64_t n_con, const int64_t* ptr,
                               const int64_t* col, const double* val, void* stream) {
    g_last_error.clear();
    if (!h) return fail(GSR_E_INVAL, "handle is NULL");
    if (n_con < 0) return fail(GSR_E_INVAL, "n_con < 0");
    if (n_con > (int64_t)INT32_MAX) return fail(GSR_E_UNSUPPORTED, "more than 2^31-1 constraint rows");
    if (n_con > 0 && !ptr) return fail(GSR_E_INVAL, "ptr is NULL");
    GSR_TRY(set_device(h));
    hipStream_t s = as_stream(stream);
    int64_t ends[2] = {0, 0};
    if (n_con > 0) {
        HIP_TRY(hipMemcpyAsync(&ends[0], ptr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&ends[1], ptr + n_con, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (ends[0] != 0) return fail(GSR_E_LAYOUT, "constraint ptr[0] must be 0");
        if (ends[1] < 0) return fail(GSR_E_LAYOUT, "constraint ptr[n_con] < 0");
        if (ends[1] > (int64_t)INT32_MAX)
            return fail(GSR_E_UNSUPPORTED, "more than 2^31-1 constraint coefficients");
        if (ends[1] > 0 && (!col || !val)) return fail(GSR_E_INVAL, "col or val is NULL");
    }
    // every solve's state depends on the number of rows: drop it (graphs included)
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamSynchronize(h->cap));
    free_work(h->fwd64);
    free_work(h->fwd64v);
    free_work(h->fwd32);
    free_work(h->trans);
    release_constraints(h);
    gsr_status rc = build_constraints(h, n_con, ends[1], ptr, col, val, s);
    if (rc != GSR_OK) release_constraints(h);
    // the preconditioner includes the constraint rows (binary64 coefficients in both
    // precisions); the workspaces of the stream-ordered solves are allocated again here
    unsigned long long n_empty = 0;
    gsr_status rc2 = colnorm<double>(h, h->vals, h->attT64, h->p64, s, &n_empty);
    if (rc2 == GSR_OK && h->vals32)
        rc2 = colnorm<float>(h, h->vals32, h->attT32, h->p32, s, &n_empty);
    if (rc2 == GSR_OK) rc2 = ensure_work(h->fwd64, h->rows(), h->g.n);
    if (rc2 == GSR_OK && h->vals32) {
        dfree(h->r);
        h->r = nullptr;
        rc2 = dalloc(&h->r, h->rows());
        if (rc2 == GSR_OK) rc2 = ensure_work(h->fwd32, h->rows(), h->g.n);
    }
    return rc != GSR_OK ? rc : rc2;
}

gsr_status gsr_aprod1(gsr_handle* h, const double* x, double* y, void* stream) {
    if (!h || !x || !y) return fail(GSR_E_INVAL, "null argument");
    GSR_TRY(set_device(h));
    launch_aprod1<double, A1_ADD>(h, h->vals, x, y, nullptr, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_aprod2(gsr_handle* h, const double* y, double* x, void* stream) {
    if (!h || !x || !y) return fail(GSR_E_INVAL, "null argument");
    GSR_TRY(set_device(h));
    launch_aprod2<double, A2_ADD>(h, h->vals, h->attT64, y, x, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_aprod1_f32v(gsr_handle* h, const double* x, double* y, void* stream) {
    if (!h || !x || !y) return fail(GSR_E_INVAL, "null argument");
    if (!h->vals32) return fail(GSR_E_UNSUPPORTED, "binary32 copy not built (build_f32 = 0)");
    GSR_TRY(set_device(h));
    launch_aprod1<float, A1_ADD>(h, h->vals32, x, y, nullptr, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_aprod2_f32v(gsr_handle* h, const double* y, double* x, void* stream) {
    if (!h || !x || !y) return fail(GSR_E_INVAL, "null argument");
    if (!h->vals32) return fail(GSR_E_UNSUPPORTED, "binary32 copy not built (build_f32 = 0)");
    GSR_TRY(set_device(h));
    launch_aprod2<float, A2_ADD>(h, h->vals32, h->attT32, y, x, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_precond(gsr_handle* h, int32_t precision, double* p, void* stream) {
    if (!h || !p) return fail(GSR_E_INVAL, "null argument");
    const double* src = precision == GSR_F32V ? h->p32 : h->p64;
    if (!src) return fail(GSR_E_UNSUPPORTED, "binary32 copy not built (build_f32 = 0)");
    GSR_TRY(set_device(h));
    HIP_TRY(hipMemcpyAsync(p, src, sizeof(double) * h->g.n, hipMemcpyDeviceToDevice,
                           as_stream(stream)));
    return GSR_OK;
}

gsr_status gsr_residual(gsr_handle* h, const double* b, const double* x, double* r,
                        void* stream) {
    if (!h || !b || !x || !r) return fail(GSR_E_INVAL, "null argument");
    GSR_TRY(set_device(h));
    launch_aprod1<double, A1_RESID>(h, h->vals, x, r, b, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

gsr_status gsr_lsqr_solve(gsr_handle* h, const double* b, double* x, const gsr_solve_opts* opts,
                          gsr_solve_info* info, void* stream) {
    g_last_error.clear();
    if (!h || !x || (!b && h->g.m > 0)) return fail(GSR_E_INVAL, "null argument");
    const gsr_solve_opts o = opts ? *opts : default_opts();
    GSR_TRY(check_opts(o));
    GSR_TRY(set_device(h));
    hipStream_t s = as_stream(stream);
    if (o.precision == GSR_F64)
        return fwd_solve<double>(h, h->fwd64, h->vals, h->attT64, h->p64, b, x, o, info, s);

    // binary32 coefficients inside, binary64 residual correction outside
    if (!h->vals32) return fail(GSR_E_UNSUPPORTED, "binary32 copy not built (build_f32 = 0)");
    const Geo& g = h->g;
    hipLaunchKernelGGL(k_ref_begin, dim3(1), dim3(64), 0, s, h->ref);
    HIP_TRY(hipMemcpyAsync(h->r, b, sizeof(double) * h->rows(), hipMemcpyDeviceToDevice, s));
    fill(x, g.n, 0.0, s);
    gsr_solve_info inner = {};
    for (int k = 0; k < o.max_refine; ++k) {
        GSR_TRY(fwd_solve<float>(h, h->fwd32, h->vals32, h->attT32, h->p32, h->r, h->dx,
                                 inner_opts(o, k), &inner, s));
        ref_step(h, x, o, s);
        HIP_TRY(hipMemcpyAsync(h->ref_host, h->ref, sizeof(RefState), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h->ref_host->stop) break;
        launch_aprod1<double, A1_RESID>(h, h->vals, x, h->r, b, s);
    }
    HIP_TRY(hipGetLastError());
    if (info) {
        *info = inner;
        info->itn = h->ref_host->itn;
        info->n_refine = h->ref_host->n_refine;
    }
    return GSR_OK;
}

gsr_status gsr_lsqr_solve_var(gsr_handle* h, const double* b, double* x, double* var,
                              const gsr_solve_opts* opts, gsr_solve_info* info, void* stream) {
    g_last_error.clear();
    if (!h || !x || !var || (!b && h->g.m > 0)) return fail(GSR_E_INVAL, "null argument");
    const gsr_solve_opts o = opts ? *opts : default_opts();
    GSR_TRY(check_opts(o));
    if (o.precision != GSR_F64)
        return fail(GSR_E_UNSUPPORTED, "the variance estimate is binary64 only");
    GSR_TRY(set_device(h));
    return fwd_solve<double, true>(h, h->fwd64v, h->vals, h->attT64, h->p64, b, x, o, info,
                                   as_stream(stream), var);
}

gsr_status gsr_lsqr_solve_async(gsr_handle* h, const double* b, double* x,
                                const gsr_solve_opts* opts, gsr_solve_info* info_dev,
                                void* stream) {
    g_last_error.clear();
    if (!h || !x || !info_dev || (!b && h->g.m > 0)) return fail(GSR_E_INVAL, "null argument");
    const gsr_solve_opts o = opts ? *opts : default_opts();
    GSR_TRY(check_opts(o));
    if (o.profile) return fail(GSR_E_INVAL, "profile needs host synchronization");
    GSR_TRY(set_device(h));
    if (o.precision == GSR_F64) return fwd_solve_async(h, b, x, o, info_dev, as_stream(stream));
    if (!h->vals32) return fail(GSR_E_UNSUPPORTED, "binary32 copy not built (build_f32 = 0)");
    return f32v_solve_async(h, b, x, o, info_dev, as_stream(stream));
}

gsr_status gsr_lsqr_solve_adjoint(gsr_handle* h, const double* gvec, double* mu, double* lam,
                                  const gsr_solve_opts* opts, gsr_solve_info* info,
                                  void* stream) {
    g_last_error.clear();
    if (!h || !gvec || !mu || !lam) return fail(GSR_E_INVAL, "null argument");
    gsr_solve_opts o = opts ? *opts : default_opts();
    GSR_TRY(check_opts(o));
    if (o.precision != GSR_F64) return fail(GSR_E_UNSUPPORTED, "adjoint solve is binary64 only");
    GSR_TRY(set_device(h));
    hipStream_t s = as_stream(stream);
    GSR_TRY(trans_solve(h, gvec, mu, o, info ? &info[0] : nullptr, s));
    return fwd_solve<double>(h, h->fwd64, h->vals, h->attT64, h->p64, mu, lam, o,
                             info ? &info[1] : nullptr,
                             s);
}

gsr_status gsr_grad_vals(gsr_handle* h, const double* r, const double* mu, const double* x,
                         const double* lam, double* dvals, void* stream) {
    if (!h || !r || !mu || !x || !lam || !dvals) return fail(GSR_E_INVAL, "null argument");
    if ((uintptr_t)dvals & 15) return fail(GSR_E_INVAL, "dvals must be 16-byte aligned");
    GSR_TRY(set_device(h));
    hipLaunchKernelGGL(k_grad_vals, dim3(h->G1), dim3(kBlock), 0, as_stream(stream), h->g,
                       h->star, h->att, h->instr, r, mu, x, lam, dvals);
    HIP_TRY(hipGetLastError());
    return GSR_OK;
}

}  // extern "C"
