// aprod 2 without a handle and without any allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// it): x += A^T y straight on the caller's arrays in the paper's row layout.
//
// The star-ordered kernel of gsr_aprod2 keeps each block's instrumental and global sums in
// LDS and writes them to a partial-sum buffer, reduced by a second kernel; here that buffer
// is `scratch`, a file-scope device array of fixed size that every call on a GPU shares
// (each GPU holds its own copy until the process ends).  Without the attitude-ordered copy a
// setup would build, the attitude columns take one atomic add per coefficient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "gsr.h"
#include "gsr_internal.hpp"
#include "kernels.hpp"
#include "products.hpp"

using namespace gsr;

namespace {

constexpr int64_t kScratchDoubles = 4 << 20;  // 32 MiB of block partial sums
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's `scratch` (looked up once per device, with it current).
gsr_status scratch_of(int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(GSR_E_UNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return GSR_OK;
}

// x[attitude columns of row r] += A[r, 5 + 4a + j] y[r]; four lanes per row, lane j takes
// column t + j of the three axes.
static __global__ __launch_bounds__(256) void k_aprod2_att_rows(Geo g,
                                                                const double* __restrict__ vals,
                                                                const int32_t* __restrict__ att,
                                                                const double* __restrict__ y,
                                                                double* __restrict__ x) {
    const int q = threadIdx.x % kQuad;
    const int64_t step = (int64_t)gridDim.x * blockDim.x / kQuad;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kQuad; r < g.m;
         r += step) {
        const double yy = y[r];
        const int64_t c = g.att0 + att[r] + q;
        const double* __restrict__ a = vals + r * kPar + kAstro + q;
#pragma unroll
        for (int ax = 0; ax < kAxes; ++ax)
            atomic_add_f64(x + c + (int64_t)ax * g.T, a[kParAxis * ax] * yy);
    }
}

}  // namespace

extern "C" gsr_status gsr_aprod2_noalloc(const gsr_dims* dims, const double* vals,
                                         const int32_t* star, const int32_t* att,
                                         const int32_t* instr, const double* y, double* x,
                                         void* stream) {
    g_last_error.clear();
    gsr_status st = check_dims(dims);
    if (st != GSR_OK) return st;
    if (dims->n_instr > kInstrLdsMax)
        return fail(GSR_E_UNSUPPORTED,
                    "n_instr %d beyond the maximum of this entry point (%d): its instrumental "
                    "sums must fit one block's LDS and the partial-sum scratch",
                    dims->n_instr, kInstrLdsMax);
    if (dims->n_rows == 0) return GSR_OK;
    if (!vals || !star || !att || !instr || !y || !x) return fail(GSR_E_INVAL, "null argument");
    int dev = 0, n_cu = 0;
    if ((st = check_device(&dev, &n_cu)) != GSR_OK) return st;
    double* part = nullptr;
    if ((st = scratch_of(dev, &part)) != GSR_OK) return st;
    const Geo g = make_geo(dims);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // one partial row (n_instr + 1 sums) per block: as many blocks as the scratch holds, at
    // most two per compute unit
    const int64_t ncols = (int64_t)g.I + 1;
    const int blocks = (int)std::max<int64_t>(
        1, std::min<int64_t>(2 * (int64_t)n_cu, kScratchDoubles / ncols));
    constexpr int kThreads = 512;
    const int64_t waves = (int64_t)blocks * kThreads / kWave;
    int64_t chunk = std::max<int64_t>(kStepRows, std::min<int64_t>(1024, g.m / (4 * waves)));
    chunk = (chunk + kStepRows - 1) / kStepRows * kStepRows;
    const size_t lds = sizeof(double) * ncols;
    hipLaunchKernelGGL((k_aprod2_star<double, A2_ADD>), dim3(blocks), dim3(kThreads), lds, s, g,
                       vals, star, instr, y, x, nullptr, part, (int)chunk, 1);
    const int slices = std::max(1, std::min(32, blocks / 8));
    hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((ncols + 255) / 256), slices),
                       dim3(256), 0, s, (int)ncols, blocks, part, x + g.ins0, nullptr, 0);
    const int64_t att_blocks = std::min<int64_t>((g.m * kQuad + 255) / 256, 8 * (int64_t)n_cu);
    hipLaunchKernelGGL(k_aprod2_att_rows, dim3((unsigned)att_blocks), dim3(256), 0, s, g, vals,
                       att, y, x);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gsr_aprod2_noalloc launch");
    return GSR_OK;
}
