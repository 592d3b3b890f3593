// FP64 reductions of FP32 data.  A fixed grid of blocks strides over the data
// in a fixed order, each block writes one FP64 partial, and one block sums the
// partials in a fixed tree: no atomics, so results are bit-reproducible.
#include "mms_internal.h"

namespace mms {
namespace {

constexpr int RBLK = 1024, RTH = 256;

__device__ double block_sum(double v, double *s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < RTH / 64; ++w) t += s[w];
    return t;
}

__global__ void __launch_bounds__(RTH) grid_dot_kernel(const float *a, const float *b, int nx, int ny,
                                                       int nz, int64_t sy, int64_t sz, double *part) {
    __shared__ double s[RTH / 64];
    double v = 0.0;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t off = (r / ny) * sz + (r % ny) * sy;
        for (int x = threadIdx.x; x < nx; x += RTH) {
            const double p = a[off + x];
            v += p * (b ? (double)b[off + x] : p);
        }
    }
    const double t = block_sum(v, s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(RTH) flat_kernel(const float *a, const float *b, float *resid,
                                                   int64_t n, int misfit, double *part) {
    __shared__ double s[RTH / 64];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RTH + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTH) {
        if (misfit) {
            const float d = a[i] - b[i];
            if (resid) resid[i] = d;
            v += 0.5 * (double)d * (double)d;
        } else {
            const double p = a[i];
            v += p * (b ? (double)b[i] : p);
        }
    }
    const double t = block_sum(v, s);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(RTH) finish_kernel(const double *part, int n, double *out) {
    __shared__ double s[RTH];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += RTH) v += part[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = RTH / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

}  // namespace

int reduce_grid_dot(const float *a, const float *b, const mms_grid *g, double *out, double *part,
                    hipStream_t s) {
    const int64_t o = (int64_t)g->halo * (g->sz + g->sy + 1);
    hipLaunchKernelGGL(grid_dot_kernel, dim3(RBLK), dim3(RTH), 0, s, a + o, b ? b + o : nullptr,
                       (int)g->nx, (int)g->ny, (int)g->nz, g->sy, g->sz, part);
    if (int rc = check_launch("grid_dot_kernel")) return rc;
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(RTH), 0, s, part, RBLK, out);
    return check_launch("finish_kernel");
}

int reduce_flat(const float *a, const float *b, float *resid, int64_t n, int misfit, double *out,
                double *part, hipStream_t s) {
    hipLaunchKernelGGL(flat_kernel, dim3(RBLK), dim3(RTH), 0, s, a, b, resid, n, misfit, part);
    if (int rc = check_launch("flat_kernel")) return rc;
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(RTH), 0, s, part, RBLK, out);
    return check_launch("finish_kernel");
}

int reduce_partials_count() { return RBLK; }

}  // namespace mms
