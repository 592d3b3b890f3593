// FP64 reductions of FP32 data.  A fixed grid of blocks strides over the data
// in a fixed order, each block writes one FP64 partial (and a count of the terms
// that were not finite), and one block sums the partials in a fixed tree: no
// atomics, so results are bit-reproducible.  The partials live in a workspace
// that the caller owns, so calls on different streams never share memory.
#include "mms_internal.h"

namespace mms {
namespace {

constexpr int RBLK = MMS_REDUCE_WORK / 2, RTH = 256;

// Block sum of (v, bad); thread 0 gets the totals.
__device__ void block_sum2(double &v, double &bad, double *s) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v += __shfl_xor(v, o);
        bad += __shfl_xor(bad, o);
    }
    if ((threadIdx.x & 63) == 0) {
        s[2 * (threadIdx.x >> 6)] = v;
        s[2 * (threadIdx.x >> 6) + 1] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v = 0.0;
        bad = 0.0;
        for (int w = 0; w < RTH / 64; ++w) {
            v += s[2 * w];
            bad += s[2 * w + 1];
        }
    }
}

__device__ __forceinline__ double nonfinite(double t) { return isfinite(t) ? 0.0 : 1.0; }

__global__ void __launch_bounds__(RTH) grid_dot_kernel(const float *a, const float *b, int nx, int ny,
                                                       int nz, int64_t sy, int64_t sz, double *part) {
    __shared__ double s[2 * (RTH / 64)];
    double v = 0.0, bad = 0.0;
    const int64_t rows = (int64_t)ny * nz;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int64_t off = (r / ny) * sz + (r % ny) * sy;
        for (int x = threadIdx.x; x < nx; x += RTH) {
            const double p = a[off + x];
            const double t = p * (b ? (double)b[off + x] : p);
            v += t;
            bad += nonfinite(t);
        }
    }
    block_sum2(v, bad, s);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v;
        part[2 * blockIdx.x + 1] = bad;
    }
}

__global__ void __launch_bounds__(RTH) flat_kernel(const float *a, const float *b, float *resid,
                                                   int64_t n, int misfit, double *part) {
    __shared__ double s[2 * (RTH / 64)];
    double v = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RTH + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTH) {
        double t;
        if (misfit) {
            const float d = a[i] - b[i];
            if (resid) resid[i] = d;
            t = 0.5 * (double)d * (double)d;
        } else {
            const double p = a[i];
            t = p * (b ? (double)b[i] : p);
        }
        v += t;
        bad += nonfinite(t);
    }
    block_sum2(v, bad, s);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v;
        part[2 * blockIdx.x + 1] = bad;
    }
}

}  // namespace

// out[0] = sum of the n partial sums, out[1] = sum of the n bad-term counts
// (part holds n (sum, count) pairs); one block, fixed tree.
__global__ void __launch_bounds__(RTH) finish_pairs_kernel(const double *part, int n, double *out) {
    __shared__ double s[RTH], c[RTH];
    double v = 0.0, bad = 0.0;
    for (int i = threadIdx.x; i < n; i += RTH) {
        v += part[2 * i];
        bad += part[2 * i + 1];
    }
    s[threadIdx.x] = v;
    c[threadIdx.x] = bad;
    __syncthreads();
    for (int w = RTH / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[threadIdx.x] += s[threadIdx.x + w];
            c[threadIdx.x] += c[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s[0];
        out[1] = c[0] + nonfinite(s[0]);
    }
}

__global__ void fill_pair_kernel(double *out, double v) {
    if (threadIdx.x == 0) {
        out[0] = v;
        out[1] = 0.0;
    }
}

__global__ void __launch_bounds__(RTH) flat_scale_kernel(const float *in, const double *scale,
                                                         float *out, int64_t n) {
    const double f = *scale;
    for (int64_t i = (int64_t)blockIdx.x * RTH + threadIdx.x; i < n; i += (int64_t)gridDim.x * RTH)
        out[i] = (float)(f * (double)in[i]);
}

int finish_pairs(const double *part, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(finish_pairs_kernel, dim3(1), dim3(RTH), 0, s, part, n, out);
    return check_launch("finish_pairs_kernel");
}

int fill_pair(double *out, double v, hipStream_t s) {
    hipLaunchKernelGGL(fill_pair_kernel, dim3(1), dim3(64), 0, s, out, v);
    return check_launch("fill_pair_kernel");
}

int reduce_grid_dot(const float *a, const float *b, const mms_grid *g, double *out, double *part,
                    hipStream_t s) {
    const int64_t o = (int64_t)g->halo * (g->sz + g->sy + 1);
    hipLaunchKernelGGL(grid_dot_kernel, dim3(RBLK), dim3(RTH), 0, s, a + o, b ? b + o : nullptr,
                       (int)g->nx, (int)g->ny, (int)g->nz, g->sy, g->sz, part);
    if (int rc = check_launch("grid_dot_kernel")) return rc;
    return finish_pairs(part, RBLK, out, s);
}

int reduce_flat(const float *a, const float *b, float *resid, int64_t n, int misfit, double *out,
                double *part, hipStream_t s) {
    hipLaunchKernelGGL(flat_kernel, dim3(RBLK), dim3(RTH), 0, s, a, b, resid, n, misfit, part);
    if (int rc = check_launch("flat_kernel")) return rc;
    return finish_pairs(part, RBLK, out, s);
}

int flat_scale(const float *in, const double *scale, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return MMS_OK;
    int64_t nb = (n + RTH - 1) / RTH;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(flat_scale_kernel, dim3((unsigned)nb), dim3(RTH), 0, s, in, scale, out, n);
    return check_launch("flat_scale_kernel");
}

}  // namespace mms
