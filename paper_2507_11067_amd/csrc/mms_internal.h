// Internal declarations shared by the HIP translation units of libmmstencil.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mmstencil.h"

namespace mms {

// Records a HIP error for mms_last_error() and returns MMS_EHIP.
int hip_fail(hipError_t e, const char *where);
// Checks hipGetLastError after a launch.
int check_launch(const char *where);
// Records a message for mms_last_error() (for errors that are not HIP's).
void set_last_error(const char *msg);

// Layout checks of the ABI (host side, before any HIP call).
bool grid_ok(const mms_grid *g, int radius);
inline int64_t grid_elems(const mms_grid *g) { return (g->nz + 2 * (int64_t)g->halo) * g->sz; }
inline bool grid_empty(const mms_grid *g) { return g->nx == 0 || g->ny == 0 || g->nz == 0; }
bool overlap(const void *a, int64_t abytes, const void *b, int64_t bbytes);

// Launch geometry that every sweep kernel receives.
struct Geom {
    const float *in0;   // interior origin of the input
    float *out0;        // interior origin of the output
    int nx, ny, nz;
    int H;
    int64_t sy, sz;
    int ntx, nty, nzc;  // tile counts along x, y and z chunks
    int zchunk;
    int txa;            // kernels with balanced x tiles: active lanes per tile row
};

// Balanced x tiles: the fewest tiles of at most `lanes` 16-byte words that cover
// a row of nx cells, all of one width (in words).  Blocks of a one-block-per-CU
// launch then move the same bytes, where fixed-width tiles would leave the last
// tile of a row partly empty (at nx = 400 and 64 lanes: 200 + 200 cells instead
// of 256 + 144).
inline int balanced_tile_words(int nx, int lanes, int *ntx) {
    const int words = (nx + 3) / 4;
    int n = (words + lanes - 1) / lanes;
    if (n < 1) n = 1;
    *ntx = n;
    const int w = (words + n - 1) / n;
    return w < 1 ? 1 : w;
}

// FP64 reduction tail shared by the reductions: out[0] = sum of n partial sums,
// out[1] = sum of n counts of non-finite terms (+1 if the sum itself is not finite);
// part holds n (sum, count) pairs.  fill_pair writes (v, 0).
int finish_pairs(const double *part, int n, double *out, hipStream_t s);
int fill_pair(double *out, double v, hipStream_t s);

// z-chunk length so that (x, y) tiles times z chunks fill `slots` concurrent
// blocks in one wave (slots = CUs x blocks per CU), clamped to [zmin, zmax].
inline int pick_zchunk(int nz, int64_t cols, int64_t slots, int zmin, int zmax) {
    int64_t chunks = cols > 0 ? slots / cols : 1;
    if (chunks < 1) chunks = 1;
    int64_t zc = (nz + chunks - 1) / chunks;
    if (zc < zmin) zc = zmin;
    if (zc > zmax) zc = zmax;
    return (int)zc;
}

// z-chunk that minimises the modelled time of a launch whose blocks all take about
// the same time: ceil(blocks / slots) rounds of (zchunk + overhead) planes, where
// overhead is the per-block fill of the z pipeline in planes, plus a quarter block
// for the uneven finish of the last round.  Larger chunks win ties.
inline int pick_zchunk_rounds(int nz, int64_t cols, int64_t slots, int zmin, int zmax,
                              int overhead) {
    if (cols < 1) cols = 1;
    if (zmax > nz) zmax = nz > zmin ? nz : zmin;
    int best = zmax;
    int64_t best_cost = -1;
    for (int zc = zmax; zc >= zmin; --zc) {
        const int64_t nzc = (nz + zc - 1) / zc;
        const int64_t rounds = (cols * nzc + slots - 1) / slots;
        const int64_t cost4 = 4 * rounds * (int64_t)(zc + overhead) + zc;  // quarter planes
        if (best_cost < 0 || cost4 < best_cost) {
            best_cost = cost4;
            best = zc;
        }
    }
    return best;
}

// Blocks of `kernel` (launched with `threads` threads, no dynamic LDS) that the
// current device holds at once: CUs times resident blocks per CU.
inline int64_t launch_slots(const void *kernel, int threads) {
    int dev = 0, cus = 256, per = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
        per < 1)
        per = 1;
    return (int64_t)cus * per;
}

// Sweep launchers (host), one per kernel family.  coeffs is a host array.
int launch_star(const float *in, float *out, const mms_grid *g, int r, const float *coeffs,
                hipStream_t s);
int launch_box_valu(const float *in, float *out, const mms_grid *g, int r, const float *coeffs,
                    hipStream_t s);
int launch_box_mfma(const float *in, float *out, const mms_grid *g, int r, const float *coeffs,
                    int precision, hipStream_t s);
int launch_plane2d(const float *in, float *out, const mms_grid *g, int shape, int r,
                   const float *coeffs, hipStream_t s);

}  // namespace mms

// 16-byte load that yields zeros when `ok` is false.  The address is replaced by
// `safe` (any valid 16-byte aligned address of the same buffer family) rather
// than the value being selected after a conditional load, which keeps the load
// a plain global load with no speculative path.
__device__ __forceinline__ float4 guarded_load(const float *p, bool ok, const float *safe) {
    const float4 v = *reinterpret_cast<const float4 *>(ok ? p : safe);
    return ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
}

// 16-byte load from p when `ok`, else from `safe`, with no masking of the value.
// For tile words that lie outside the array: they only feed outputs that are never
// stored, so their value does not matter, and an unmasked value keeps the compiler
// from turning the load into a branch (which would force a full wait on every
// load in flight, the prefetch of the next plane included).
__device__ __forceinline__ float4 select_load(const float *p, bool ok, const float *safe) {
    return *reinterpret_cast<const float4 *>(ok ? p : safe);
}

// Absorbing sponge: g(d) = exp(-(a (W - d))^2) for a cell at distance d < W from a
// damped face, 1 elsewhere; gaxis is the factor of one axis at interior index i of n.
__device__ __forceinline__ float mms_g1(int d, int W, float a) {
    if (d >= W) return 1.0f;
    const float t = a * (float)(W - d);
    return __expf(-t * t);
}
__device__ __forceinline__ float gaxis(int i, int n, int W, float a, bool lo, bool hi) {
    float f = 1.0f;
    if (lo) f *= mms_g1(i, W, a);
    if (hi) f *= mms_g1(n - 1 - i, W, a);
    return f;
}

// Blocks are dispatched round-robin over the 8 XCDs of the MI355X (block b runs
// on XCD b % 8).  This bijection gives every XCD one contiguous range of
// logical tiles, so tiles that share halo cells share one L2.
__device__ __forceinline__ int mms_xcd_remap(int b, int n) {
    const int per = n >> 3, rem = n & 7;
    const int xcd = b & 7, idx = b >> 3;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}
