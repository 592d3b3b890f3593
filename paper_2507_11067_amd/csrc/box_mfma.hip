// Box-stencil sweep on the matrix cores (MFMA) with split BF16 / FP16 operands.
//
// The paper maps a one-dimensional stencil onto an outer-product matrix unit by
// multiplying the input rows with a zero-padded coefficient column (Sec. IV-A);
// written as a matrix product this is  out_row = T * in_window  with T a banded
// Toeplitz matrix.  The box is (2r+1)^2 such one-dimensional stencils, one per
// (dz, dy) pair (Sec. IV-C).  Here every (dz, dy) pair becomes a 16 x 24 Toeplitz
// block along x,
//     T_{dz,dy}[m][x'] = c[dz][dy][x' - 4 - m]   (zero outside |x' - 4 - m| <= r),
// and the 2r+1 dy blocks of one dz are laid side by side along K:
//     D(16 x, 16 y) += [T_{dz,-r} .. T_{dz,r}] * [In_{z+dz}(rows y-r..) ; ... ; In(rows y+r..)]
// K per dz is (2r+1)*24, padded to whole 32-wide steps of
// v_mfma_f32_16x16x32_{bf16,f16}.
//
// FP32 accuracy from 16-bit multipliers: every operand x is split as x = hi + lo
// (BF16: hi = RN(x), lo = RN(x - hi); FP16: the same after scaling by a power of
// two that keeps the block's largest |x| below 2^14), and each product is
// formed as hi*hi + hi*lo + lo*hi with FP32 accumulation (lo*lo is dropped).
// The BF16X1 variant keeps hi*hi only.
//
// Work split.  A block owns a 16*NT (x) by 16 (y) output tile and streams z.
// The NW waves of a block split K: wave w owns the 32-wide K steps (chunks)
// c = w, w + NW, ...  and holds their Toeplitz fragments for all 2r+1 dz in
// registers for the whole kernel.  One input plane at a time sits in LDS as
// hi/lo 16-bit arrays (double-buffered); its B fragments are read once per
// chunk and reused by every dz (input plane z' feeds output z' - dz), so each
// wave keeps 2r+1 output accumulators in flight.  After each plane the oldest
// output is complete in every wave; the NW partial tiles are summed through LDS
// and written out.
#include <hip/hip_runtime.h>

#include "mms_internal.h"

namespace mms {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct MfmaArgs {
    Geom g;
    float c[729];      // [dz][dy][dx]
    float cscale;      // FP16 path: power-of-two scale of the weights
};

__device__ __forceinline__ uint32_t f2u(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ float u2f(uint32_t x) { return __builtin_bit_cast(float, x); }

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t bf16_rn(float x) {
    uint32_t u = f2u(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t h) { return u2f((uint32_t)h << 16); }

template <int PREC>
__device__ __forceinline__ void split(float x, float scale, uint16_t &hi, uint16_t &lo) {
    if constexpr (PREC == MMS_FP16X3S) {
        const float xs = x * scale;
        const _Float16 h = (_Float16)xs;
        const _Float16 l = (_Float16)(xs - (float)h);
        hi = __builtin_bit_cast(uint16_t, h);
        lo = __builtin_bit_cast(uint16_t, l);
    } else {
        hi = bf16_rn(x);
        lo = bf16_rn(x - bf16_f(hi));
    }
}

template <int PREC>
__device__ __forceinline__ floatx4 mfma(const uint4 &a, const uint4 &b, floatx4 c) {
    if constexpr (PREC == MMS_FP16X3S) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
}

template <int R, int PREC, int NW, int NT>
__global__ void __launch_bounds__(64 * NW) box_mfma_kernel(MfmaArgs a) {
    constexpr int Q = 2 * R + 1;          // output planes in flight
    constexpr int WX = 24;                // x window per dy (16 + 2r <= 24, 8-aligned)
    constexpr int KD = Q * WX;            // K per dz
    constexpr int NCH = (KD + 31) / 32;   // 32-wide K steps per dz
    constexpr int CPW = (NCH + NW - 1) / NW;
    constexpr int LR = 16 + 2 * R;        // LDS rows per plane
    constexpr int LP = 16 * NT + 8 + 8;   // LDS row pitch in 16-bit cells (8 spare for banks)
    constexpr int NTH = 64 * NW;
    constexpr int C4 = 4 * NT + 2;        // float4 per staged row
    constexpr int NS = LR * C4;           // float4 per staged plane
    constexpr int NSK = (NS + NTH - 1) / NTH;
    constexpr bool SPLIT3 = PREC != MMS_BF16X1;

    __shared__ __attribute__((aligned(16))) uint16_t dhi[2][LR][LP];
    __shared__ __attribute__((aligned(16))) uint16_t dlo[2][LR][LP];
    __shared__ floatx4 red[2][NW][NT][64];
    __shared__ float smax[NW];

    const Geom &g = a.g;
    int b = mms_xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % g.ntx;
    b /= g.ntx;
    const int tyi = b % g.nty;
    const int zci = b / g.nty;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int xt = txi * 16 * NT, yt = tyi * 16;
    const int zb = zci * g.zchunk;
    const int ze = min(zb + g.zchunk, g.nz);
    const int nx4 = (g.nx + 3) & ~3;
    const int ylim = g.ny + g.H;
    const int64_t sy = g.sy, sz = g.sz;

    // staging items: float4 (row, col4) of the plane window
    int64_t s_off[NSK];
    bool s_ok[NSK];
#pragma unroll
    for (int k = 0; k < NSK; ++k) {
        const int i = tid + k * NTH;
        const int row = i / C4, col = i % C4;
        const int yy = yt - R + row, xx = xt - 4 + 4 * col;
        s_ok[k] = (i < NS) && (yy < ylim) && (xx <= nx4);
        s_off[k] = (int64_t)yy * sy + xx;
    }
    const int z_first = zb - R, z_last = ze + R;

    // FP16 path: one power-of-two scale per block from the largest |x| it reads
    float dscale = 1.0f;
    if constexpr (PREC == MMS_FP16X3S) {
        float m = 0.f;
        for (int zi = z_first; zi < z_last; ++zi) {
            const float *p = g.in0 + (int64_t)zi * sz;
#pragma unroll
            for (int k = 0; k < NSK; ++k) {
                const float4 v = guarded_load(p + s_off[k], s_ok[k], g.in0);
                m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        if (lane == 0) smax[wave] = m;
        __syncthreads();
        m = smax[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = fmaxf(m, smax[w]);
        if (m > 0.f && m < 3.0e38f) {
            int e;
            frexpf(m, &e);  // m = f 2^e, 0.5 <= f < 1
            dscale = ldexpf(1.0f, 14 - e);
        }
    }
    const float cscale = (PREC == MMS_FP16X3S) ? a.cscale : 1.0f;

    // Toeplitz fragments of this wave's chunks for every dz (A operand, registers)
    uint4 ahi[CPW][Q], alo[CPW][Q];
    {
        const int m = lane & 15, grp = lane >> 4;
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const int ch = wave + NW * i;
#pragma unroll
            for (int dz = 0; dz < Q; ++dz) {
                uint16_t h[8], l[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int k = 32 * ch + 8 * grp + j;
                    const int dyi = k / WX, xp = k % WX;
                    const int dx = xp - 4 - m;
                    float v = 0.f;
                    if (ch < NCH && dyi < Q && dx >= -R && dx <= R) v = a.c[(dz * Q + dyi) * Q + dx + R];
                    split<PREC>(v, cscale, h[j], l[j]);
                }
                ahi[i][dz] = make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16,
                                        h[4] | (uint32_t)h[5] << 16, h[6] | (uint32_t)h[7] << 16);
                alo[i][dz] = make_uint4(l[0] | (uint32_t)l[1] << 16, l[2] | (uint32_t)l[3] << 16,
                                        l[4] | (uint32_t)l[5] << 16, l[6] | (uint32_t)l[7] << 16);
            }
        }
    }

    float4 stage[NSK];
    auto load_plane = [&](int z) {
        const float *p = g.in0 + (int64_t)z * sz;
#pragma unroll
        for (int k = 0; k < NSK; ++k)
            stage[k] = guarded_load(p + s_off[k], s_ok[k], g.in0);
    };
    auto store_plane = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NSK; ++k) {
            const int i = tid + k * NTH;
            if (i < NS) {
                const int row = i / C4, col = i % C4;
                uint16_t h0, l0, h1, l1, h2, l2, h3, l3;
                split<PREC>(stage[k].x, dscale, h0, l0);
                split<PREC>(stage[k].y, dscale, h1, l1);
                split<PREC>(stage[k].z, dscale, h2, l2);
                split<PREC>(stage[k].w, dscale, h3, l3);
                *reinterpret_cast<uint2 *>(&dhi[buf][row][4 * col]) =
                    make_uint2(h0 | (uint32_t)h1 << 16, h2 | (uint32_t)h3 << 16);
                *reinterpret_cast<uint2 *>(&dlo[buf][row][4 * col]) =
                    make_uint2(l0 | (uint32_t)l1 << 16, l2 | (uint32_t)l3 << 16);
            }
        }
    };

    floatx4 acc[Q][NT];
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[s][t] = floatx4{0.f, 0.f, 0.f, 0.f};

    // B-fragment coordinates of this lane: output row n, K group grp
    const int n = lane & 15, grp = lane >> 4;
    const float outscale = 1.0f / (dscale * cscale);

    load_plane(z_first);
    store_plane(0);
    __syncthreads();
    int buf = 0;
    for (int zi = z_first; zi < z_last;) {
#pragma unroll
        for (int ph = 0; ph < Q; ++ph) {
            if (zi < z_last) {
                const bool more = zi + 1 < z_last;
                if (more) load_plane(zi + 1);
#pragma unroll
                for (int i = 0; i < CPW; ++i) {
                    const int ch = wave + NW * i;
                    if (ch < NCH) {
                        const int k0 = 32 * ch + 8 * grp;
                        const int dyi = k0 / WX, xg = (k0 % WX) / 8;
                        const bool kval = dyi < Q;
                        const int row = kval ? n + dyi : 0;
                        uint4 bhi[NT], blo[NT];
#pragma unroll
                        for (int t = 0; t < NT; ++t) {
                            const uint4 z4 = make_uint4(0, 0, 0, 0);
                            bhi[t] = kval ? *reinterpret_cast<const uint4 *>(&dhi[buf][row][16 * t + 8 * xg]) : z4;
                            blo[t] = (SPLIT3 && kval)
                                         ? *reinterpret_cast<const uint4 *>(&dlo[buf][row][16 * t + 8 * xg])
                                         : z4;
                        }
                        // products outermost so that consecutive MFMAs feed independent
                        // accumulators (2r+1 planes x NT tiles) and never wait on each other
#pragma unroll
                        for (int p = 0; p < (SPLIT3 ? 3 : 1); ++p) {
#pragma unroll
                            for (int dz = -R; dz <= R; ++dz) {
                                const int zo = zi - dz;
                                if (zo < zb || zo >= ze) continue;
                                const int slot = (ph + R - dz + Q) % Q;
                                const uint4 &af = (p == 2) ? alo[i][dz + R] : ahi[i][dz + R];
#pragma unroll
                                for (int t = 0; t < NT; ++t) {
                                    const uint4 &bf = (p == 1) ? blo[t] : bhi[t];
                                    acc[slot][t] = mfma<PREC>(af, bf, acc[slot][t]);
                                }
                            }
                        }
                    }
                }
                // output plane zi - R is complete in this wave's share of K
                const int zo = zi - R;
                const bool emit = zo >= zb && zo < ze;
                if (emit) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) red[buf][wave][t][lane] = acc[ph][t];
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[ph][t] = floatx4{0.f, 0.f, 0.f, 0.f};
                if (more) store_plane(buf ^ 1);
                __syncthreads();
                if (emit) {
                    for (int i = tid; i < NT * 64; i += NTH) {
                        const int t = i / 64, l = i % 64;
                        floatx4 s = red[buf][0][t][l];
#pragma unroll
                        for (int w = 1; w < NW; ++w) s += red[buf][w][t][l];
                        const int y = yt + (l & 15);
                        const int x = xt + 16 * t + 4 * (l >> 4);
                        if (y < g.ny && x < g.nx) {
                            float *po = g.out0 + (int64_t)zo * sz + (int64_t)y * sy + x;
                            const float4 o = make_float4(s[0] * outscale, s[1] * outscale,
                                                         s[2] * outscale, s[3] * outscale);
                            if (x + 3 < g.nx) {
                                *reinterpret_cast<float4 *>(po) = o;
                            } else {
                                if (x + 0 < g.nx) po[0] = o.x;
                                if (x + 1 < g.nx) po[1] = o.y;
                                if (x + 2 < g.nx) po[2] = o.z;
                            }
                        }
                    }
                }
                buf ^= 1;
                ++zi;
            }
        }
    }
}

template <int R, int PREC>
int launch_rp(const float *in, float *out, const mms_grid *gd, const float *coeffs, hipStream_t s) {
    constexpr int NW = 4, NT = 2;
    constexpr int Q = 2 * R + 1;
    MfmaArgs a{};
    Geom &g = a.g;
    g.H = gd->halo;
    g.in0 = in + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.out0 = out + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    g.ntx = (g.nx + 16 * NT - 1) / (16 * NT);
    g.nty = (g.ny + 15) / 16;
    int zc = zchunk_override(MMS_BOX, PREC);
    if (zc <= 0) {
        const int64_t cols = (int64_t)g.ntx * g.nty;
        zc = (int)((int64_t)g.nz * cols / 2048);
        zc = zc < 32 ? 32 : zc;
    }
    g.zchunk = zc;
    g.nzc = (g.nz + zc - 1) / zc;
    float cmax = 0.f;
    for (int i = 0; i < Q * Q * Q; ++i) {
        a.c[i] = coeffs[i];
        const float v = coeffs[i] < 0 ? -coeffs[i] : coeffs[i];
        cmax = v > cmax ? v : cmax;
    }
    a.cscale = 1.0f;
    if (PREC == MMS_FP16X3S && cmax > 0.f && cmax < 3.0e38f) {
        int e;
        frexpf(cmax, &e);
        a.cscale = ldexpf(1.0f, 14 - e);
    }
    const int64_t nblk = (int64_t)g.ntx * g.nty * g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    hipLaunchKernelGGL((box_mfma_kernel<R, PREC, NW, NT>), dim3((unsigned)nblk), dim3(64 * NW), 0,
                       s, a);
    return check_launch("box_mfma_kernel");
}

template <int R>
int launch_r(const float *in, float *out, const mms_grid *g, const float *coeffs, int prec,
             hipStream_t s) {
    switch (prec) {
        case MMS_BF16X3: return launch_rp<R, MMS_BF16X3>(in, out, g, coeffs, s);
        case MMS_FP16X3S: return launch_rp<R, MMS_FP16X3S>(in, out, g, coeffs, s);
        case MMS_BF16X1: return launch_rp<R, MMS_BF16X1>(in, out, g, coeffs, s);
        default: return MMS_EUNSUPPORTED;
    }
}

}  // namespace

int launch_box_mfma(const float *in, float *out, const mms_grid *g, int r, const float *coeffs,
                    int precision, hipStream_t s) {
    switch (r) {
        case 1: return launch_r<1>(in, out, g, coeffs, precision, s);
        case 2: return launch_r<2>(in, out, g, coeffs, precision, s);
        case 3: return launch_r<3>(in, out, g, coeffs, precision, s);
        case 4: return launch_r<4>(in, out, g, coeffs, precision, s);
        default: return MMS_EUNSUPPORTED;
    }
}

}  // namespace mms
