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
// K per dz is (2r+1)*24, cut into 32-wide steps ("chunks") of
// v_mfma_f32_16x16x32_{bf16,f16}; A = Toeplitz fragment, B = input fragment.
//
// FP32 accuracy from 16-bit multipliers: every operand x is split as x = hi + lo
// (BF16: hi = RN(x), lo = RN(x - hi); FP16: the same after scaling by a power of
// two that keeps the block's largest |x| below 2^14), and each product is
// formed as hi*hi + hi*lo + lo*hi with FP32 accumulation (lo*lo is dropped).
// The BF16X1 variant keeps hi*hi only.
//
// Work split.  A block of NW waves owns a (16*NT) x (16*NW) output tile of the (x, y)
// plane and streams a chunk of z.  All Toeplitz fragments (hi and lo, every dz
// and chunk) are built once per block into LDS.  One input plane at a time sits
// in LDS as hi/lo 16-bit arrays.  Each wave owns NT 16x16 tiles (16 rows) and
// walks the full K: per chunk it loads the NT input fragments once and reuses
// them for every dz and product (input plane z' feeds output z' - dz), and each
// Toeplitz fragment pair it loads feeds NT tiles.  A wave therefore keeps 2r+1
// output planes of accumulators in flight; after each input plane the oldest is
// complete, is written, and the window shifts by one.  The next input plane is
// requested from memory one plane ahead, so its latency hides behind a whole
// plane of MFMA work.
#include <hip/hip_runtime.h>

#include "mms_internal.h"

namespace mms {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Launch shape per radius: NW waves per block (one 16-row band each), NT 16x16
// tiles per wave along x.  The block's Toeplitz fragments take 2 KB per (dz,
// chunk) unit of LDS, so radius 4 (63 units) leaves room for 4 waves only
// (4 tiles each); up to radius 3, 8 waves of 2 tiles fit and two waves share
// each SIMD (measured at 512^3: +9 % at radius 3, +19 % at radius 2).
template <int R>
struct MCfg {
    static constexpr int NW = R == 4 ? 4 : 8;
    static constexpr int NT = R == 4 ? 4 : 2;
};

struct MfmaArgs {
    Geom g;
    float c[729];      // [dz][dy][dx]
    float cscale;      // FP16 path: power-of-two scale of the weights
};

// FP32 -> BF16 with round to nearest even (one v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint16_t bf16_rn(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf16_f(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

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

template <int R, int NW, int NT>
struct Shape {
    static constexpr int BXT = 16 * NT;
    static constexpr int BYT = 16 * NW;
    static constexpr int Q = 2 * R + 1;             // output planes in flight, dz values
    static constexpr int WX = 24;                   // x window per dy (16 + 2r <= 24)
    static constexpr int NCH = (Q * WX + 31) / 32;  // 32-wide K steps per dz
    static constexpr int NU = Q * NCH;              // Toeplitz fragment pairs
    static constexpr int LR = BYT + 2 * R;          // LDS rows of a plane
    // LDS row pitch in 16-bit cells, >= BXT + 8 with 2*LP bytes = 16 mod 128, so the 16-byte B-fragment
    // reads of 8 consecutive rows land on 8 distinct groups of 4 banks
    static constexpr int LP = (BXT + 63) / 64 * 64 + 8;
    static constexpr int C4 = BXT / 4 + 2;          // float4 per staged row
    static constexpr int NS = LR * C4;              // float4 per staged plane
    static constexpr int NSK = (NS + 64 * NW - 1) / (64 * NW);
};

template <int R, int NW, int NT>
struct Smem {
    using S = Shape<R, NW, NT>;
    uint4 afrag[S::NU][2][64];   // [unit][hi, lo][lane]
    uint16_t dhi[S::LR][S::LP];
    uint16_t dlo[S::LR][S::LP];
    float smax[NW];
};

template <int R, int PREC, int NW, int NT>
__global__ void __launch_bounds__(64 * NW) box_mfma_kernel(MfmaArgs a) {
    using S = Shape<R, NW, NT>;
    constexpr int BXT = S::BXT, BYT = S::BYT;
    constexpr int Q = S::Q, NCH = S::NCH, C4 = S::C4, NS = S::NS, NSK = S::NSK, WX = S::WX;
    constexpr int NTH = 64 * NW;
    constexpr bool SPLIT3 = PREC != MMS_BF16X1;
    __shared__ Smem<R, NW, NT> sm;

    const Geom &g = a.g;
    int b = mms_xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % g.ntx;
    b /= g.ntx;
    const int tyi = b % g.nty;
    const int zci = b / g.nty;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int xt = txi * BXT, yt = tyi * BYT;
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
        if (lane == 0) sm.smax[wave] = m;
        __syncthreads();
        m = sm.smax[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = fmaxf(m, sm.smax[w]);
        if (m > 0.f && m < 3.0e38f) {
            int e;
            frexpf(m, &e);  // m = f 2^e, 0.5 <= f < 1
            dscale = ldexpf(1.0f, 14 - e);
        }
    }
    const float cscale = (PREC == MMS_FP16X3S) ? a.cscale : 1.0f;

    // Toeplitz fragments of every (dz, chunk) into LDS (A operand)
    for (int item = tid; item < S::NU * 64; item += NTH) {
        const int u = item >> 6, l = item & 63;
        const int dz = u / NCH, ch = u % NCH;
        const int m = l & 15, grp = l >> 4;
        uint16_t h[8], lo[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 32 * ch + 8 * grp + j;
            const int dyi = k / WX, xp = k % WX;
            const int dx = xp - 4 - m;
            float v = 0.f;
            if (dyi < Q && dx >= -R && dx <= R) v = a.c[(dz * Q + dyi) * Q + dx + R];
            split<PREC>(v, cscale, h[j], lo[j]);
        }
        sm.afrag[u][0][l] = make_uint4(h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16,
                                       h[4] | (uint32_t)h[5] << 16, h[6] | (uint32_t)h[7] << 16);
        sm.afrag[u][1][l] = make_uint4(lo[0] | (uint32_t)lo[1] << 16, lo[2] | (uint32_t)lo[3] << 16,
                                       lo[4] | (uint32_t)lo[5] << 16, lo[6] | (uint32_t)lo[7] << 16);
    }

    float4 stage[NSK];
    uint2 shi[NSK], slo[NSK];   // the staged plane split into packed 16-bit hi and lo parts
    auto load_plane = [&](int z) {
        const float *p = g.in0 + (int64_t)z * sz;
#pragma unroll
        for (int k = 0; k < NSK; ++k) stage[k] = guarded_load(p + s_off[k], s_ok[k], g.in0);
    };
    // the split runs while the previous plane's MFMAs execute; only the LDS writes wait
    // for the barrier that frees the plane buffer
    auto split_plane = [&]() {
#pragma unroll
        for (int k = 0; k < NSK; ++k) {
            uint16_t h0, l0, h1, l1, h2, l2, h3, l3;
            split<PREC>(stage[k].x, dscale, h0, l0);
            split<PREC>(stage[k].y, dscale, h1, l1);
            split<PREC>(stage[k].z, dscale, h2, l2);
            split<PREC>(stage[k].w, dscale, h3, l3);
            shi[k] = make_uint2(h0 | (uint32_t)h1 << 16, h2 | (uint32_t)h3 << 16);
            slo[k] = make_uint2(l0 | (uint32_t)l1 << 16, l2 | (uint32_t)l3 << 16);
        }
    };
    auto write_plane = [&]() {
#pragma unroll
        for (int k = 0; k < NSK; ++k) {
            const int i = tid + k * NTH;
            if (i < NS) {
                const int row = i / C4, col = i % C4;
                *reinterpret_cast<uint2 *>(&sm.dhi[row][4 * col]) = shi[k];
                *reinterpret_cast<uint2 *>(&sm.dlo[row][4 * col]) = slo[k];
            }
        }
    };

    // acc[k][t] holds the partial sum of output plane zi - R + k
    floatx4 acc[Q][NT];
#pragma unroll
    for (int s = 0; s < Q; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[s][t] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int n = lane & 15, grp = lane >> 4;   // B fragment: output row n, K group grp
    const int wrow = 16 * wave;
    const float outscale = 1.0f / (dscale * cscale);

    load_plane(z_first);
    split_plane();
    write_plane();
    if (z_first + 1 < z_last) load_plane(z_first + 1);
    __syncthreads();
    // B fragments of chunk ch (hi and lo) into buffer set `buf`
    uint4 bh[2][NT], bl[2][NT];
    auto load_b = [&](int ch, int buf) {
        const int k0 = 32 * ch + 8 * grp;
        const int dyi = k0 / WX, xg = (k0 % WX) / 8;
        const bool kval = dyi < Q;
        // the padded tail of K reads a valid row and is masked to zero
        const uint32_t km = kval ? 0xffffffffu : 0u;
        const int row = wrow + n + (kval ? dyi : 0);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint4 h = *reinterpret_cast<const uint4 *>(&sm.dhi[row][16 * t + 8 * xg]);
            bh[buf][t] = make_uint4(h.x & km, h.y & km, h.z & km, h.w & km);
            if constexpr (SPLIT3) {
                const uint4 l = *reinterpret_cast<const uint4 *>(&sm.dlo[row][16 * t + 8 * xg]);
                bl[buf][t] = make_uint4(l.x & km, l.y & km, l.z & km, l.w & km);
            }
        }
    };
    // A fragments of unit u = ch * Q + (dz + R) into ring slot `slot`
    constexpr int PF = 3;   // A-fragment ring: unit u+2 is requested while unit u computes
    uint4 ah[PF], al[PF];
    auto load_a = [&](int u, int slot) {
        const int ch = u / Q, dzi = u % Q;
        ah[slot] = sm.afrag[dzi * NCH + ch][0][lane];
        if constexpr (SPLIT3) al[slot] = sm.afrag[dzi * NCH + ch][1][lane];
    };

    for (int zi = z_first; zi < z_last; ++zi) {
        // software pipeline over the (chunk, dz) units of this plane: the next chunk's B
        // fragments and the A fragments two units ahead are in flight while a unit's
        // 3 x NT MFMAs issue
        load_b(0, 0);
        load_a(0, 0);
        if (S::NU > 1) load_a(1, 1);
#pragma unroll
        for (int u = 0; u < S::NU; ++u) {
            const int ch = u / Q, dzi = u % Q;
            if (dzi == 0 && ch + 1 < NCH) load_b(ch + 1, (ch + 1) & 1);
            if (u + 2 < S::NU) load_a(u + 2, (u + 2) % PF);
            if (u == S::NU / 2 && zi + 1 < z_last) split_plane();   // plane zi + 1
            // keep the requests above this unit's MFMAs (the scheduler would sink them)
            __builtin_amdgcn_sched_barrier(0);
            const uint4 &ahi = ah[u % PF];
            // input plane zi feeds output zi - dz (dz = dzi - R), held in acc[Q - 1 - dzi]
            floatx4 *ac = acc[Q - 1 - dzi];
            const uint4 *bhi = bh[ch & 1];
#pragma unroll
            for (int t = 0; t < NT; ++t) ac[t] = mfma<PREC>(ahi, bhi[t], ac[t]);
            if constexpr (SPLIT3) {
                const uint4 &alo = al[u % PF];
                const uint4 *blo = bl[ch & 1];
#pragma unroll
                for (int t = 0; t < NT; ++t) ac[t] = mfma<PREC>(ahi, blo[t], ac[t]);
#pragma unroll
                for (int t = 0; t < NT; ++t) ac[t] = mfma<PREC>(alo, bhi[t], ac[t]);
            }
        }
        // output plane zi - R is complete (outputs outside [zb, ze) are dropped)
        const int zo = zi - R;
        if (zo >= zb && zo < ze) {
            const int y = yt + wrow + n;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int x = xt + 16 * t + 4 * grp;
                if (y < g.ny && x < g.nx) {
                    float *po = g.out0 + (int64_t)zo * sz + (int64_t)y * sy + x;
                    const floatx4 s = acc[0][t];
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
#pragma unroll
        for (int s = 0; s + 1 < Q; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[s][t] = acc[s + 1][t];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[Q - 1][t] = floatx4{0.f, 0.f, 0.f, 0.f};
        __syncthreads();   // every wave is done with plane zi
        if (zi + 1 < z_last) {
            write_plane();                              // plane zi + 1
            if (zi + 2 < z_last) load_plane(zi + 2);    // requested a whole plane ahead
        }
        __syncthreads();
    }
}

template <int R, int PREC>
int launch_rp(const float *in, float *out, const mms_grid *gd, const float *coeffs, hipStream_t s) {
    constexpr int Q = 2 * R + 1;
    constexpr int NW = MCfg<R>::NW, NT = MCfg<R>::NT;
    constexpr int BXT = 16 * NT, BYT = 16 * NW;
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
    g.ntx = (g.nx + BXT - 1) / BXT;
    g.nty = (g.ny + BYT - 1) / BYT;
    // one block per CU: about 256 blocks, chunks of at most 128 planes
    const int64_t cols = (int64_t)g.ntx * g.nty;
    int zc = (int)((int64_t)g.nz * cols / 256);
    zc = zc < 32 ? 32 : (zc > 128 ? 128 : zc);
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
