// Box-stencil sweep on the vector ALUs, FP32 FMA (radius 1..4).
//
// out(p) = sum_{dz,dy,dx in [-r,r]} c[dz][dy][dx] in(p + (dz,dy,dx))   (Sec. I)
//
// With (2r+1)^3 FMAs per point the box is bound by the FP32 FMA rate.  The
// kernel follows the box decomposition of Sec. IV-C: the box is (2r+1)^2
// one-dimensional x stencils, one per (dz, dy) pair, and each loaded input row
// feeds all of them before it is dropped:
//  * a block owns a (4*TX) x (TY*rows) tile and streams z; one input plane of the tile
//    (plus 4 cells of x halo and r rows of y halo) sits in LDS at a time,
//    double-buffered, one barrier per plane;
//  * each lane owns 4 consecutive x of one row (of two rows from radius 2 on)
//    and keeps 2r+1 partial sums per row for the 2r+1 output planes the current
//    input plane feeds (input plane z' contributes to output z'-dz through
//    weights c[dz]); the oldest sum is complete after each plane and the window
//    shifts by one;
//  * a lane reads 12 consecutive cells of one input row (three 16-byte LDS
//    words) and applies all (2r+1) x (2r+1) weights of that dy to them, so LDS
//    traffic is 3 words per (2r+1)^2 * 4 FMAs.
//  * the next input plane is requested one plane ahead, two planes ahead at
//    radius 1, where one plane's FMAs are too few to cover the latency.  From
//    radius 2 on the requests go straight from memory into LDS (no staging
//    registers, no LDS stores); at radius 1 they pass through registers.
// Where the weights come from sets the FMA rate on gfx950.  The SIMD reaches its
// FP32 rate only by issuing FMAs of two waves in the same cycle, which an FMA with
// a scalar-register operand, or with all three operands in one VGPR bank, does
// not do: with scalar-register weights the sweep runs at about 75 TFLOP/s
// chip-wide, with all operands in vector registers at about 110-130.  From
// radius 2 on the weights are therefore copied once into LDS, laid out
// [dy][dz][dx] with rows padded to 12 floats, and every lane reads the 2r+1
// weights of one (dy, dz) row as broadcast LDS loads into vector registers; each
// is used by 4 * rows FMAs.  At radius 1 the sweep is bound by HBM, and the
// weights stay in scalar registers, loaded from the kernel-argument segment.
#include <type_traits>

#include "mms_internal.h"

namespace mms {
namespace {

struct BoxArgs {
    Geom g;
    float c[729];  // [dz][dy][dx] for radius r, (2r+1)^3 used
};

// One 16-byte word per lane from memory straight into LDS: lane l's word lands at
// dst + l, where dst must be the same for the whole wave.  Completion is counted by
// vmcnt (not lgkmcnt) and makes the word visible to this lane's LDS reads; other
// lanes see it after a barrier.
__device__ __forceinline__ void load_lds16(const float *src, float4 *dst) {
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

// R: radius; TX x TY lanes, each with 4 x-cells of NYL rows; LDSW: weights in LDS
// and the plane tile loaded straight into LDS (radius 2 on); ONEPATH: one plane
// body with a per-dz test instead of a tested and an untested copy; DYU: dy loop
// unrolled; MINW: waves per SIMD the register allocation must leave room for.
template <int R, int TX, int TY, bool LDSW, int NYL, bool ONEPATH, bool DYU, int MINW>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(MINW)))
box_valu_kernel(BoxArgs a) {
    constexpr int W = 2 * R + 1;
    constexpr int BX = 4 * TX;
    constexpr int BY = TY * NYL;              // NYL output rows per lane
    constexpr int LW4 = TX + 2;
    constexpr int LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    constexpr int NL = LW4 * LH;              // float4 per plane tile
    constexpr int NLK = (NL + NT - 1) / NT;
    constexpr int CP = 12;                    // padded weights per (dy, dz) row in LDS
    constexpr bool DIRECT = LDSW;
    // direct loads write whole waves of words: the buffer is padded to NLK * NT
    constexpr int NLP = DIRECT ? NLK * NT : NL;
    // two arrays rather than one [2][...]: with each step's buffer fixed at compile
    // time the compiler can tell the words being read from the words that direct
    // loads are filling, and adds no wait for those loads before the reads
    __shared__ float4 tile0[NLP];
    __shared__ float4 tile1[NLP];
    __shared__ __attribute__((aligned(16))) float wl[LDSW ? W : 1][LDSW ? W : 1][CP];

    const Geom &g = a.g;
    int b = mms_xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % g.ntx;
    b /= g.ntx;
    const int tyi = b % g.nty;
    const int zci = b / g.nty;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int xt = txi * BX, yt = tyi * BY;
    const int x0 = xt + 4 * tx, y = yt + NYL * ty;   // the lane's rows: y .. y + NYL - 1
    const int zb = zci * g.zchunk;
    const int ze = min(zb + g.zchunk, g.nz);
    const int nx4 = (g.nx + 3) & ~3;
    const int ylim = g.ny + g.H;
    const int64_t sy = g.sy, sz = g.sz;

    if (LDSW) {
        // [dz][dy][dx] -> [dy][dz][dx]; the first barrier below publishes it
        for (int i = tid; i < W * W * W; i += NT) wl[(i / W) % W][i / (W * W)][i % W] = a.c[i];
    }
    // cooperative tile load: item i -> (row, col4) of the tile.  Words outside the
    // array (rows at or beyond ny + H, columns beyond nx4) feed only outputs that are
    // never stored: staged loads zero them, direct loads read the tile origin instead.
    constexpr int NKS = DIRECT ? 1 : NLK;     // staged items per lane
    constexpr int NKD = DIRECT ? NLK : 1;     // direct items per lane
    int64_t l_off[NKS];
    bool l_ok[NKS];
    uint32_t d_off[NKD];                      // from the tile origin (row yt - R, column xt - 4)
#pragma unroll
    for (int k = 0; k < NLK; ++k) {
        const int i = tid + k * NT;
        const int row = i / LW4, col = i % LW4;
        const int yy = yt - R + row, xx = xt - 4 + 4 * col;
        const bool ok = (i < NL) && (yy < ylim) && (xx <= nx4);
        if constexpr (DIRECT) {
            d_off[k] = ok ? (uint32_t)row * (uint32_t)sy + 4u * (uint32_t)col : 0u;
        } else {
            l_ok[k] = ok;
            l_off[k] = (int64_t)yy * sy + xx;
        }
    }
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    auto tbuf = [&](auto B) { return decltype(B)::value ? tile1 : tile0; };
    auto direct_plane = [&](int z, auto B) {
        const float *p = g.in0 + (int64_t)z * sz + (int64_t)(yt - R) * sy + (xt - 4);
        float4 *dst = tbuf(B) + __builtin_amdgcn_readfirstlane(tid & ~63);
#pragma unroll
        for (int k = 0; k < NKD; ++k) load_lds16(p + d_off[k], dst + k * NT);
    };
    // staged input planes in flight (radius 1): two planes of requests outstanding,
    // since one plane's work does not cover the latency of the next plane's loads
    constexpr int NSB = DIRECT ? 1 : 2;
    float4 stage[NSB][NKS];
    auto load_plane = [&](int z, auto S) {
        const float *p = g.in0 + (int64_t)z * sz;
#pragma unroll
        for (int k = 0; k < NKS; ++k)
            stage[decltype(S)::value][k] = guarded_load(p + l_off[k], l_ok[k], g.in0);
    };
    auto store_plane = [&](auto B, auto S) {
        float4 *t = tbuf(B);
#pragma unroll
        for (int k = 0; k < NKS; ++k)
            if (tid + k * NT < NL) t[tid + k * NT] = stage[decltype(S)::value][k];
    };

    float acc[W][NYL][4];
#pragma unroll
    for (int s = 0; s < W; ++s)
#pragma unroll
        for (int j = 0; j < NYL; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[s][j][e] = 0.f;

    const int z_first = zb - R, z_last = ze + R;  // input planes [z_first, z_last)
    if constexpr (DIRECT) {
        direct_plane(z_first, S0{});
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    } else {
        load_plane(z_first, S0{});
        store_plane(S0{}, S0{});
        if (z_first + 1 < z_last) load_plane(z_first + 1, S1{});
    }
    __syncthreads();
    // one input plane zi, held in buffer B.  Staged (radius 1): stage[B] held plane zi
    // and receives plane zi + 2, stage[B ^ 1] holds plane zi + 1.
    auto step = [&](int zi, auto B) {
        constexpr int sb = decltype(B)::value;
        using BN = std::integral_constant<int, sb ^ 1>;
        const bool more = zi + 1 < z_last;
        if constexpr (DIRECT) {
            if (more) direct_plane(zi + 1, BN{});
        } else {
            if (zi + 2 < z_last) load_plane(zi + 2, B);
        }
        const float4 *t = tbuf(B);
        // Input planes within r of the chunk's ends feed some output planes outside
        // it; those (dz) terms are skipped there.
        auto plane = [&](auto checked) {
            // dy stays a loop with scalar-register weights: unrolled, all (2r+1)^3
            // would be hoisted into scalar registers and spill to vector-register
            // lanes.
            constexpr int NDY = DYU ? 2 * R + 1 : 1;
#pragma unroll NDY
            for (int dy = -R; dy <= R; ++dy) {
                // input rows y + j + dy (j < NYL): each weight below feeds 4 NYL FMAs
                float w[NYL][12];
#pragma unroll
                for (int j = 0; j < NYL; ++j) {
                    const float4 *row = t + (NYL * ty + j + R + dy) * LW4;
                    const float4 L = row[tx], C = row[tx + 1], Rr = row[tx + 2];
                    const float v[12] = {L.x, L.y, L.z, L.w, C.x, C.y, C.z, C.w,
                                         Rr.x, Rr.y, Rr.z, Rr.w};
#pragma unroll
                    for (int i = 0; i < 12; ++i) w[j][i] = v[i];
                }
                const float *cdy = a.c + (dy + R) * W;
#pragma unroll
                for (int dz = -R; dz <= R; ++dz) {
                    if (decltype(checked)::value) {
                        const int zo = zi - dz;  // output plane fed through c[dz]
                        if (zo < zb || zo >= ze) continue;
                    }
                    const float *cc = LDSW ? &wl[dy + R][dz + R][0] : cdy + (dz + R) * W * W;
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        const float ck = cc[dx + R];
#pragma unroll
                        for (int j = 0; j < NYL; ++j)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                acc[R - dz][j][e] = fmaf(ck, w[j][4 + e + dx], acc[R - dz][j][e]);
                    }
                }
            }
        };
        // With two copies of the plane body (untested for the planes that feed all
        // 2r+1 accumulators, tested near the chunk's ends) the compiler keeps the
        // accumulators of each copy in registers of their own where both are large.
        if (ONEPATH || !(zi >= zb + R && zi < ze - R))
            plane(std::true_type{});
        else
            plane(std::false_type{});
        if constexpr (DIRECT) {
            // the next plane is in LDS once this lane's requests are done; the barrier
            // publishes every lane's words and ends all reads of this plane.  The
            // output stores come after it, so the wait does not cover them.
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
        }
        // output plane zi - R is complete
        const int zo = zi - R;
#pragma unroll
        for (int j = 0; j < NYL; ++j) {
            if (zo >= zb && y + j < g.ny && x0 < g.nx) {
                float *po = g.out0 + (int64_t)zo * sz + (int64_t)(y + j) * sy + x0;
                if (x0 + 3 < g.nx) {
                    *reinterpret_cast<float4 *>(po) =
                        make_float4(acc[0][j][0], acc[0][j][1], acc[0][j][2], acc[0][j][3]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (x0 + e < g.nx) po[e] = acc[0][j][e];
                }
            }
        }
#pragma unroll
        for (int s = 0; s + 1 < W; ++s)
#pragma unroll
            for (int j = 0; j < NYL; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[s][j][e] = acc[s + 1][j][e];
#pragma unroll
        for (int j = 0; j < NYL; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[W - 1][j][e] = 0.f;
        if constexpr (!DIRECT) {
            if (more) store_plane(BN{}, BN{});
            __syncthreads();
        }
    };
    // the buffer (and staging slot) is a compile-time index: planes in pairs
    int zi = z_first;
    for (; zi + 1 < z_last; zi += 2) {
        step(zi, S0{});
        step(zi + 1, S1{});
    }
    if (zi < z_last) step(zi, S0{});
}

// Per-radius shape, measured at 512^3 (warm clocks, outputs bit-identical between
// shapes; Gpoints/s):
//  * two output rows per lane from radius 2 on: each weight read from LDS feeds 8
//    FMAs and each plane's fixed work (barrier, accumulator shift, stores) is shared
//    by twice the outputs (radius 3: 109 -> 117);
//  * radius 2 (128 VGPRs, 4 waves per SIMD): dy unrolled, two plane bodies, 314
//    against 304 with one body;
//  * radius 3: dy unrolled and one plane body, held to 128 VGPRs for 4 waves per SIMD
//    (32 bytes per lane spilled): 133 against 128 at 134 VGPRs and 3 waves, 119 with
//    two bodies (151 VGPRs) and 117 with dy as a loop (101 VGPRs, 4 waves per SIMD);
//  * radius 4: dy as a loop and one plane body (128 VGPRs, 4 waves per SIMD),
//    67.6-68.9 against 66.3-67.2 for one row per lane; with two bodies, or dy
//    unrolled, two rows need 170-220 VGPRs;
//  * radius 1 is bound by HBM: wide 256 x 16 tiles (1024 threads) cut the halo
//    share (576 against 513 with 64 x 16 tiles).
// Eight x-cells per lane (half the weight reads per FMA) measured slower at radius
// 2 and 3 (270, 103) and equal at radius 4.
template <int R>
struct BoxShape {
    static constexpr int TX = R == 1 ? 64 : 16, TY = 16;
    static constexpr int NYL = R >= 2 ? 2 : 1;
    static constexpr bool ONEPATH = R >= 3;
    static constexpr bool DYU = R == 2 || R == 3;
    static constexpr int MINW = R == 3 ? 4 : 1;
};

template <int R>
int launch_r(const float *in, float *out, const mms_grid *gd, const float *coeffs, hipStream_t s) {
    using S = BoxShape<R>;
    constexpr int TX = S::TX, TY = S::TY, NYL = S::NYL;
    constexpr int W = 2 * R + 1;
    constexpr bool LDSW = R >= 2;
    BoxArgs a{};
    Geom &g = a.g;
    g.H = gd->halo;
    g.in0 = in + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.out0 = out + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    // direct loads address the plane tile with 32-bit offsets from its origin
    if (LDSW && (int64_t)(TY * NYL + 2 * R + 1) * g.sy >= ((int64_t)1 << 32)) {
        set_last_error("box sweep: grid rows too long for 32-bit tile offsets "
                       "(the row pitch must be below 2^32 / (rows of a tile + 1))");
        return MMS_EUNSUPPORTED;
    }
    g.ntx = (g.nx + 4 * TX - 1) / (4 * TX);
    g.nty = (g.ny + TY * NYL - 1) / (TY * NYL);
    const int64_t cols = (int64_t)g.ntx * g.nty;
    // about 4096 blocks of one output row per lane (2048 of two); a round model of the
    // resident blocks (as in the 2-D sweeps) measured no faster at 512^3
    int zc = (int)((int64_t)g.nz * cols * NYL / 4096);
    zc = zc < 16 ? 16 : zc;
    // radius 1 is bound by HBM: long chunks cut the re-read halo planes
    // (measured at 512^3: 512 Gpoints/s at 128 planes against 441 at 32)
    if (R == 1) zc = 128;
    g.zchunk = zc;
    g.nzc = (g.nz + zc - 1) / zc;
    for (int i = 0; i < W * W * W; ++i) a.c[i] = coeffs[i];
    const int64_t nblk = (int64_t)g.ntx * g.nty * g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    hipLaunchKernelGGL((box_valu_kernel<R, TX, TY, LDSW, NYL, S::ONEPATH, S::DYU, S::MINW>),
                       dim3((unsigned)nblk), dim3(TX * TY), 0, s, a);
    return check_launch("box_valu_kernel");
}

}  // namespace

int launch_box_valu(const float *in, float *out, const mms_grid *g, int r, const float *coeffs,
                    hipStream_t s) {
    switch (r) {
        case 1: return launch_r<1>(in, out, g, coeffs, s);
        case 2: return launch_r<2>(in, out, g, coeffs, s);
        case 3: return launch_r<3>(in, out, g, coeffs, s);
        case 4: return launch_r<4>(in, out, g, coeffs, s);
        default: return MMS_EUNSUPPORTED;
    }
}

}  // namespace mms
