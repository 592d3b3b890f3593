// Star-stencil sweep (radius 1..4) for gfx950.
//
// out(p) = sum_{axis a} sum_{k=-r..r} c[a][k+r] in(p + k e_a)   (Sec. I, Fig. 1)
//
// The sweep is bound by HBM: 4 bytes read and 4 written per point.  Each block
// owns a (4*txa) x TY tile of the (x, y) plane (txa <= TX lanes per row, the same
// for every tile of a row: balanced x tiles) and streams a chunk of z planes
// through it:
//  * every lane owns 4 consecutive x (one 16-byte load) of one row and keeps the
//    z planes of those cells in a register queue, so the z-axis terms never
//    touch LDS;
//  * the tile of each plane, with 4 cells of x halo and r rows of y halo, is
//    requested two planes before the plane enters the centre of the queue
//    (together with the neighbouring tiles, which read the same rows as their
//    own cells, so the shared rows are fetched from HBM once and served from
//    L2) and parked in an LDS ring of r+2 planes until it becomes the centre
//    plane; the x and y terms read 16-byte words from it; one barrier per plane;
//  * outputs are written with streaming (non-temporal) stores;
//  * the z loop runs in rounds of the queue length so the queue rotates by
//    renaming registers instead of moving them.
// Block indices are remapped so that each XCD works on one contiguous range of
// tiles and the halo re-reads of neighbouring tiles hit the same L2.
//
// Small grids (at most 2^20 points and fewer z-marching blocks than the GPU has
// CUs, e.g. 64^3): a plane step of the marching kernel costs about one round of
// memory latency, so a block that walks its chunk is latency-bound and most CUs
// idle.  There one lane per 16-byte word reads its 4r + 3 words (the x halo words
// on either side, r rows above and below, r planes in front and behind) straight
// from memory; they are independent, so a sweep takes about one round of (mostly
// L2) latency.  Measured at radius 4 (kernel time, launches replayed from a graph):
// 4.3 against 14.2 us at 64^3 and 9.5 against 13.9 at 96^3; from 128^3 on the
// marching kernel is faster (14.3 against 16.5 us), since the direct reads re-fetch
// every word 4r + 3 times through L2.
#include <utility>

#include "mms_internal.h"

namespace mms {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

struct StarArgs {
    Geom g;
    float c[3][9];  // axis z, y, x; k + r
};

// Two planes of prefetch.  Plane p's words (own word into the register queue,
// halo words into one of two register sets) are requested at iteration p-R-2 and
// parked in the LDS ring at the end of iteration p-R-1, so every load has about
// two iterations to land.  The queue has S = 2r+4 slots (plane p in slot
// (p - zb) mod S, S even so that the halo set index p mod 2 is fixed per phase),
// and the loop runs in rounds of S phases with no branch inside a full round, so
// the wait before parking a plane only covers that plane's loads.
template <int R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) star_kernel(StarArgs a) {
    constexpr int Q = 2 * R + 1;
    constexpr int S = Q + 3;         // queue slots (even)
    constexpr int NR = R + 2;        // LDS ring planes
    constexpr int BY = TY;
    constexpr int LW4 = TX + 2, LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * R * LW4 + 2 * BY;
    constexpr int NHK = (NH + NT - 1) / NT;
    __shared__ float4 ring[NR][LH][LW4];

    const Geom &g = a.g;
    int b = mms_xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % g.ntx;
    b /= g.ntx;
    const int tyi = b % g.nty;
    const int zci = b / g.nty;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    // balanced x tiles: txa <= TX lanes of each row own words, the rest only help
    // with the halo and the barriers
    const int txa = g.txa, lw = txa + 2, bxa = 4 * txa;
    const bool lane_on = tx < txa;
    const int xt = txi * bxa, yt = tyi * BY;
    const int x0 = xt + 4 * tx, y0 = yt + ty;
    const int zb = zci * g.zchunk;
    const int ze = min(zb + g.zchunk, g.nz);
    const int zmax = g.nz + R - 1;      // last plane held in memory (halo >= R)
    const int nx4 = (g.nx + 3) & ~3;
    const int ylim = g.ny + g.H;
    const float *in0 = g.in0;
    const int64_t sy = g.sy, sz = g.sz;

    const bool own_ok = lane_on && (x0 <= nx4) && (y0 < ylim);
    const int64_t own_off = (int64_t)y0 * sy + x0;
    int64_t h_off[NHK];
    int h_lds[NHK];
    bool h_ok[NHK], h_on[NHK];  // h_on: item k is one of this tile's halo words
#pragma unroll
    for (int k = 0; k < NHK; ++k) {
        const int i = tid + k * NT;
        int row, lrow, col4, x;
        if (i < 2 * R * lw) {
            const int hr = i / lw, hc = i % lw;
            row = hr < R ? yt - R + hr : yt + BY + (hr - R);
            lrow = hr < R ? hr : hr + BY;
            col4 = hc;
            x = xt - 4 + 4 * hc;
        } else {
            const int j = i - 2 * R * lw;
            row = yt + j / 2;
            lrow = R + j / 2;
            col4 = (j & 1) ? txa + 1 : 0;
            x = (j & 1) ? xt + bxa : xt - 4;
        }
        h_on[k] = i < 2 * R * lw + 2 * BY;
        h_ok[k] = h_on[k] && (row < ylim) && (x <= nx4);
        h_off[k] = (int64_t)row * sy + x;
        h_lds[k] = lrow * LW4 + col4;
    }
    auto own_load = [&](int z) { return select_load(in0 + (int64_t)z * sz + own_off, own_ok, in0); };
    auto halo_load = [&](int z, float4 *dst) {
        const float *p = in0 + (int64_t)z * sz;
#pragma unroll
        for (int k = 0; k < NHK; ++k) dst[k] = select_load(p + h_off[k], h_ok[k], in0);
    };
    auto ring_store = [&](int z, const float4 &own, const float4 *halo) {
        float4 *t = &ring[z % NR][0][0];
        if (lane_on) t[(R + ty) * LW4 + tx + 1] = own;
#pragma unroll
        for (int k = 0; k < NHK; ++k)
            if (h_on[k]) t[h_lds[k]] = halo[k];
    };

    float4 q[S];
    float4 hs[2][NHK];
    // prologue: planes zb-R .. zb+R+1 into the queue, tiles of zb .. zb+R into the ring,
    // the halo of zb+R+1 into its register set
#pragma unroll
    for (int k = -R; k <= R + 1; ++k) q[(k + S) % S] = own_load(min(zb + k, zmax));
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        float4 h[NHK];
        halo_load(zb + k, h);
        ring_store(zb + k, q[k % S], h);
    }
    halo_load(min(zb + R + 1, zmax), hs[(R + 1) % 2]);
    __syncthreads();

    const float *c = &a.c[0][0];
    float *out0 = g.out0;
    // one phase: plane z = (round start) + ph, slots relative to zb
    auto phase = [&](int z, auto PH) {
        constexpr int ph = decltype(PH)::value;
        // plane z+R+2 is requested now (clamped at the end of the grid; the extra
        // loads of the last planes are never used)
        const int zl = min(z + R + 2, zmax);
        q[(ph + R + 2) % S] = own_load(zl);
        halo_load(zl, hs[(ph + R + 2) % 2]);
        const float4 *t = &ring[z % NR][0][0];
        const float4 ctr = q[ph % S];
        float4 s;
        s.x = c[R] * ctr.x;
        s.y = c[R] * ctr.y;
        s.z = c[R] * ctr.z;
        s.w = c[R] * ctr.w;
#pragma unroll
        for (int k = -R; k <= R; ++k) {
            if (k == 0) continue;
            const float4 v = q[(ph + k + S) % S];
            const float ck = c[R + k];
            s.x = fmaf(ck, v.x, s.x);
            s.y = fmaf(ck, v.y, s.y);
            s.z = fmaf(ck, v.z, s.z);
            s.w = fmaf(ck, v.w, s.w);
        }
#pragma unroll
        for (int k = -R; k <= R; ++k) {
            const float4 v = k == 0 ? ctr : t[(R + ty + k) * LW4 + tx + 1];
            const float ck = c[9 + R + k];
            s.x = fmaf(ck, v.x, s.x);
            s.y = fmaf(ck, v.y, s.y);
            s.z = fmaf(ck, v.z, s.z);
            s.w = fmaf(ck, v.w, s.w);
        }
        const float4 L = t[(R + ty) * LW4 + tx];
        const float4 Rr = t[(R + ty) * LW4 + tx + 2];
        const float w[12] = {L.x, L.y, L.z, L.w, ctr.x, ctr.y, ctr.z, ctr.w, Rr.x, Rr.y, Rr.z, Rr.w};
        float o[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
        for (int k = -R; k <= R; ++k) {
            const float ck = c[18 + R + k];
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = fmaf(ck, w[4 + e + k], o[e]);
        }
        if (lane_on && y0 < g.ny && x0 < g.nx) {
            float *po = out0 + (int64_t)z * sz + own_off;
            if (x0 + 3 < g.nx) {
                const f4v v = {o[0], o[1], o[2], o[3]};
                __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(po));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (x0 + e < g.nx) po[e] = o[e];
            }
        }
        // park plane z+R+1 (requested one iteration ago); its ring slot held plane z-1
        ring_store(z + R + 1, q[(ph + R + 1) % S], hs[(ph + R + 1) % 2]);
        __syncthreads();
    };
    int z = zb;
    for (; z + S <= ze; z += S) {
        [&]<int... P>(std::integer_sequence<int, P...>) {
            (phase(z + P, std::integral_constant<int, P>{}), ...);
        }(std::make_integer_sequence<int, S>{});
    }
    // last partial round
    [&]<int... P>(std::integer_sequence<int, P...>) {
        ((z + P < ze ? (phase(z + P, std::integral_constant<int, P>{}), 0) : 0), ...);
    }(std::make_integer_sequence<int, S>{});
}

template <int R>
__global__ void __launch_bounds__(256) star_direct_kernel(StarArgs a, int64_t nwords, int nxw) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nwords) return;
    const Geom &g = a.g;
    const int xw = (int)(i % nxw);
    const int64_t yz = i / nxw;
    const int y = (int)(yz % g.ny), z = (int)(yz / g.ny);
    const int x0 = 4 * xw;
    // x0 - 4 .. x0 + 7 stay inside the row (halo of at least 4 cells, pitch of at least
    // roundup4(nx) + 2H); rows and planes within r of the interior lie in the halo
    const float *p = g.in0 + (int64_t)z * g.sz + (int64_t)y * g.sy + x0;
    auto ld = [](const float *q) { return *reinterpret_cast<const float4 *>(q); };
    auto at = [](const float4 &v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; };
    const float4 L = ld(p - 4), C = ld(p), Rr = ld(p + 4);
    const float w[12] = {L.x, L.y, L.z, L.w, C.x, C.y, C.z, C.w, Rr.x, Rr.y, Rr.z, Rr.w};
    float4 yu[R], yd[R], zu[R], zd[R];
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        yu[k - 1] = ld(p + k * g.sy);
        yd[k - 1] = ld(p - k * g.sy);
        zu[k - 1] = ld(p + k * g.sz);
        zd[k - 1] = ld(p - k * g.sz);
    }
    const float c0 = a.c[0][R] + a.c[1][R] + a.c[2][R];
    float o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float v = c0 * w[4 + e];
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            const float yv = at(yu[k - 1], e), ydv = at(yd[k - 1], e);
            const float zv = at(zu[k - 1], e), zdv = at(zd[k - 1], e);
            v = fmaf(a.c[2][R + k], w[4 + e + k], v);
            v = fmaf(a.c[2][R - k], w[4 + e - k], v);
            v = fmaf(a.c[1][R + k], yv, v);
            v = fmaf(a.c[1][R - k], ydv, v);
            v = fmaf(a.c[0][R + k], zv, v);
            v = fmaf(a.c[0][R - k], zdv, v);
        }
        o[e] = v;
    }
    float *po = g.out0 + (int64_t)z * g.sz + (int64_t)y * g.sy + x0;
    if (x0 + 3 < g.nx) {
        *reinterpret_cast<float4 *>(po) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (x0 + e < g.nx) po[e] = o[e];
    }
}

template <int R>
int launch_r(const float *in, float *out, const mms_grid *gd, const float *coeffs, hipStream_t s) {
    constexpr int TX = 64, TY = 16;
    StarArgs a{};
    Geom &g = a.g;
    g.H = gd->halo;
    g.in0 = in + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.out0 = out + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    g.txa = balanced_tile_words(g.nx, TX, &g.ntx);
    g.nty = (g.ny + TY - 1) / TY;
    // one block per CU (the LDS ring fills most of a CU's LDS): enough z chunks
    // to give every CU one block, chunks of 8 to 128 planes
    const int zc = pick_zchunk(g.nz, (int64_t)g.ntx * g.nty, 256, 8, 128);
    g.zchunk = zc;
    g.nzc = (g.nz + zc - 1) / zc;
    for (int a_ = 0; a_ < 3; ++a_)
        for (int k = 0; k < 2 * R + 1; ++k) a.c[a_][k] = coeffs[a_ * (2 * R + 1) + k];
    const int64_t nblk = (int64_t)g.ntx * g.nty * g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    if (nblk < 256 && (int64_t)g.nx * g.ny * g.nz <= ((int64_t)1 << 20)) {
        // small grid: fewer marching blocks than CUs
        const int nxw = (g.nx + 3) / 4;
        const int64_t nwords = (int64_t)g.nz * g.ny * nxw;
        const int64_t nb = (nwords + 255) / 256;
        hipLaunchKernelGGL((star_direct_kernel<R>), dim3((unsigned)nb), dim3(256), 0, s, a, nwords,
                           nxw);
        return check_launch("star_direct_kernel");
    }
    hipLaunchKernelGGL((star_kernel<R, TX, TY>), dim3((unsigned)nblk), dim3(TX * TY), 0, s, a);
    return check_launch("star_kernel");
}

}  // namespace

int launch_star(const float *in, float *out, const mms_grid *g, int r, const float *coeffs,
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
