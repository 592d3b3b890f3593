// Star-stencil sweep (radius 1..4) for gfx950.
//
// out(p) = sum_{axis a} sum_{k=-r..r} c[a][k+r] in(p + k e_a)   (Sec. I, Fig. 1)
//
// The sweep is bound by HBM: 4 bytes read and 4 written per point.  Each block
// owns a (4*TX) x (TY*NY) tile of the (x, y) plane and streams a chunk of z
// planes through it:
//  * every lane owns 4 consecutive x (one 16-byte load) in NY rows and keeps
//    the 2r+1 z planes of those cells in a register queue, so the z-axis terms
//    never touch LDS;
//  * the tile of each plane, with 4 cells of x halo and r rows of y halo, is
//    requested when the plane enters the queue (together with the neighbouring
//    tiles, which read the same rows as their own cells, so the shared rows are
//    fetched from HBM once and served from L2) and parked in an LDS ring of
//    r+2 planes until it becomes the centre plane; the x and y terms read
//    16-byte words from it; one barrier per plane;
//  * outputs are written with streaming (non-temporal) stores;
//  * the z loop is unrolled by the queue length so the queue rotates by
//    renaming registers instead of moving them.
// Block indices are remapped so that each XCD works on one contiguous range of
// tiles and the halo re-reads of neighbouring tiles hit the same L2.
#include "mms_internal.h"

namespace mms {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

struct StarArgs {
    Geom g;
    float c[3][9];  // axis z, y, x; k + r
};

template <int R, int TX, int TY, int NY>
__global__ void __launch_bounds__(TX *TY) star_kernel(StarArgs a) {
    constexpr int Q = 2 * R + 1;     // planes in the register queue
    constexpr int NR = R + 2;        // planes in the LDS ring: z .. z+R+1
    constexpr int BX = 4 * TX;       // tile width in cells
    constexpr int BY = TY * NY;      // tile height in rows
    constexpr int LW4 = TX + 2;      // LDS row in float4 (one float4 of halo each side)
    constexpr int LH = BY + 2 * R;   // LDS rows
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * R * LW4 + 2 * BY;  // halo float4 per plane
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
    const int xt = txi * BX;            // first cell of the tile
    const int x0 = xt + 4 * tx;         // first of this lane's 4 cells
    const int yt = tyi * BY;
    const int y0 = yt + ty * NY;
    const int zb = zci * g.zchunk;
    const int ze = min(zb + g.zchunk, g.nz);
    const int nx4 = (g.nx + 3) & ~3;
    const int ylim = g.ny + g.H;        // rows below this exist in memory

    const float *in0 = g.in0;
    const int64_t sy = g.sy, sz = g.sz;

    // this lane's rows and whether their 16-byte words exist in memory
    bool own_ok[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) own_ok[j] = (x0 <= nx4) && (y0 + j < ylim);

    // halo items of one plane handled by this lane: memory offset within a plane and LDS slot
    int64_t h_off[NHK];
    int h_lds[NHK];
    bool h_ok[NHK];
#pragma unroll
    for (int k = 0; k < NHK; ++k) {
        const int i = tid + k * NT;
        int row, lrow, col4, x;
        if (i < 2 * R * LW4) {
            const int hr = i / LW4, hc = i % LW4;
            row = hr < R ? yt - R + hr : yt + BY + (hr - R);
            lrow = hr < R ? hr : hr + BY;
            col4 = hc;
            x = xt - 4 + 4 * hc;
        } else {
            const int j = i - 2 * R * LW4;
            row = yt + j / 2;
            lrow = R + j / 2;
            col4 = (j & 1) ? LW4 - 1 : 0;
            x = (j & 1) ? xt + BX : xt - 4;
        }
        h_ok[k] = (i < NH) && (row < ylim) && (x <= nx4);
        h_off[k] = (int64_t)row * sy + x;
        h_lds[k] = (lrow * LW4 + col4);
    }

    auto own_load = [&](int z, float4 *dst) {
        const float *p = in0 + (int64_t)z * sz + (int64_t)y0 * sy + x0;
#pragma unroll
        for (int j = 0; j < NY; ++j) dst[j] = guarded_load(p + j * sy, own_ok[j], in0);
    };
    auto halo_load = [&](int z, float4 *dst) {
        const float *p = in0 + (int64_t)z * sz;
#pragma unroll
        for (int k = 0; k < NHK; ++k) dst[k] = guarded_load(p + h_off[k], h_ok[k], in0);
    };
    auto ring_store = [&](int slot, const float4 *own, const float4 *halo) {
        float4 *t = &ring[slot][0][0];
#pragma unroll
        for (int j = 0; j < NY; ++j) t[(R + ty * NY + j) * LW4 + tx + 1] = own[j];
#pragma unroll
        for (int k = 0; k < NHK; ++k)
            if (tid + k * NT < NH) t[h_lds[k]] = halo[k];
    };

    float4 q[Q][NY];
    float4 hreg[NHK];
    // prologue: planes zb-R .. zb+R into the queue; the tiles of planes zb .. zb+R
    // (own cells and halo) into the LDS ring
#pragma unroll
    for (int i = 0; i < Q; ++i) own_load(zb - R + i, q[i]);
#pragma unroll
    for (int i = 0; i <= R; ++i) {
        halo_load(zb + i, hreg);
        ring_store((zb + i) % NR, q[R + i], hreg);
    }
    __syncthreads();

    const float *c = &a.c[0][0];
    float *out0 = g.out0;
    for (int z = zb; z < ze;) {
#pragma unroll
        for (int ph = 0; ph < Q; ++ph) {
            if (z < ze) {
                // the tile of plane z+R+1 is requested now, alongside the neighbouring
                // tiles that read the same rows as their own cells, and parked in the
                // ring until it becomes the centre plane
                const bool more = z + 1 < ze;
                float4 nq[NY];
                if (more) {
                    own_load(z + R + 1, nq);
                    halo_load(z + R + 1, hreg);
                }
                const float4 *t = &ring[z % NR][0][0];
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const float4 ctr = q[(ph + R) % Q][j];
                    // z axis from the register queue (slot of plane z+k is (ph+R+k) % Q)
                    float4 s;
                    s.x = c[0 * 9 + R] * ctr.x;
                    s.y = c[0 * 9 + R] * ctr.y;
                    s.z = c[0 * 9 + R] * ctr.z;
                    s.w = c[0 * 9 + R] * ctr.w;
#pragma unroll
                    for (int k = -R; k <= R; ++k) {
                        if (k == 0) continue;
                        const float4 v = q[(ph + R + k + Q) % Q][j];
                        const float ck = c[0 * 9 + R + k];
                        s.x = fmaf(ck, v.x, s.x);
                        s.y = fmaf(ck, v.y, s.y);
                        s.z = fmaf(ck, v.z, s.z);
                        s.w = fmaf(ck, v.w, s.w);
                    }
                    // y axis: rows from LDS, own rows from registers
#pragma unroll
                    for (int k = -R; k <= R; ++k) {
                        const int jj = j + k;
                        const float4 v = (jj >= 0 && jj < NY)
                                             ? q[(ph + R) % Q][(jj >= 0 && jj < NY) ? jj : 0]
                                             : t[(R + ty * NY + jj) * LW4 + tx + 1];
                        const float ck = c[1 * 9 + R + k];
                        s.x = fmaf(ck, v.x, s.x);
                        s.y = fmaf(ck, v.y, s.y);
                        s.z = fmaf(ck, v.z, s.z);
                        s.w = fmaf(ck, v.w, s.w);
                    }
                    // x axis: left and right neighbours' words from LDS
                    const float4 L = t[(R + ty * NY + j) * LW4 + tx];
                    const float4 Rr = t[(R + ty * NY + j) * LW4 + tx + 2];
                    const float w[12] = {L.x,   L.y,   L.z,   L.w,  ctr.x, ctr.y,
                                         ctr.z, ctr.w, Rr.x, Rr.y, Rr.z,  Rr.w};
                    float o[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
                    for (int k = -R; k <= R; ++k) {
                        const float ck = c[2 * 9 + R + k];
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[e] = fmaf(ck, w[4 + e + k], o[e]);
                    }
                    const int y = y0 + j;
                    if (y < g.ny && x0 < g.nx) {
                        float *po = out0 + (int64_t)z * sz + (int64_t)y * sy + x0;
                        if (x0 + 3 < g.nx) {
                            // streaming store: the output is not read again by this sweep
                            const f4v v = {o[0], o[1], o[2], o[3]};
                            __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(po));
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (x0 + e < g.nx) po[e] = o[e];
                        }
                    }
                }
                if (more) {
                    ring_store((z + R + 1) % NR, nq, hreg);
#pragma unroll
                    for (int j = 0; j < NY; ++j) q[ph][j] = nq[j];
                }
                __syncthreads();
                ++z;
            }
        }
    }
}

template <int R>
int launch_r(const float *in, float *out, const mms_grid *gd, const float *coeffs, hipStream_t s) {
    constexpr int TX = 64, TY = 16, NY = 1;
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
    g.ntx = (g.nx + 4 * TX - 1) / (4 * TX);
    g.nty = (g.ny + TY * NY - 1) / (TY * NY);
    int zc = zchunk_override(MMS_STAR, MMS_FP32);
    if (zc <= 0) {
        // one block per CU (the LDS ring fills most of a CU's LDS): enough z chunks
        // to give every CU one block, chunks of 8 to 128 planes
        zc = pick_zchunk(g.nz, (int64_t)g.ntx * g.nty, 256, 8, 128);
    }
    g.zchunk = zc;
    g.nzc = (g.nz + zc - 1) / zc;
    for (int a_ = 0; a_ < 3; ++a_)
        for (int k = 0; k < 2 * R + 1; ++k) a.c[a_][k] = coeffs[a_ * (2 * R + 1) + k];
    const int64_t nblk = (int64_t)g.ntx * g.nty * g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    hipLaunchKernelGGL((star_kernel<R, TX, TY, NY>), dim3((unsigned)nblk), dim3(TX * TY), 0, s, a);
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
