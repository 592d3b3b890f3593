// 2-D star and box sweeps (radius 1..4) over every z-plane of a stack, for gfx950
// (Table I: 2DStarR2 / 2DStarR4, 2DBoxR2 / 2DBoxR3).
//
//   star: out(z,y,x) = sum_k cy[k] in(z, y+k, x) + sum_k cx[k] in(z, y, x+k)
//   box:  out(z,y,x) = sum_{dy,dx} c[dy][dx] in(z, y+dy, x+dx)
//
// Both read 4 bytes and write 4 bytes per point; the star is HBM bound and the
// radius-3 box (49 FMA per point) sits near the FP32-FMA / HBM balance point.
// A block owns a (4 TX) x TY tile of the (x, y) plane and walks a chunk of
// planes.  Each plane's tile, with 4 cells of x halo and r rows of y halo, is
// requested one plane ahead into registers and parked in the other half of a
// double-buffered LDS tile; every lane owns 4 consecutive x (one 16-byte word)
// and reads its 12-cell row windows as three 16-byte LDS words per row.  No
// plane depends on another, so z chunks need no halo planes.  Outputs are
// written with streaming stores; block indices are remapped per XCD as in the
// 3-D sweeps.  The radius-3 box reads its 49 weights from LDS into vector
// registers once (an FMA with a scalar-register operand issues at a lower rate
// on gfx950); at the other radii that costs more occupancy than it gains
// (measured).
#include "mms_internal.h"

namespace mms {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int SH_STAR2D = 0, SH_BOX2D = 1;

struct PlaneArgs {
    Geom g;
    float c[81];  // star: [axis y, x][k + r]; box: [dy + r][dx + r], both with row length 2r+1
};

template <int SHAPE, int R, int TX, int TY, int NY>
__global__ void __launch_bounds__(TX *TY) plane_kernel(PlaneArgs a) {
    constexpr int W = 2 * R + 1;
    constexpr int BX = 4 * TX, BY = TY * NY;
    constexpr int LW4 = TX + 2, LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * R * LW4 + 2 * BY;  // halo words per plane
    constexpr int NHK = (NH + NT - 1) / NT;
    constexpr int NWIN = NY + 2 * R;          // LDS rows one lane reads
    constexpr bool LDSW = SHAPE == SH_BOX2D && R == 3;
    __shared__ float4 tile[2][LH][LW4];
    __shared__ float wl[LDSW ? W * W : 1];

    const Geom &g = a.g;
    int b = mms_xcd_remap(blockIdx.x, gridDim.x);
    const int txi = b % g.ntx;
    b /= g.ntx;
    const int tyi = b % g.nty;
    const int zci = b / g.nty;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int xt = txi * BX, yt = tyi * BY;
    const int x0 = xt + 4 * tx, y0 = yt + ty * NY;
    const int zb = zci * g.zchunk;
    const int ze = min(zb + g.zchunk, g.nz);
    const int nx4 = (g.nx + 3) & ~3;
    const int ylim = g.ny + g.H;
    const int64_t sy = g.sy, sz = g.sz;
    const float *in0 = g.in0;

    bool own_ok[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) own_ok[j] = (x0 <= nx4) && (y0 + j < ylim);
    const int64_t own_off = (int64_t)y0 * sy + x0;
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
        h_lds[k] = lrow * LW4 + col4;
    }
    auto load_plane = [&](int z, float4 *own, float4 *halo) {
        const float *p = in0 + (int64_t)z * sz;
#pragma unroll
        for (int j = 0; j < NY; ++j) own[j] = guarded_load(p + own_off + j * sy, own_ok[j], in0);
#pragma unroll
        for (int k = 0; k < NHK; ++k) halo[k] = guarded_load(p + h_off[k], h_ok[k], in0);
    };
    auto tile_store = [&](int buf, const float4 *own, const float4 *halo) {
        float4 *t = &tile[buf][0][0];
#pragma unroll
        for (int j = 0; j < NY; ++j) t[(R + ty * NY + j) * LW4 + tx + 1] = own[j];
#pragma unroll
        for (int k = 0; k < NHK; ++k)
            if (tid + k * NT < NH) t[h_lds[k]] = halo[k];
    };

    if (LDSW) {
        // published by the first barrier below
        for (int i = tid; i < W * W; i += NT) wl[i] = a.c[i];
    }
    float4 own[NY], hreg[NHK];
    load_plane(zb, own, hreg);
    tile_store(0, own, hreg);
    __syncthreads();

    const float *c = a.c;
    float *out0 = g.out0;
    for (int z = zb; z < ze; ++z) {
        const int buf = (z - zb) & 1;
        const bool more = z + 1 < ze;
        if (more) load_plane(z + 1, own, hreg);
        // this lane's window: LDS rows ty*NY .. ty*NY + NY + 2R - 1 (output row j
        // sits at window row j + R)
        const float4 *t = &tile[buf][ty * NY][tx];
        float o[NY][4];
#pragma unroll
        for (int j = 0; j < NY; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) o[j][e] = 0.f;
        if constexpr (SHAPE == SH_STAR2D) {
            // y terms: the centre word of every window row, read once
#pragma unroll
            for (int i = 0; i < NWIN; ++i) {
                const float4 v = t[i * LW4 + 1];
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const int k = i - R - j;
                    if (k < -R || k > R) continue;
                    const float cy = c[R + k];
                    o[j][0] = fmaf(cy, v.x, o[j][0]);
                    o[j][1] = fmaf(cy, v.y, o[j][1]);
                    o[j][2] = fmaf(cy, v.z, o[j][2]);
                    o[j][3] = fmaf(cy, v.w, o[j][3]);
                }
            }
            // x terms: the 12-cell window of each output row
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const float4 *row = t + (R + j) * LW4;
                const float4 L = row[0], C = row[1], Rr = row[2];
                const float w[12] = {L.x, L.y, L.z, L.w, C.x,  C.y,
                                     C.z, C.w, Rr.x, Rr.y, Rr.z, Rr.w};
#pragma unroll
                for (int k = -R; k <= R; ++k) {
                    const float cx = c[W + R + k];
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[j][e] = fmaf(cx, w[4 + e + k], o[j][e]);
                }
            }
        } else {
            // every window row feeds the outputs it is within r rows of
#pragma unroll
            for (int i = 0; i < NWIN; ++i) {
                const float4 *row = t + i * LW4;
                const float4 L = row[0], C = row[1], Rr = row[2];
                const float w[12] = {L.x, L.y, L.z, L.w, C.x,  C.y,
                                     C.z, C.w, Rr.x, Rr.y, Rr.z, Rr.w};
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    const int dy = i - R - j;
                    if (dy < -R || dy > R) continue;
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        const float cc = LDSW ? wl[(dy + R) * W + dx + R] : c[(dy + R) * W + dx + R];
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[j][e] = fmaf(cc, w[4 + e + dx], o[j][e]);
                    }
                }
            }
        }
        if (x0 < g.nx) {
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                if (y0 + j >= g.ny) break;
                float *po = out0 + (int64_t)z * sz + own_off + j * sy;
                if (x0 + 3 < g.nx) {
                    const f4v v = {o[j][0], o[j][1], o[j][2], o[j][3]};
                    __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(po));
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (x0 + e < g.nx) po[e] = o[j][e];
                }
            }
        }
        if (more) tile_store(buf ^ 1, own, hreg);
        __syncthreads();
    }
}

// Launch shapes, measured at 512^3: one output row per lane and 256 x 16 tiles
// for the short stencils; the wider ones give each lane NY output rows, so every
// LDS row window it reads feeds up to NY outputs (the radius-3 and -4 boxes run
// 256 x 16 tiles of 256 threads, three blocks per CU).
template <int SHAPE, int R>
struct PlaneCfg {
    static constexpr bool WIDE = SHAPE == SH_STAR2D ? R >= 3 : R >= 2;
    static constexpr int TX = 64;
    static constexpr int TY = !WIDE ? 16 : SHAPE == SH_STAR2D ? 8 : R == 2 ? 16 : 4;
    static constexpr int NY = !WIDE ? 1 : SHAPE == SH_STAR2D ? 4 : R == 2 ? 2 : 4;
};

template <int SHAPE, int R>
int launch_plane_r(const float *in, float *out, const mms_grid *gd, const float *coeffs,
                   hipStream_t s) {
    constexpr int PTX = PlaneCfg<SHAPE, R>::TX, PTY = PlaneCfg<SHAPE, R>::TY;
    constexpr int PNY = PlaneCfg<SHAPE, R>::NY;
    const void *kern = reinterpret_cast<const void *>(&plane_kernel<SHAPE, R, PTX, PTY, PNY>);
    PlaneArgs a{};
    Geom &g = a.g;
    g.H = gd->halo;
    g.in0 = in + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.out0 = out + (int64_t)g.H * (gd->sz + gd->sy + 1);
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    g.ntx = (g.nx + 4 * PTX - 1) / (4 * PTX);
    g.nty = (g.ny + PTY * PNY - 1) / (PTY * PNY);
    // planes are independent, so the only per-block overhead is the first
    // plane's load
    const int zc = pick_zchunk_rounds(g.nz, (int64_t)g.ntx * g.nty,
                                      launch_slots(kern, PTX * PTY), 1, 128, 1);
    g.zchunk = zc;
    g.nzc = (g.nz + zc - 1) / zc;
    const int n = SHAPE == SH_STAR2D ? 2 * (2 * R + 1) : (2 * R + 1) * (2 * R + 1);
    for (int i = 0; i < n; ++i) a.c[i] = coeffs[i];
    const int64_t nblk = (int64_t)g.ntx * g.nty * g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    hipLaunchKernelGGL((plane_kernel<SHAPE, R, PTX, PTY, PNY>), dim3((unsigned)nblk),
                       dim3(PTX * PTY), 0, s, a);
    return check_launch("plane_kernel");
}

template <int SHAPE>
int launch_plane_shape(const float *in, float *out, const mms_grid *g, int r,
                       const float *coeffs, hipStream_t s) {
    switch (r) {
        case 1: return launch_plane_r<SHAPE, 1>(in, out, g, coeffs, s);
        case 2: return launch_plane_r<SHAPE, 2>(in, out, g, coeffs, s);
        case 3: return launch_plane_r<SHAPE, 3>(in, out, g, coeffs, s);
        case 4: return launch_plane_r<SHAPE, 4>(in, out, g, coeffs, s);
        default: return MMS_EUNSUPPORTED;
    }
}

}  // namespace

int launch_plane2d(const float *in, float *out, const mms_grid *g, int shape, int r,
                   const float *coeffs, hipStream_t s) {
    if (shape == MMS_STAR2D) return launch_plane_shape<SH_STAR2D>(in, out, g, r, coeffs, s);
    if (shape == MMS_BOX2D) return launch_plane_shape<SH_BOX2D>(in, out, g, r, coeffs, s);
    return MMS_EUNSUPPORTED;
}

}  // namespace mms
