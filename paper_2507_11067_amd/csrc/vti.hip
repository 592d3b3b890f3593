// Fused pseudo-acoustic VTI step (gfx950): the two-field anisotropic update that
// RTM in VTI media runs (Sec. II-A, Sec. V-F), in the well-posed form the TTI
// system of Sec. II-A takes for zero tilt and zero shear velocity:
//   H^{n+1} = G (2 H^n - G H^{n-1} + C2 (a Sxy H^n + b Szz V^n)) + dt^2 f^n delta_src
//   V^{n+1} = G (2 V^n - G V^{n-1} + C2 (b Sxy H^n +   Szz V^n)) + dt^2 f^n delta_src
// a = 1 + 2 epsilon and b = sqrt(1 + 2 delta) are fields; Sxy = Sxx + Syy and Szz
// are the axis parts of the star.  Only H needs x and y neighbours and only V
// needs z neighbours, so (following the paper's decomposition of complex kernels
// into one-dimensional stencils on small blocks, Sec. IV-G):
//  * H travels through a double-buffered LDS tile (x/y halo), requested one plane
//    ahead together with the neighbouring tiles;
//  * V travels through a register queue of 2r+1 planes (z terms only);
//  * the five point-wise operands (H^{n-1}, V^{n-1}, C2, a, b) are requested one
//    plane ahead; both outputs are written with streaming stores.
#include "mms_internal.h"

namespace mms {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

struct VtiArgs {
    Geom g;
    float c[9];            // per-axis weights, k + r (symmetric)
    const float *hc, *vc;  // H^n, V^n
    const float *hp, *vp;  // H^{n-1}, V^{n-1}
    const float *c2, *fa, *fb;
    float c2s;
    float *hn, *vn;        // outputs
    float *traces;         // [ny][nx] plane of level n, or NULL
    const float *src;
    int src_z, src_y, src_x;
    int sponge_w;
    float sponge_a;
    int faces;
};

template <int R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) vti_kernel(VtiArgs a) {
    constexpr int Q = 2 * R + 1;
    constexpr int BY = TY;
    constexpr int LW4 = TX + 2, LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * R * LW4 + 2 * BY;
    constexpr int NHK = (NH + NT - 1) / NT;
    __shared__ float4 tile[2][LH][LW4];

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
    const int x0 = xt + 4 * tx, y = yt + ty;
    const int zb = zci * g.zchunk;
    const int ze = min(zb + g.zchunk, g.nz);
    const int nx4 = (g.nx + 3) & ~3;
    const int ylim = g.ny + g.H;
    const int64_t sy = g.sy, sz = g.sz;
    const int W = a.sponge_w;
    const float sa = a.sponge_a;

    const bool own_ok = lane_on && (x0 <= nx4) && (y < ylim);
    const int64_t own_off = (int64_t)y * sy + x0;
    float gown[4];
    {
        const float gy = gaxis(y, g.ny, W, sa, a.faces & 4, a.faces & 8);
#pragma unroll
        for (int e = 0; e < 4; ++e) gown[e] = gy * gaxis(x0 + e, g.nx, W, sa, a.faces & 1, a.faces & 2);
    }
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
    auto ld = [&](const float *base, int z, int64_t off, bool ok) -> float4 {
        return guarded_load(base + (int64_t)z * sz + off, ok, a.c2);
    };
    auto tile_store = [&](int buf, const float4 &own, const float4 *halo) {
        float4 *t = &tile[buf][0][0];
        if (lane_on) t[(R + ty) * LW4 + tx + 1] = own;
#pragma unroll
        for (int k = 0; k < NHK; ++k)
            if (h_on[k]) t[h_lds[k]] = halo[k];
    };

    // point-wise operands of a plane: H^{n-1}, V^{n-1}, C2, a, b
    struct Pw {
        float4 hp, vp, c2, fa, fb;
    };
    auto load_pw = [&](int z) {
        Pw p;
        p.hp = ld(a.hp, z, own_off, own_ok);
        p.vp = ld(a.vp, z, own_off, own_ok);
        p.c2 = ld(a.c2, z, own_off, own_ok);
        p.fa = ld(a.fa, z, own_off, own_ok);
        p.fb = ld(a.fb, z, own_off, own_ok);
        return p;
    };

    float4 q[Q];          // V at planes z-R .. z+R
    float4 hreg[NHK];
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = ld(a.vc, zb - R + i, own_off, own_ok);
    {
        const float4 own = ld(a.hc, zb, own_off, own_ok);
#pragma unroll
        for (int k = 0; k < NHK; ++k) hreg[k] = ld(a.hc, zb, h_off[k], h_ok[k]);
        tile_store(0, own, hreg);
    }
    Pw pw = load_pw(zb);
    __syncthreads();

    const float *c = a.c;
    const float srcv = a.src ? *a.src : 0.f;
    const bool zlo = a.faces & 16, zhi = a.faces & 32;
    int buf = 0;
    for (int z = zb; z < ze;) {
#pragma unroll
        for (int ph = 0; ph < Q; ++ph) {
            if (z < ze) {
                const bool more = z + 1 < ze;
                float4 nq = q[ph], nown = make_float4(0.f, 0.f, 0.f, 0.f);
                Pw npw = pw;
                if (more) {
                    nq = ld(a.vc, z + R + 1, own_off, own_ok);
                    nown = ld(a.hc, z + 1, own_off, own_ok);
#pragma unroll
                    for (int k = 0; k < NHK; ++k) hreg[k] = ld(a.hc, z + 1, h_off[k], h_ok[k]);
                    npw = load_pw(z + 1);
                }
                const float4 *t = &tile[buf][0][0];
                const float4 hc4 = t[(R + ty) * LW4 + tx + 1];
                const float4 L = t[(R + ty) * LW4 + tx];
                const float4 Rr = t[(R + ty) * LW4 + tx + 2];
                const float w[12] = {L.x,   L.y,   L.z,   L.w,  hc4.x, hc4.y,
                                     hc4.z, hc4.w, Rr.x, Rr.y, Rr.z,  Rr.w};
                float sxy[4] = {0.f, 0.f, 0.f, 0.f}, szz[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = -R; k <= R; ++k) {
                    const float ck = c[R + k];
                    const float4 vy = k == 0 ? hc4 : t[(R + ty + k) * LW4 + tx + 1];
                    const float4 vz = q[(ph + R + k + Q) % Q];
                    const float yv[4] = {vy.x, vy.y, vy.z, vy.w};
                    const float zv[4] = {vz.x, vz.y, vz.z, vz.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        sxy[e] = fmaf(ck, yv[e] + w[4 + e + k], sxy[e]);
                        szz[e] = fmaf(ck, zv[e], szz[e]);
                    }
                }
                const float gz = gaxis(z, g.nz, W, sa, zlo, zhi);
                const float4 vc4 = q[(ph + R) % Q];
                const float hcv[4] = {hc4.x, hc4.y, hc4.z, hc4.w};
                const float vcv[4] = {vc4.x, vc4.y, vc4.z, vc4.w};
                const float hpv[4] = {pw.hp.x, pw.hp.y, pw.hp.z, pw.hp.w};
                const float vpv[4] = {pw.vp.x, pw.vp.y, pw.vp.z, pw.vp.w};
                const float c2v[4] = {pw.c2.x, pw.c2.y, pw.c2.z, pw.c2.w};
                const float fav[4] = {pw.fa.x, pw.fa.y, pw.fa.z, pw.fa.w};
                const float fbv[4] = {pw.fb.x, pw.fb.y, pw.fb.z, pw.fb.w};
                float rh[4], rv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float G = gz * gown[e];
                    const float C2 = a.c2s * c2v[e];
                    rh[e] = G * (2.0f * hcv[e] - G * hpv[e] + C2 * (fav[e] * sxy[e] + fbv[e] * szz[e]));
                    rv[e] = G * (2.0f * vcv[e] - G * vpv[e] + C2 * (fbv[e] * sxy[e] + szz[e]));
                }
                if (srcv != 0.f && z == a.src_z && y == a.src_y && a.src_x >= x0 &&
                    a.src_x < x0 + 4) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (x0 + e == a.src_x) {
                            rh[e] += srcv;
                            rv[e] += srcv;
                        }
                }
                if (lane_on && y < g.ny && x0 < g.nx) {
                    float *ph_ = a.hn + (int64_t)z * sz + own_off;
                    float *pv_ = a.vn + (int64_t)z * sz + own_off;
                    if (x0 + 3 < g.nx) {
                        const f4v vh = {rh[0], rh[1], rh[2], rh[3]};
                        const f4v vv = {rv[0], rv[1], rv[2], rv[3]};
                        __builtin_nontemporal_store(vh, reinterpret_cast<f4v *>(ph_));
                        __builtin_nontemporal_store(vv, reinterpret_cast<f4v *>(pv_));
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (x0 + e < g.nx) {
                                ph_[e] = rh[e];
                                pv_[e] = rv[e];
                            }
                    }
                    if (a.traces && z == 0) {
                        float *pt = a.traces + (int64_t)y * g.nx + x0;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (x0 + e < g.nx) pt[e] = hcv[e];
                    }
                }
                if (more) {
                    tile_store(buf ^ 1, nown, hreg);
                    q[ph] = nq;
                    pw = npw;
                }
                __syncthreads();
                buf ^= 1;
                ++z;
            }
        }
    }
}

constexpr int VTX = 64, VTY = 8;

}  // namespace

int vti_step(const mms_wave *w, int n, const float *fa, const float *fb, const float *hp,
             const float *hc, float *hn, const float *vp, const float *vc, float *vn,
             hipStream_t s) {
    VtiArgs a{};
    Geom &g = a.g;
    const mms_grid *gd = &w->g;
    g.H = gd->halo;
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    g.txa = balanced_tile_words(g.nx, VTX, &g.ntx);
    g.nty = (g.ny + VTY - 1) / VTY;
    // one 512-thread block per CU (VGPR-bound), 256 CUs; the V queue fill costs
    // about one plane of traffic
    g.zchunk = pick_zchunk_rounds(g.nz, (int64_t)g.ntx * g.nty, 256, 8, 128, 1);
    g.nzc = (g.nz + g.zchunk - 1) / g.zchunk;
    const int r = w->radius;
    for (int k = -r; k <= r; ++k) a.c[k + r] = w->lap[k < 0 ? -k : k];
    const int64_t o = (int64_t)gd->halo * (gd->sz + gd->sy + 1);
    a.hc = hc + o;
    a.vc = vc + o;
    a.hp = hp + o;
    a.vp = vp + o;
    a.c2 = w->c2 + o;
    a.fa = fa + o;
    a.fb = fb + o;
    a.c2s = w->c2_scale;
    a.hn = hn + o;
    a.vn = vn + o;
    a.traces = w->traces ? w->traces + (int64_t)n * gd->ny * gd->nx : nullptr;
    a.src = (w->src_dt2f && n >= 0 && n < w->nt) ? w->src_dt2f + n : nullptr;
    a.src_z = (int)w->src_z;
    a.src_y = (int)w->src_y;
    a.src_x = (int)w->src_x;
    a.sponge_w = w->sponge_width;
    a.sponge_a = w->sponge_alpha;
    a.faces = w->sponge_faces;
    const int64_t nblk = (int64_t)g.ntx * g.nty * g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    const dim3 grid((unsigned)nblk), block(VTX * VTY);
    switch (r) {
        case 1: hipLaunchKernelGGL((vti_kernel<1, VTX, VTY>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((vti_kernel<2, VTX, VTY>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((vti_kernel<3, VTX, VTY>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((vti_kernel<4, VTX, VTY>), grid, block, 0, s, a); break;
        default: return MMS_EUNSUPPORTED;
    }
    return check_launch("vti_kernel");
}

}  // namespace mms
