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
//    ahead straight from memory into LDS (no staging registers), together with the
//    neighbouring tiles;
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

// One 16-byte word per lane from memory straight into LDS: lane l's word lands at
// dst + l (dst the same for the whole wave); completion is counted by vmcnt.
__device__ __forceinline__ void load_lds16(const float *src, float4 *dst) {
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

template <int R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) vti_kernel(VtiArgs a) {
    constexpr int Q = 2 * R + 1;
    constexpr int BY = TY;
    constexpr int LW4 = TX + 2, LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    constexpr int NL = LH * LW4;              // words of the H tile, row-major
    constexpr int NLK = (NL + NT - 1) / NT;
    // two arrays, each step's buffer fixed at compile time (phases in pairs), so that the
    // compiler does not wait on the direct loads before the current plane's reads
    __shared__ float4 tile0[NL];
    __shared__ float4 tile1[NL];

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
    auto ld = [&](const float *base, int z, int64_t off, bool ok) -> float4 {
        return guarded_load(base + (int64_t)z * sz + off, ok, a.c2);
    };
    // H tile word i -> (row i / LW4, col i % LW4) from the tile origin (row yt - R, column
    // xt - 4); words outside this tile's lw columns or outside the array are read from the
    // origin instead (never used)
    uint32_t d_off[NLK];
#pragma unroll
    for (int k = 0; k < NLK; ++k) {
        const int i = tid + k * NT;
        const int row = i / LW4, col = i % LW4;
        const bool ok = (i < NL) && (col < lw) && (yt - R + row < ylim) && (xt - 4 + 4 * col <= nx4);
        d_off[k] = ok ? (uint32_t)row * (uint32_t)sy + 4u * (uint32_t)col : 0u;
    }
    const int wave_base = __builtin_amdgcn_readfirstlane(tid & ~63);
    auto load_tile = [&](int z, float4 *t) {
        const float *p = a.hc + (int64_t)z * sz + (int64_t)(yt - R) * sy + (xt - 4);
#pragma unroll
        for (int k = 0; k < NLK; ++k)
            if (tid + k * NT < NL) load_lds16(p + d_off[k], t + wave_base + k * NT);
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
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = ld(a.vc, zb - R + i, own_off, own_ok);
    load_tile(zb, tile0);
    Pw pw = load_pw(zb);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    const float *c = a.c;
    const float srcv = a.src ? *a.src : 0.f;
    const bool zlo = a.faces & 16, zhi = a.faces & 32;
    // 2Q phases per round: the queue slot (ph mod Q) and the tile buffer (ph mod 2) are both
    // compile-time indices
    for (int z = zb; z < ze;) {
#pragma unroll
        for (int ph = 0; ph < 2 * Q; ++ph) {
            if (z < ze) {
                const bool more = z + 1 < ze;
                float4 *cur = (ph & 1) ? tile1 : tile0;
                float4 *nxt = (ph & 1) ? tile0 : tile1;
                float4 nq = q[ph % Q];
                Pw npw = pw;
                if (more) {
                    nq = ld(a.vc, z + R + 1, own_off, own_ok);
                    load_tile(z + 1, nxt);
                    npw = load_pw(z + 1);
                }
                const float4 *t = cur;
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
                    const float4 vz = q[(ph % Q + R + k + Q) % Q];
                    const float yv[4] = {vy.x, vy.y, vy.z, vy.w};
                    const float zv[4] = {vz.x, vz.y, vz.z, vz.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        sxy[e] = fmaf(ck, yv[e] + w[4 + e + k], sxy[e]);
                        szz[e] = fmaf(ck, zv[e], szz[e]);
                    }
                }
                const float gz = gaxis(z, g.nz, W, sa, zlo, zhi);
                const float4 vc4 = q[(ph % Q + R) % Q];
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
                // the next H tile is in LDS once this lane's requests are done; the barrier
                // publishes every lane's words and ends all reads of this plane; the output
                // stores come after it, so that the wait does not cover them
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
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
                    q[ph % Q] = nq;
                    pw = npw;
                }
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
    // the H tile is addressed with 32-bit offsets from its origin
    if ((int64_t)(VTY + 2 * w->radius + 1) * g.sy >= ((int64_t)1 << 32)) {
        set_last_error("VTI step: grid rows too long for 32-bit tile offsets");
        return MMS_EUNSUPPORTED;
    }
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
