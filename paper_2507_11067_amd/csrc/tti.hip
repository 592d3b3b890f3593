// Pseudo-acoustic TTI step (gfx950): the two-field update of RTM in tilted
// transversely isotropic media (Sec. II-A, Sec. V-F), in units of
// C2 = (v_pz dt / h)^2:
//   p'' = C2 [ (1+2eps) H2 p + alpha H1 q + sigma H1 (p - alpha q) ]
//   q'' = C2 [ ((1+2delta)/alpha) H2 p + H1 q - sigma H2 (p/alpha - q) ]
//   H1 = (n . grad)^2 with n = (sin t cos f, sin t sin f, cos t),  H2 = Laplacian - H1,
// stepped as u^{n+1} = G (2u^n - G u^{n-1} + dt^2 u'') + dt^2 f^n delta_src.
//
// The six second derivatives follow the paper's decomposition into
// one-dimensional stencils (Sec. IV-G): Dxx, Dyy, Dzz with the per-axis
// second-derivative weights; the mixed ones as products of first-derivative
// stencils D (weights d_1..d_r, antisymmetric).  Two passes:
//  * pass 1 (z only): Dz f and Dzz f of both fields for every cell of the padded
//    (x, y) extent, streamed through a register queue of 2r+1 planes; written to
//    a workspace of four grids.  Each plane of the padded array is contiguous,
//    so a lane owns one 16-byte word of it and the loads are fully coalesced.
//  * pass 2 (x and y): per plane, the tiles of p, q, Dz p and Dz q with r rows
//    and 4 cells of halo go from memory straight into a double-buffered LDS tile
//    (requested after the current plane's derivatives, with no staging
//    registers); Dxx, Dyy and Dxy = Dx(Dy f) come from the p / q tiles, Dxz =
//    Dx(Dz f) and Dyz = Dy(Dz f) from the Dz tiles; the direction cosines come
//    from theta / phi per cell; the update is fused with the sponge, source and
//    receivers; outputs are written with streaming stores.
#include "mms_internal.h"

namespace mms {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 f4(float a) { return make_float4(a, a, a, a); }

// sin and cos of an angle on the transcendental unit (v_sin_f32 / v_cos_f32 take the
// argument in revolutions and are valid below 256 revolutions in magnitude).  Measured
// on MI355X against FP64 over [-4 pi, 4 pi]: absolute error at most 9.2e-7, RMS 2.4e-7;
// one instruction each where a reduction plus polynomials took about 25, which made
// the eight evaluations per lane and plane 9 % of the kernel's time.
__device__ __forceinline__ void angle_sincos(float x, float *sn, float *cs) {
    const float t = x * 0.159154943091895336f;   // x / (2 pi)
    *sn = __builtin_amdgcn_sinf(t);
    *cs = __builtin_amdgcn_cosf(t);
}

// ------------------------------------------------------------------ pass 1
struct DzArgs {
    const float *p, *q;          // plane 0 of the padded array, z = 0 (interior)
    float *dzp, *dzq, *dzzp, *dzzq;
    int64_t plane_words;         // 16-byte words per plane ((ny + 2H) * sy / 4)
    int64_t sz;                  // plane stride in floats
    int nz, zchunk, ncol_blocks;
    float c2w[5];                // second-derivative weights: centre, k = 1..r
    float d1[4];                 // first-derivative weights d_1..d_r
};

template <int R>
__global__ void __launch_bounds__(256) tti_dz_kernel(DzArgs a) {
    constexpr int Q = 2 * R + 1;
    const int cb = blockIdx.x % a.ncol_blocks;
    const int zc = blockIdx.x / a.ncol_blocks;
    const int64_t word = (int64_t)cb * 256 + threadIdx.x;
    if (word >= a.plane_words) return;
    const int zb = zc * a.zchunk;
    const int ze = min(zb + a.zchunk, a.nz);
    const int64_t off = word * 4;
    auto ld = [&](const float *base, int z) -> float4 {
        return *reinterpret_cast<const float4 *>(base + (int64_t)z * a.sz + off);
    };
    float4 qp[Q], qq[Q];
#pragma unroll
    for (int i = 0; i < Q - 1; ++i) {
        qp[i] = ld(a.p, zb - R + i);
        qq[i] = ld(a.q, zb - R + i);
    }
    for (int z = zb; z < ze;) {
#pragma unroll
        for (int ph = 0; ph < Q; ++ph) {
            if (z < ze) {
                // slot of plane z+k is (ph + R + k) % Q; plane z+R enters now
                qp[(ph + 2 * R) % Q] = ld(a.p, z + R);
                qq[(ph + 2 * R) % Q] = ld(a.q, z + R);
                float4 f[2][2];  // [field][dz, dzz]
#pragma unroll
                for (int fi = 0; fi < 2; ++fi) {
                    const float4 *qu = fi == 0 ? qp : qq;
                    const float4 c = qu[(ph + R) % Q];
                    float4 d = f4(0.f), s = make_float4(a.c2w[0] * c.x, a.c2w[0] * c.y,
                                                        a.c2w[0] * c.z, a.c2w[0] * c.w);
#pragma unroll
                    for (int k = 1; k <= R; ++k) {
                        const float4 up = qu[(ph + R + k) % Q], dn = qu[(ph + R - k + Q) % Q];
                        const float dk = a.d1[k - 1], ck = a.c2w[k];
                        d.x = fmaf(dk, up.x - dn.x, d.x);
                        d.y = fmaf(dk, up.y - dn.y, d.y);
                        d.z = fmaf(dk, up.z - dn.z, d.z);
                        d.w = fmaf(dk, up.w - dn.w, d.w);
                        s.x = fmaf(ck, up.x + dn.x, s.x);
                        s.y = fmaf(ck, up.y + dn.y, s.y);
                        s.z = fmaf(ck, up.z + dn.z, s.z);
                        s.w = fmaf(ck, up.w + dn.w, s.w);
                    }
                    f[fi][0] = d;
                    f[fi][1] = s;
                }
                const int64_t o = (int64_t)z * a.sz + off;
                float *outs[4] = {a.dzp, a.dzzp, a.dzq, a.dzzq};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float4 v = f[i / 2][i % 2];
                    const f4v vv = {v.x, v.y, v.z, v.w};
                    __builtin_nontemporal_store(vv, reinterpret_cast<f4v *>(outs[i] + o));
                }
                ++z;
            }
        }
    }
}

// ------------------------------------------------------------------ pass 2
// One 16-byte word per lane from memory straight into LDS: lane l's word lands at
// dst + l (dst the same for the whole wave); completion is counted by vmcnt.
__device__ __forceinline__ void load_lds16(const float *src, float4 *dst) {
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

struct TtiArgs {
    Geom g;
    float c2w[5], d1[4];
    const float *pc, *qc, *dzp, *dzq;   // tiles
    const float *dzzp, *dzzq, *pp, *qp, *c2, *eps, *delta, *theta, *phi;  // own words
    float c2s, sigma, alpha, inv_alpha;
    float *pn, *qn;
    float *traces;
    const float *src;
    int src_z, src_y, src_x;
    int sponge_w;
    float sponge_a;
    int faces;
};

constexpr int NTILE = 4;   // p, q, Dz p, Dz q
constexpr int NOWN = 9;    // Dzz p, Dzz q, p^{n-1}, q^{n-1}, C2, eps, delta, theta, phi

template <int R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) tti_kernel(TtiArgs a) {
    constexpr int BY = TY;
    constexpr int LW4 = TX + 2, LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    __shared__ float4 tile[2][NTILE][LH][LW4];

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
    // tile word i -> (row i / LW4, col i % LW4) from the tile origin (row yt - R, column
    // xt - 4), loaded straight into LDS; words outside this tile's lw columns or outside the
    // array are read from the origin instead (they are never used)
    constexpr int NL = LH * LW4;
    constexpr int NLK = (NL + NT - 1) / NT;
    uint32_t d_off[NLK];
#pragma unroll
    for (int k = 0; k < NLK; ++k) {
        const int i = tid + k * NT;
        const int row = i / LW4, col = i % LW4;
        const bool ok = (i < NL) && (col < lw) && (yt - R + row < ylim) && (xt - 4 + 4 * col <= nx4);
        d_off[k] = ok ? (uint32_t)row * (uint32_t)sy + 4u * (uint32_t)col : 0u;
    }
    const float *tsrc[NTILE] = {a.pc, a.qc, a.dzp, a.dzq};
    // point-wise operands (theta and phi, the last two, are loaded separately)
    const float *osrc[NOWN] = {a.dzzp, a.dzzq, a.pp, a.qp, a.c2, a.eps, a.delta, a.theta, a.phi};
    const int wave_base = __builtin_amdgcn_readfirstlane(tid & ~63);
    auto load_tiles = [&](int z, int buf) {
        const int64_t zo = (int64_t)z * sz + (int64_t)(yt - R) * sy + (xt - 4);
#pragma unroll
        for (int f = 0; f < NTILE; ++f) {
            float4 *dst = &tile[buf][f][0][0] + wave_base;
#pragma unroll
            for (int k = 0; k < NLK; ++k)
                if (tid + k * NT < NL) load_lds16(tsrc[f] + zo + d_off[k], dst + k * NT);
        }
    };

    load_tiles(zb, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    const float srcv = a.src ? *a.src : 0.f;
    const bool zlo = a.faces & 16, zhi = a.faces & 32;
    for (int z = zb; z < ze; ++z) {
        const int buf = (z - zb) & 1;
        const bool more = z + 1 < ze;
        const int64_t zo = (int64_t)z * sz;
        // direction cosines of this plane's cells
        const float4 th4 = select_load(a.theta + zo + own_off, own_ok, a.c2);
        const float4 ph4 = select_load(a.phi + zo + own_off, own_ok, a.c2);
        // the other point-wise operands are requested here, so that the derivative phase
        // covers their latency (they are used only in the update)
        float4 ow[NOWN];
#pragma unroll
        for (int f = 0; f < NOWN - 2; ++f) ow[f] = select_load(osrc[f] + zo + own_off, own_ok, a.c2);
        auto comp = [](const float4 &v, int e) {
            return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
        };
        // H1 weights per cell: n_x^2, n_y^2, n_z^2, 2 n_x n_y, 2 n_y n_z, 2 n_x n_z
        float cf[6][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float st, ct, sp, cp;
            angle_sincos(comp(th4, e), &st, &ct);
            angle_sincos(comp(ph4, e), &sp, &cp);
            const float nx_ = st * cp, ny_ = st * sp, nz_ = ct;
            cf[0][e] = nx_ * nx_;
            cf[1][e] = ny_ * ny_;
            cf[2][e] = nz_ * nz_;
            cf[3][e] = 2.f * nx_ * ny_;
            cf[4][e] = 2.f * ny_ * nz_;
            cf[5][e] = 2.f * nx_ * nz_;
        }

        // x/y parts of L f and H1 f for both fields: [field][e].  Rows y+k and y-k are
        // taken together (they share the weights d_k and c_k); k runs as a loop so
        // that only one pair of rows per field is in registers at a time.
        float sxx[2][4], syy[2][4], sxz[2][4], syz[2][4];
        // Dy f over the 12-cell window of each field, summed over k; Dxy = Dx(Dy f)
        // is taken once after the k loop
        float dyw[2][12];
        auto window = [&](const float4 *row, float *w) {
            const float4 L = row[0], C = row[1], Rr = row[2];
            w[0] = L.x; w[1] = L.y; w[2] = L.z; w[3] = L.w;
            w[4] = C.x; w[5] = C.y; w[6] = C.z; w[7] = C.w;
            w[8] = Rr.x; w[9] = Rr.y; w[10] = Rr.z; w[11] = Rr.w;
        };
        auto dx1 = [&](const float *w, int e) {   // first x derivative at cell e
            float d = 0.f;
#pragma unroll
            for (int j = 1; j <= R; ++j) d = fmaf(a.d1[j - 1], w[4 + e + j] - w[4 + e - j], d);
            return d;
        };
#pragma unroll
        for (int fi = 0; fi < 2; ++fi) {
            const float4 *t = &tile[buf][fi][0][0] + ty * LW4 + tx;      // row 0 = y - R
            const float4 *tz = &tile[buf][2 + fi][0][0] + ty * LW4 + tx;
            float w[12], wz[12];
            window(t + R * LW4, w);
            window(tz + R * LW4, wz);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float s2 = a.c2w[0] * w[4 + e];
#pragma unroll
                for (int j = 1; j <= R; ++j) s2 = fmaf(a.c2w[j], w[4 + e + j] + w[4 + e - j], s2);
                sxx[fi][e] = s2;
                syy[fi][e] = a.c2w[0] * w[4 + e];
                sxz[fi][e] = dx1(wz, e);
                syz[fi][e] = 0.f;
            }
#pragma unroll
            for (int i = 0; i < 12; ++i) dyw[fi][i] = 0.f;
        }
#pragma unroll 1
        for (int k = 1; k <= R; ++k) {
            const float dk = a.d1[k - 1], ck = a.c2w[k];
#pragma unroll
            for (int fi = 0; fi < 2; ++fi) {
                const float4 *t = &tile[buf][fi][0][0] + ty * LW4 + tx;
                const float4 *tz = &tile[buf][2 + fi][0][0] + ty * LW4 + tx;
                float wu[12], wd[12];
                window(t + (R + k) * LW4, wu);
                window(t + (R - k) * LW4, wd);
                // Dx and Dy commute: Dxy f = Dx(sum_k d_k (row y+k - row y-k)), so the
                // rows' difference is summed over the window and differentiated in x
                // once, after the loop
#pragma unroll
                for (int i = 0; i < 12; ++i) dyw[fi][i] = fmaf(dk, wu[i] - wd[i], dyw[fi][i]);
                const float4 zu = tz[(R + k) * LW4 + 1], zd = tz[(R - k) * LW4 + 1];
                const float zuv[4] = {zu.x, zu.y, zu.z, zu.w}, zdv[4] = {zd.x, zd.y, zd.z, zd.w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    syy[fi][e] = fmaf(ck, wu[4 + e] + wd[4 + e], syy[fi][e]);
                    syz[fi][e] = fmaf(dk, zuv[e] - zdv[e], syz[fi][e]);
                }
            }
        }
        float lxy[2][4], h1[2][4];
#pragma unroll
        for (int fi = 0; fi < 2; ++fi)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                lxy[fi][e] = sxx[fi][e] + syy[fi][e];
                h1[fi][e] = cf[0][e] * sxx[fi][e] + cf[1][e] * syy[fi][e] +
                            cf[3][e] * dx1(dyw[fi], e) + cf[4][e] * syz[fi][e] +
                            cf[5][e] * sxz[fi][e];
            }
        // the next plane's tiles are requested after the last reads of this plane's tiles
        // (issued earlier, the compiler waits on them inside the k loop), so their latency
        // overlaps this plane's update and stores
        __builtin_amdgcn_sched_barrier(0);
        // the centre words of p and q are read before the next plane's tiles are requested
        const float4 *ctrp = &tile[buf][0][0][0] + (R + ty) * LW4 + tx + 1;
        const float4 *ctrq = &tile[buf][1][0][0] + (R + ty) * LW4 + tx + 1;
        const float4 pc4 = *ctrp, qc4 = *ctrq;
        if (more) load_tiles(z + 1, buf ^ 1);

        const float pcv[4] = {pc4.x, pc4.y, pc4.z, pc4.w}, qcv[4] = {qc4.x, qc4.y, qc4.z, qc4.w};
        const float gz = gaxis(z, g.nz, W, sa, zlo, zhi);
        float rp[4], rq[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float H1[2], H2[2];
#pragma unroll
            for (int fi = 0; fi < 2; ++fi) {
                const float dzz = comp(ow[fi], e);
                H1[fi] = fmaf(cf[2][e], dzz, h1[fi][e]);
                H2[fi] = (lxy[fi][e] + dzz) - H1[fi];
            }
            const float eps = comp(ow[5], e), del = comp(ow[6], e);
            const float sg = a.sigma, al = a.alpha, ia = a.inv_alpha;   // ia = 1 / alpha
            const float accp = (1.f + 2.f * eps) * H2[0] + al * H1[1] + sg * (H1[0] - al * H1[1]);
            const float accq = (1.f + 2.f * del) * ia * H2[0] + H1[1] - sg * (H2[0] * ia - H2[1]);
            const float G = gz * gown[e];
            const float C2 = a.c2s * comp(ow[4], e);
            rp[e] = G * (2.0f * pcv[e] - G * comp(ow[2], e) + C2 * accp);
            rq[e] = G * (2.0f * qcv[e] - G * comp(ow[3], e) + C2 * accq);
        }
        if (srcv != 0.f && z == a.src_z && y == a.src_y && a.src_x >= x0 && a.src_x < x0 + 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (x0 + e == a.src_x) {
                    rp[e] += srcv;
                    rq[e] += srcv;
                }
        }
        // the next plane's tiles are in LDS once this lane's requests are done; the barrier
        // publishes every lane's words and ends all reads of this plane; the output stores
        // come after it, so that the wait does not cover them
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (lane_on && y < g.ny && x0 < g.nx) {
            float *pp_ = a.pn + (int64_t)z * sz + own_off;
            float *qq_ = a.qn + (int64_t)z * sz + own_off;
            if (x0 + 3 < g.nx) {
                const f4v vp = {rp[0], rp[1], rp[2], rp[3]};
                const f4v vq = {rq[0], rq[1], rq[2], rq[3]};
                __builtin_nontemporal_store(vp, reinterpret_cast<f4v *>(pp_));
                __builtin_nontemporal_store(vq, reinterpret_cast<f4v *>(qq_));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (x0 + e < g.nx) {
                        pp_[e] = rp[e];
                        qq_[e] = rq[e];
                    }
            }
            if (a.traces && z == 0) {
                float *pt = a.traces + (int64_t)y * g.nx + x0;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (x0 + e < g.nx) pt[e] = pcv[e];
            }
        }
    }
}

// 256 x 8 tiles, 512 threads: four double-buffered plane tiles fill 135 KB of LDS
// at radius 4, one block per CU
constexpr int TTX = 64, TTY = 8;

template <int R>
int launch_tti(const mms_wave *w, const mms_tti *t, int n, const float *pp, const float *pc,
               float *pn, const float *qp, const float *qc, float *qn, hipStream_t s) {
    const mms_grid *gd = &w->g;
    const int64_t o = (int64_t)gd->halo * (gd->sz + gd->sy + 1);
    // pass 2 addresses its plane tiles with 32-bit offsets from the tile origin; checked
    // before either pass is launched
    if ((int64_t)(TTY + 2 * R + 1) * gd->sy >= ((int64_t)1 << 32)) {
        set_last_error("TTI step: grid rows too long for 32-bit tile offsets");
        return MMS_EUNSUPPORTED;
    }
    const int64_t L = grid_elems(gd);
    float *dzp = t->work, *dzq = t->work + L, *dzzp = t->work + 2 * L, *dzzq = t->work + 3 * L;
    // pass 1 over every word of the interior planes (rows of the y halo included)
    {
        DzArgs a{};
        const int64_t zo = (int64_t)gd->halo * gd->sz;
        a.p = pc + zo;
        a.q = qc + zo;
        a.dzp = dzp + zo;
        a.dzq = dzq + zo;
        a.dzzp = dzzp + zo;
        a.dzzq = dzzq + zo;
        a.plane_words = (gd->ny + 2 * gd->halo) * gd->sy / 4;
        a.sz = gd->sz;
        a.nz = (int)gd->nz;
        for (int k = 0; k <= R; ++k) a.c2w[k] = w->lap[k];
        for (int k = 0; k < R; ++k) a.d1[k] = t->d1[k];
        const int64_t ncb = (a.plane_words + 255) / 256;
        const int zc = pick_zchunk_rounds(a.nz, ncb, launch_slots(
            reinterpret_cast<const void *>(&tti_dz_kernel<R>), 256), 8, 128, 2 * R);
        a.zchunk = zc;
        a.ncol_blocks = (int)ncb;
        const int64_t nblk = ncb * ((a.nz + zc - 1) / zc);
        if (nblk > 0x7fffffff) return MMS_EINVAL;
        hipLaunchKernelGGL((tti_dz_kernel<R>), dim3((unsigned)nblk), dim3(256), 0, s, a);
        if (int rc = check_launch("tti_dz_kernel")) return rc;
    }
    TtiArgs a{};
    Geom &g = a.g;
    g.H = gd->halo;
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    g.txa = balanced_tile_words(g.nx, TTX, &g.ntx);
    g.nty = (g.ny + TTY - 1) / TTY;
    g.zchunk = pick_zchunk_rounds(g.nz, (int64_t)g.ntx * g.nty,
                                  launch_slots(reinterpret_cast<const void *>(&tti_kernel<R, TTX, TTY>),
                                               TTX * TTY), 8, 128, 1);
    g.nzc = (g.nz + g.zchunk - 1) / g.zchunk;
    for (int k = 0; k <= R; ++k) a.c2w[k] = w->lap[k];
    for (int k = 0; k < R; ++k) a.d1[k] = t->d1[k];
    a.pc = pc + o;
    a.qc = qc + o;
    a.dzp = dzp + o;
    a.dzq = dzq + o;
    a.dzzp = dzzp + o;
    a.dzzq = dzzq + o;
    a.pp = pp + o;
    a.qp = qp + o;
    a.c2 = w->c2 + o;
    a.eps = t->eps + o;
    a.delta = t->delta + o;
    a.theta = t->theta + o;
    a.phi = t->phi + o;
    a.c2s = w->c2_scale;
    a.sigma = t->sigma;
    a.alpha = t->alpha;
    a.inv_alpha = 1.0f / t->alpha;
    a.pn = pn + o;
    a.qn = qn + o;
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
    hipLaunchKernelGGL((tti_kernel<R, TTX, TTY>), dim3((unsigned)nblk), dim3(TTX * TTY), 0, s, a);
    return check_launch("tti_kernel");
}

}  // namespace

int tti_step(const mms_wave *w, const mms_tti *t, int n, const float *pp, const float *pc,
             float *pn, const float *qp, const float *qc, float *qn, hipStream_t s) {
    switch (w->radius) {
        case 1: return launch_tti<1>(w, t, n, pp, pc, pn, qp, qc, qn, s);
        case 2: return launch_tti<2>(w, t, n, pp, pc, pn, qp, qc, qn, s);
        case 3: return launch_tti<3>(w, t, n, pp, pc, pn, qp, qc, qn, s);
        case 4: return launch_tti<4>(w, t, n, pp, pc, pn, qp, qc, qn, s);
        default: return MMS_EUNSUPPORTED;
    }
}

}  // namespace mms
