// Fused acoustic wave step, its adjoint, and the discrete energy (gfx950).
//
// Forward step (the leapfrog update RTM is built on, Sec. II-A), one launch per
// time level:
//   u^{n+1} = G (2 u^n - G u^{n-1} + C2 S(u^n)) + dt^2 f^n delta_src
// with the receiver reading d^n = u^n(z = 0) and the FP64 image
// I += (u^{n+1})^2 fused in (every step, or per block of K steps summed in FP32,
// which halves the image traffic).  Adjoint step (exact transpose of the recurrence):
//   lam^n = 2 G lam^{n+1} - G^2 lam^{n+2} + S(C2 G lam^{n+1}) + R^T r^n
//   grad += G lam^{n+1} S(u^n)                    (FP64)
// S is the symmetric star, so S^T = S.  The gradient is a second pass of the same
// kernel with u^n as its stencil field (one stencil field per pass keeps the tile
// at 256 x 16 cells and four waves per SIMD).  Every pass streams z through an
// (x, y) tile like the star sweep: the stencil operand travels through a
// register queue of 2r+1 planes (z terms) and an LDS ring of r+2 plane tiles
// (x and y terms); the point-wise operands are requested one plane ahead.
// The intermediate fields S(u^n), C2 G lam^{n+1} and S(C2 G lam^{n+1}) never
// reach memory (the paper's thread-private intermediate buffers, Sec. IV-G).
// The sponge factor is separable, G = gz(z) gy(y) gx(x); each lane evaluates
// the x and y factors of its cells once and gz once per plane.
#include "mms_internal.h"

namespace mms {
namespace {

// ADJMU: the adjoint step carried in mu = C2 G lam, which has the forward step's form
//   mu^n = G (2 mu^{n+1} - G mu^{n+2} + C2 S(mu^{n+1})) + C2 G R^T r^n
// (one stencil stream, where the lam form forms C2 G lam from two)
enum { MODE_FWD = 0, MODE_ADJ = 1, MODE_ENERGY = 2, MODE_GRAD = 3, MODE_ADJMU = 4 };

typedef float f4v __attribute__((ext_vector_type(4)));

struct WaveArgs {
    Geom g;
    float c[9];           // per-axis weights, k + r (symmetric)
    const float *f0;      // stencil field: u^n (FWD, ENERGY, GRAD) or lam^{n+1} (ADJ)
    const float *c2;      // c2 field (interior origin); C2 = c2s * c2
    float c2s;
    const float *p0;      // point-wise: u^{n-1} (FWD), lam^{n+2} (ADJ), u^{n+1} (ENERGY),
                          // lam^{n+1} (GRAD)
    float *out;           // u^{n+1} (FWD), lam^n (ADJ)
    float *traces;        // FWD: [ny][nx] plane of level n, or NULL
    const float *resid;   // ADJ: [ny][nx] plane of level n, or NULL
    double *acc64;        // FWD: image, GRAD: grad (dense [nz][ny][nx]), or NULL
    float *part;          // FP32 partial of the current block (image or grad), or NULL
    int part_first;       // with part: first step of a block (part = term)
    int part_last;        // with part: last step of a block (acc64 += part + term)
    double *partials;     // ENERGY: one (FP64 partial, non-finite count) pair per block
    const float *src;     // device pointer to dt^2 f^n, or NULL
    int src_z, src_y, src_x;
    int sponge_w;
    float sponge_a;
    int faces;
    int mu_form;          // GRAD, first adjoint step: the adjoint variable is mu = C2 G lam
};

template <int R, int MODE, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) wave_kernel(WaveArgs a) {
    constexpr int Q = 2 * R + 1;
    constexpr int BY = TY;
    constexpr int LW4 = TX + 2, LH = BY + 2 * R;
    constexpr int NT = TX * TY;
    constexpr int NH = 2 * R * LW4 + 2 * BY;
    constexpr int NHK = (NH + NT - 1) / NT;
    constexpr int NR = R + 2;   // LDS ring: planes z .. z+R+1
    __shared__ float4 ring[NR][LH][LW4];
    __shared__ double sred[2 * (NT / 64)];

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
    // sponge factors gy(y) gx(x) of the lane's own cells
    float gown[4];
    {
        const float gy = gaxis(y, g.ny, W, sa, a.faces & 4, a.faces & 8);
#pragma unroll
        for (int e = 0; e < 4; ++e) gown[e] = gy * gaxis(x0 + e, g.nx, W, sa, a.faces & 1, a.faces & 2);
    }
    int64_t h_off[NHK];
    int h_lds[NHK];
    bool h_ok[NHK], h_on[NHK];  // h_on: item k is one of this tile's halo words
    float hg[NHK][4];  // ADJ: gy gx of the halo cells (C2 G lam is formed on load)
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
        if constexpr (MODE == MODE_ADJ) {
            const float gy = gaxis(row, g.ny, W, sa, a.faces & 4, a.faces & 8);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                hg[k][e] = gy * gaxis(x + e, g.nx, W, sa, a.faces & 1, a.faces & 2);
        }
    }
    (void)hg;
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool zlo = a.faces & 16, zhi = a.faces & 32;

    auto ld = [&](const float *base, int z, int64_t off, bool ok) -> float4 {
        return guarded_load(base + (int64_t)z * sz + off, ok, a.c2);
    };
    auto mul4 = [](float4 v, const float *s, float t) {
        return make_float4(v.x * s[0] * t, v.y * s[1] * t, v.z * s[2] * t, v.w * s[3] * t);
    };
    // stencil field of plane z at the lane's own cells / halo item k (ADJ: C2 G lam)
    auto own_field = [&](int z) -> float4 {
        if (MODE == MODE_ADJ) {
            const float4 l = ld(a.f0, z, own_off, own_ok);
            const float4 c = ld(a.c2, z, own_off, own_ok);
            const float gz = a.c2s * gaxis(z, g.nz, W, sa, zlo, zhi);
            return mul4(make_float4(l.x * c.x, l.y * c.y, l.z * c.z, l.w * c.w), gown, gz);
        }
        return ld(a.f0, z, own_off, own_ok);
    };
    auto halo_field = [&](int z, int k) -> float4 {
        if (MODE == MODE_ADJ) {
            const float4 l = ld(a.f0, z, h_off[k], h_ok[k]);
            const float4 c = ld(a.c2, z, h_off[k], h_ok[k]);
            const float gz = a.c2s * gaxis(z, g.nz, W, sa, zlo, zhi);
            return mul4(make_float4(l.x * c.x, l.y * c.y, l.z * c.z, l.w * c.w), hg[k], gz);
        }
        return ld(a.f0, z, h_off[k], h_ok[k]);
    };
    // tile of one plane (own cells + halo) into ring slot `slot`
    auto ring_store = [&](int slot, const float4 &own, const float4 *halo) {
        float4 *t = &ring[slot][0][0];
        if (lane_on) t[(R + ty) * LW4 + tx + 1] = own;
#pragma unroll
        for (int k = 0; k < NHK; ++k)
            if (h_on[k]) t[h_lds[k]] = halo[k];
    };

    float4 q[Q];
    float4 hreg[NHK];
    // prologue: planes zb-R .. zb+R into the queue; tiles of planes zb .. zb+R into the ring
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = own_field(zb - R + i);
#pragma unroll
    for (int i = 0; i <= R; ++i) {
#pragma unroll
        for (int k = 0; k < NHK; ++k) hreg[k] = halo_field(zb + i, k);
        ring_store((zb + i) % NR, q[R + i], hreg);
    }
    // point-wise operands of the first plane
    // second point-wise operand: lam^{n+1} (ADJ), C2 (FWD, ENERGY); GRAD: the FP32 block
    // partial of the lane's cells (when it is read and the row allows 16-byte access)
    auto ld_pw1 = [&](int z) -> float4 {
        if constexpr (MODE == MODE_GRAD) {
            // the same condition as the 16-byte path of the accumulation below
            // (otherwise the load reads the interior origin of C2 and the value is unused)
            const int64_t d = ((int64_t)z * g.ny + y) * g.nx + x0;
            const bool use = a.part && !a.part_first && lane_on && y < g.ny && x0 + 3 < g.nx &&
                             (d & 3) == 0;
            return *reinterpret_cast<const float4 *>(use ? a.part + d : a.c2);
        }
        return ld(MODE == MODE_ADJ ? a.f0 : a.c2, z, own_off, own_ok);
    };
    float4 pw0 = ld(a.p0, zb, own_off, own_ok);
    float4 pw1 = ld_pw1(zb);
    __syncthreads();

    const float *c = a.c;
    const float srcv = (MODE == MODE_FWD && a.src) ? *a.src : 0.f;
    double esum = 0.0, ebad = 0.0;
    for (int z = zb; z < ze;) {
#pragma unroll
        for (int ph = 0; ph < Q; ++ph) {
            if (z < ze) {
                const bool more = z + 1 < ze;
                float4 nq = zero4;
                float4 npw0 = pw0, npw1 = pw1;   // replaced below unless this is the last plane
                if (more) {
                    // the tile of plane z+R+1 is requested together with the neighbouring
                    // tiles that read the same rows, and parked in the ring
                    nq = own_field(z + R + 1);
#pragma unroll
                    for (int k = 0; k < NHK; ++k) hreg[k] = halo_field(z + R + 1, k);
                    npw0 = ld(a.p0, z + 1, own_off, own_ok);
                    npw1 = ld_pw1(z + 1);
                }
                // o = S f at the lane's 4 cells
                float o[4] = {0.f, 0.f, 0.f, 0.f};
                const float4 *t = &ring[z % NR][0][0];
                const float4 ctr = q[(ph + R) % Q];
#pragma unroll
                for (int k = -R; k <= R; ++k) {
                    const float4 vz = q[(ph + R + k + Q) % Q];
                    const float4 vy = k == 0 ? ctr : t[(R + ty + k) * LW4 + tx + 1];
                    const float ck = c[R + k];
                    o[0] = fmaf(ck, vz.x + vy.x, o[0]);
                    o[1] = fmaf(ck, vz.y + vy.y, o[1]);
                    o[2] = fmaf(ck, vz.z + vy.z, o[2]);
                    o[3] = fmaf(ck, vz.w + vy.w, o[3]);
                }
                {
                    const float4 L = t[(R + ty) * LW4 + tx];
                    const float4 Rr = t[(R + ty) * LW4 + tx + 2];
                    const float w[12] = {L.x,   L.y,   L.z,   L.w,  ctr.x, ctr.y,
                                         ctr.z, ctr.w, Rr.x, Rr.y, Rr.z,  Rr.w};
#pragma unroll
                    for (int k = -R; k <= R; ++k)
#pragma unroll
                        for (int e = 0; e < 4; ++e) o[e] = fmaf(c[R + k], w[4 + e + k], o[e]);
                }
                const float gz = gaxis(z, g.nz, W, sa, zlo, zhi);
                const bool live = lane_on && y < g.ny && x0 < g.nx;
                const int64_t dense = ((int64_t)z * g.ny + y) * g.nx + x0;
                float *po = a.out ? a.out + (int64_t)z * sz + own_off : nullptr;
                const float p0v[4] = {pw0.x, pw0.y, pw0.z, pw0.w};
                const float p1v[4] = {pw1.x, pw1.y, pw1.z, pw1.w};
                const float cv[4] = {ctr.x, ctr.y, ctr.z, ctr.w};
                float r[4] = {0.f, 0.f, 0.f, 0.f};
                if constexpr (MODE == MODE_FWD || MODE == MODE_ADJMU) {
                    // FWD: p0 = u^{n-1}, p1 = C2, ctr = u^n; ADJMU: p0 = mu^{n+2}, ctr = mu^{n+1}
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float G = gz * gown[e];
                        r[e] = G * (2.0f * cv[e] - G * p0v[e] + a.c2s * p1v[e] * o[e]);
                    }
                    if constexpr (MODE == MODE_FWD) {
                        if (srcv != 0.f && z == a.src_z && y == a.src_y && a.src_x >= x0 &&
                            a.src_x < x0 + 4) {
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (x0 + e == a.src_x) r[e] += srcv;
                        }
                    } else {
                        // receivers: + C2 G r^n on the plane z = 0
                        if (a.resid && z == 0 && live) {
                            const float *rs = a.resid + (int64_t)y * g.nx + x0;
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (x0 + e < g.nx) r[e] += a.c2s * p1v[e] * (gz * gown[e]) * rs[e];
                        }
                    }
                } else if constexpr (MODE == MODE_ADJ) {
                    // p0 = lam^{n+2}, p1 = lam^{n+1}
                    const float *rs = (a.resid && z == 0) ? a.resid + (int64_t)y * g.nx + x0 : nullptr;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float G = gz * gown[e];
                        r[e] = 2.0f * G * p1v[e] - G * G * p0v[e] + o[e];
                        if (rs && live && x0 + e < g.nx) r[e] += rs[e];
                    }
                } else if constexpr (MODE == MODE_ENERGY) {
                    // ENERGY: p0 = u^{n+1}, p1 = C2, ctr = u^n, o = S u^n
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (live && x0 + e < g.nx) {
                            const double d = (double)p0v[e] - (double)cv[e];
                            double t = -(double)p0v[e] * (double)o[e];
                            if (p1v[e] != 0.f) t += d * d / ((double)a.c2s * (double)p1v[e]);
                            esum += t;
                            ebad += isfinite(t) ? 0.0 : 1.0;
                        }
                    }
                }
                if (MODE != MODE_ENERGY && live) {
                    if (MODE == MODE_GRAD) {
                        // no field output
                    } else if (x0 + 3 < g.nx) {
                        // streaming store: the next step reads this field from HBM anyway
                        const f4v v = {r[0], r[1], r[2], r[3]};
                        __builtin_nontemporal_store(v, reinterpret_cast<f4v *>(po));
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (x0 + e < g.nx) po[e] = r[e];
                    }
                    if (MODE == MODE_FWD && a.traces && z == 0) {
                        float *pt = a.traces + (int64_t)y * g.nx + x0;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (x0 + e < g.nx) pt[e] = cv[e];
                    }
                    if (MODE == MODE_FWD || MODE == MODE_GRAD) if (a.acc64) {
                        // the accumulated term of each cell: FWD (u^{n+1})^2, GRAD
                        // G lam^{n+1} S(u^n) (p0 = lam^{n+1}, o = S u^n); in FP32 for the
                        // block partial, in FP64 for a direct update (t64)
                        float t[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            t[e] = MODE == MODE_FWD ? r[e] * r[e]
                                   : a.mu_form ? p0v[e] * o[e]      // mu^{n+1} S(u^n), / c2 below
                                               : a.c2s * gz * gown[e] * p0v[e] * o[e];
                        // mu form: c2 G lam^{n+1} S(u^n) = mu^{n+1} S(u^n) / c2, with c2 the field
                        // (C2 = c2s c2); the division is done in FP64 where a sum reaches acc64,
                        // so the c2 field is read (cell by cell) once per block of steps
                        const bool div_c2 = MODE == MODE_GRAD && a.mu_form;
                        const float *c2row = a.c2 + (int64_t)z * sz + own_off;
                        auto fin = [&](int e, double v) -> double {
                            return div_c2 ? v / (double)c2row[e] : v;
                        };
                        auto t64 = [&](int e) -> double {
                            return MODE == MODE_FWD ? (double)r[e] * (double)r[e] : fin(e, (double)t[e]);
                        };
                        double *pa = a.acc64 + dense;
                        // four cells in range on a 16-byte aligned dense row: one 16-byte
                        // access per operand (two for the FP64 sums) instead of four
                        const bool vec = x0 + 3 < g.nx && (dense & 3) == 0;
                        if (!a.part) {
                            if (vec) {
                                double2 *p2 = reinterpret_cast<double2 *>(pa);
                                double2 lo = p2[0], hi = p2[1];
                                lo.x += t64(0);
                                lo.y += t64(1);
                                hi.x += t64(2);
                                hi.y += t64(3);
                                p2[0] = lo;
                                p2[1] = hi;
                            } else {
#pragma unroll
                                for (int e = 0; e < 4; ++e)
                                    if (x0 + e < g.nx) pa[e] += t64(e);
                            }
                        } else {
                            // FP32 partial over the block, added in FP64 at its end
                            float *pp = a.part + dense;
                            if (vec) {
                                // GRAD: the partial came with the point-wise operands
                                const float4 pv = a.part_first ? zero4
                                                  : MODE == MODE_GRAD ? pw1
                                                                      : *reinterpret_cast<const float4 *>(pp);
                                const float pa4[4] = {pv.x, pv.y, pv.z, pv.w};
                                float sum[4];
#pragma unroll
                                for (int e = 0; e < 4; ++e) sum[e] = a.part_first ? t[e] : pa4[e] + t[e];
                                if (a.part_last) {
                                    double2 *p2 = reinterpret_cast<double2 *>(pa);
                                    double2 lo = p2[0], hi = p2[1];
                                    lo.x += fin(0, (double)sum[0]);
                                    lo.y += fin(1, (double)sum[1]);
                                    hi.x += fin(2, (double)sum[2]);
                                    hi.y += fin(3, (double)sum[3]);
                                    p2[0] = lo;
                                    p2[1] = hi;
                                } else {
                                    *reinterpret_cast<float4 *>(pp) = make_float4(sum[0], sum[1], sum[2], sum[3]);
                                }
                            } else {
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    if (x0 + e < g.nx) {
                                        const float sum = a.part_first ? t[e] : pp[e] + t[e];
                                        if (a.part_last)
                                            pa[e] += fin(e, (double)sum);
                                        else
                                            pp[e] = sum;
                                    }
                                }
                            }
                        }
                    }
                }
                if (more) {
                    ring_store((z + R + 1) % NR, nq, hreg);
                    q[ph] = nq;
                    pw0 = npw0;
                    pw1 = npw1;
                }
                __syncthreads();
                ++z;
            }
        }
    }
    if constexpr (MODE == MODE_ENERGY) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            esum += __shfl_xor(esum, o);
            ebad += __shfl_xor(ebad, o);
        }
        if ((tid & 63) == 0) {
            sred[2 * (tid >> 6)] = esum;
            sred[2 * (tid >> 6) + 1] = ebad;
        }
        __syncthreads();
        if (tid == 0) {
            double s = 0.0, bad = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) {
                s += sred[2 * w];
                bad += sred[2 * w + 1];
            }
            a.partials[2 * blockIdx.x] = s;
            a.partials[2 * blockIdx.x + 1] = bad;
        }
    }
}

// lam^0 = -G^2 lam^2 + R^T r^0 (point-wise; u^0 enters only through step 1's G^2 term)
__global__ void adjoint_first_kernel(WaveArgs a) {
    const Geom &g = a.g;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (int64_t)g.nx * g.ny * g.nz;
    if (i >= np) return;
    const int x = (int)(i % g.nx);
    const int y = (int)((i / g.nx) % g.ny);
    const int z = (int)(i / ((int64_t)g.nx * g.ny));
    const int64_t off = (int64_t)z * g.sz + (int64_t)y * g.sy + x;
    const int W = a.sponge_w;
    const float G = gaxis(z, g.nz, W, a.sponge_a, a.faces & 16, a.faces & 32) *
                    gaxis(y, g.ny, W, a.sponge_a, a.faces & 4, a.faces & 8) *
                    gaxis(x, g.nx, W, a.sponge_a, a.faces & 1, a.faces & 2);
    float v = -G * G * a.p0[off];
    if (a.resid && z == 0) {
        const float r = a.resid[(int64_t)y * g.nx + x];
        v += a.mu_form ? a.c2s * a.c2[off] * G * r : r;   // mu form: C2 G R^T r^0
    }
    a.out[off] = v;
}

// mu = C2 G lam (dir > 0) or lam = mu / (C2 G) (dir < 0) on the interior; in may equal out
__global__ void scale_mu_kernel(WaveArgs a, const float *in, float *out, int dir) {
    const Geom &g = a.g;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (int64_t)g.nx * g.ny * g.nz;
    if (i >= np) return;
    const int x = (int)(i % g.nx);
    const int y = (int)((i / g.nx) % g.ny);
    const int z = (int)(i / ((int64_t)g.nx * g.ny));
    const int64_t off = (int64_t)z * g.sz + (int64_t)y * g.sy + x;
    const int W = a.sponge_w;
    const float G = gaxis(z, g.nz, W, a.sponge_a, a.faces & 16, a.faces & 32) *
                    gaxis(y, g.ny, W, a.sponge_a, a.faces & 4, a.faces & 8) *
                    gaxis(x, g.nx, W, a.sponge_a, a.faces & 1, a.faces & 2);
    const float f = a.c2s * a.c2[off] * G;
    out[off] = dir > 0 ? in[off] * f : in[off] / f;
}

__global__ void dense_to_grid_kernel(const double *in, float *out, int nx, int ny, int64_t sy,
                                     int64_t sz, double scale) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x < nx) out[(int64_t)z * sz + (int64_t)y * sy + x] =
        (float)(scale * in[((int64_t)z * ny + y) * nx + x]);
}

__global__ void record_kernel(const float *u0, float *tr, int nx, int ny, int64_t sy) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x < nx) tr[(int64_t)y * nx + x] = u0[(int64_t)y * sy + x];
}

// Tile shape: up to 256 x 16 cells per block (64 x 16 lanes); the LDS ring fills most
// of a CU's LDS, so one block runs per CU.
constexpr int WTX = 64, WTY = 16;

void fill_geom(Geom &g, const mms_grid *gd) {
    g.H = gd->halo;
    g.nx = (int)gd->nx;
    g.ny = (int)gd->ny;
    g.nz = (int)gd->nz;
    g.sy = gd->sy;
    g.sz = gd->sz;
    g.txa = balanced_tile_words(g.nx, WTX, &g.ntx);
    g.nty = (g.ny + WTY - 1) / WTY;
    // one block per CU (LDS-bound): the columns split evenly over the CUs
    g.zchunk = pick_zchunk(g.nz, (int64_t)g.ntx * g.nty, 256, 8, 128);
    g.nzc = (g.nz + g.zchunk - 1) / g.zchunk;
}

WaveArgs base_args(const mms_wave *w) {
    WaveArgs a{};
    const int r = w->radius;
    for (int k = -r; k <= r; ++k) a.c[k + r] = w->lap[k < 0 ? -k : k];
    a.sponge_w = w->sponge_width;
    a.sponge_a = w->sponge_alpha;
    a.faces = w->sponge_faces;
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    a.c2 = w->c2 + o;
    a.c2s = w->c2_scale;
    return a;
}

template <int MODE>
int launch_mode(WaveArgs &a, const mms_grid *gd, int r, hipStream_t s) {
    constexpr int TX = WTX, TY = WTY;
    fill_geom(a.g, gd);
    const int64_t nblk = (int64_t)a.g.ntx * a.g.nty * a.g.nzc;
    if (nblk > 0x7fffffff) return MMS_EINVAL;
    const dim3 grid((unsigned)nblk), block(TX * TY);
    switch (r) {
        case 1: hipLaunchKernelGGL((wave_kernel<1, MODE, TX, TY>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((wave_kernel<2, MODE, TX, TY>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((wave_kernel<3, MODE, TX, TY>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((wave_kernel<4, MODE, TX, TY>), grid, block, 0, s, a); break;
        default: return MMS_EUNSUPPORTED;
    }
    return check_launch("wave_kernel");
}

}  // namespace

int wave_step(const mms_wave *w, int n, const float *up, const float *uc, float *un, hipStream_t s) {
    WaveArgs a = base_args(w);
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    a.f0 = uc + o;
    a.p0 = up + o;
    a.out = un + o;
    a.traces = w->traces ? w->traces + (int64_t)n * w->g.ny * w->g.nx : nullptr;
    a.acc64 = w->image;
    if (w->image && w->acc_block > 1) {
        const int K = w->acc_block, ph = (n - 1) % K;
        a.part = w->acc_part;
        a.part_first = ph == 0;
        a.part_last = ph == K - 1 || n == w->nt - 1;
    }
    a.src = (w->src_dt2f && n >= 0 && n < w->nt) ? w->src_dt2f + n : nullptr;
    a.src_z = (int)w->src_z;
    a.src_y = (int)w->src_y;
    a.src_x = (int)w->src_x;
    return launch_mode<MODE_FWD>(a, &w->g, w->radius, s);
}

int wave_adjoint_step(const mms_wave *w, int n, const float *l2, const float *l1, float *l0,
                      const float *resid, const float *un, double *grad, hipStream_t s) {
    WaveArgs a = base_args(w);
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    a.p0 = l2 + o;
    a.out = l0 + o;
    a.resid = resid ? resid + (int64_t)n * w->g.ny * w->g.nx : nullptr;
    if (n == 0) {
        fill_geom(a.g, &w->g);
        const int64_t np = w->g.nx * w->g.ny * w->g.nz;
        const unsigned nb = (unsigned)((np + 255) / 256);
        hipLaunchKernelGGL(adjoint_first_kernel, dim3(nb), dim3(256), 0, s, a);
        return check_launch("adjoint_first_kernel");
    }
    a.f0 = l1 + o;
    const int rc = launch_mode<MODE_ADJ>(a, &w->g, w->radius, s);
    if (rc || !grad) return rc;
    // gradient: a second one-field pass over u^n (stencil) and lam^{n+1}.  Fused into
    // the adjoint pass it needs two register queues and two LDS rings, which halves
    // the tile and the occupancy; two passes move 6 B more per point and run faster.
    WaveArgs b = base_args(w);
    b.f0 = un + o;
    b.p0 = l1 + o;
    b.acc64 = grad;
    if (w->acc_block > 1) {
        // blocks counted down from n = nt-1, the order the adjoint runs in
        const int K = w->acc_block, ph = (w->nt - 1 - n) % K;
        b.part = w->acc_part;
        b.part_first = ph == 0;
        b.part_last = ph == K - 1 || n == 1;
    }
    return launch_mode<MODE_GRAD>(b, &w->g, w->radius, s);
}

int wave_adjoint_mu_step(const mms_wave *w, int n, const float *m2, const float *m1, float *m0,
                         const float *resid, const float *un, double *grad, hipStream_t s) {
    WaveArgs a = base_args(w);
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    a.p0 = m2 + o;
    a.out = m0 + o;
    a.resid = resid ? resid + (int64_t)n * w->g.ny * w->g.nx : nullptr;
    a.mu_form = 1;
    if (n == 0) {
        fill_geom(a.g, &w->g);
        const int64_t np = w->g.nx * w->g.ny * w->g.nz;
        hipLaunchKernelGGL(adjoint_first_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, a);
        return check_launch("adjoint_first_kernel");
    }
    a.f0 = m1 + o;
    const int rc = launch_mode<MODE_ADJMU>(a, &w->g, w->radius, s);
    if (rc || !grad) return rc;
    // gradient terms mu^{n+1} S(u^n) / c2 (the division where a sum reaches grad)
    WaveArgs b = base_args(w);
    b.f0 = un + o;
    b.p0 = m1 + o;
    b.acc64 = grad;
    b.mu_form = 1;
    if (w->acc_block > 1) {
        const int K = w->acc_block, ph = (w->nt - 1 - n) % K;
        b.part = w->acc_part;
        b.part_first = ph == 0;
        b.part_last = ph == K - 1 || n == 1;
    }
    return launch_mode<MODE_GRAD>(b, &w->g, w->radius, s);
}

int wave_scale_mu(const mms_wave *w, const float *in, float *out, int dir, hipStream_t s) {
    WaveArgs a = base_args(w);
    fill_geom(a.g, &w->g);
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    const int64_t np = w->g.nx * w->g.ny * w->g.nz;
    hipLaunchKernelGGL(scale_mu_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, a,
                       in + o, out + o, dir);
    return check_launch("scale_mu_kernel");
}

int wave_record(const mms_wave *w, int n, const float *u, hipStream_t s) {
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    const dim3 grid((unsigned)((w->g.nx + 255) / 256), (unsigned)w->g.ny);
    hipLaunchKernelGGL(record_kernel, grid, dim3(256), 0, s, u + o,
                       w->traces + (int64_t)n * w->g.ny * w->g.nx, (int)w->g.nx, (int)w->g.ny,
                       w->g.sy);
    return check_launch("record_kernel");
}

int dense_to_grid(const double *in, float *out, const mms_grid *g, double scale, hipStream_t s) {
    const int64_t o = (int64_t)g->halo * (g->sz + g->sy + 1);
    const dim3 grid((unsigned)((g->nx + 255) / 256), (unsigned)g->ny, (unsigned)g->nz);
    hipLaunchKernelGGL(dense_to_grid_kernel, grid, dim3(256), 0, s, in, out + o, (int)g->nx,
                       (int)g->ny, g->sy, g->sz, scale);
    return check_launch("dense_to_grid_kernel");
}

int wave_energy(const mms_wave *w, const float *un, const float *unp1, double *out, double *partials,
                hipStream_t s) {
    WaveArgs a = base_args(w);
    const int64_t o = (int64_t)w->g.halo * (w->g.sz + w->g.sy + 1);
    a.f0 = un + o;
    a.p0 = unp1 + o;
    a.partials = partials;
    fill_geom(a.g, &w->g);
    const int64_t nblk = (int64_t)a.g.ntx * a.g.nty * a.g.nzc;
    int rc = launch_mode<MODE_ENERGY>(a, &w->g, w->radius, s);
    if (rc) return rc;
    return finish_pairs(partials, (int)nblk, out, s);
}

int64_t wave_energy_blocks(const mms_wave *w) {
    Geom g{};
    fill_geom(g, &w->g);
    return (int64_t)g.ntx * g.nty * g.nzc;
}

}  // namespace mms
