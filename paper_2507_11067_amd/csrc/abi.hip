// C ABI of libmmstencil: argument checks, dispatch and error reporting.
// Every check runs on the host before any HIP call, so it is testable without
// a GPU.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>

#include "mms_internal.h"

namespace mms {

int wave_step(const mms_wave *w, int n, const float *up, const float *uc, float *un, hipStream_t s);
int wave_adjoint_step(const mms_wave *w, int n, const float *l2, const float *l1, float *l0,
                      const float *resid, const float *un, double *grad, hipStream_t s);
int wave_record(const mms_wave *w, int n, const float *u, hipStream_t s);
int wave_adjoint_mu_step(const mms_wave *w, int n, const float *m2, const float *m1, float *m0,
                         const float *resid, const float *un, double *grad, hipStream_t s);
int wave_scale_mu(const mms_wave *w, const float *in, float *out, int dir, hipStream_t s);
int wave_energy(const mms_wave *w, const float *un, const float *unp1, double *out, double *partials,
                hipStream_t s);
int64_t wave_energy_blocks(const mms_wave *w);
int dense_to_grid(const double *in, float *out, const mms_grid *g, double scale, hipStream_t s);
int tti_step(const mms_wave *w, const mms_tti *t, int n, const float *pp, const float *pc,
             float *pn, const float *qp, const float *qc, float *qn, hipStream_t s);
int vti_step(const mms_wave *w, int n, const float *fa, const float *fb, const float *hp,
             const float *hc, float *hn, const float *vp, const float *vc, float *vn,
             hipStream_t s);
int reduce_grid_dot(const float *a, const float *b, const mms_grid *g, double *out, double *part,
                    hipStream_t s);
int reduce_flat(const float *a, const float *b, float *resid, int64_t n, int misfit, double *out,
                double *part, hipStream_t s);
int flat_scale(const float *in, const double *scale, float *out, int64_t n, hipStream_t s);

namespace {
thread_local char g_last[256] = "";
}  // namespace

// Scratch of mms_wave_energy_noalloc: the energy kernel's per-block (partial sum,
// non-finite count) pairs, in a static device array instead of a caller workspace.
// Every GPU the library runs on holds its own copy (512 KiB) until the process ends.
constexpr int64_t kEnergyScratch = 1 << 16;  // doubles: grids of up to 32768 energy blocks
static __device__ __align__(256) double scratch[kEnergyScratch];

namespace {
// Device address of `scratch` per device: the host-side name is only a stand-in, so the
// address is looked up once per device (with that device current) and reused.
constexpr int kMaxDev = 64;
std::atomic<double *> g_scratch[kMaxDev];

int scratch_address(double **p) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDev) {
        snprintf(g_last, sizeof g_last, "device %d beyond the %d devices with a scratch address",
                 dev, kMaxDev);
        return MMS_EINVAL;
    }
    double *q = g_scratch[dev].load(std::memory_order_acquire);
    if (!q) {
        e = hipGetSymbolAddress((void **)&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!q) {
            snprintf(g_last, sizeof g_last, "hipGetSymbolAddress(scratch) gave a null address");
            return MMS_EHIP;
        }
        g_scratch[dev].store(q, std::memory_order_release);
    }
    *p = q;
    return MMS_OK;
}
}  // namespace

void set_last_error(const char *msg) { snprintf(g_last, sizeof g_last, "%s", msg); }

int hip_fail(hipError_t e, const char *where) {
    snprintf(g_last, sizeof g_last, "%s: %s", where, hipGetErrorString(e));
    return MMS_EHIP;
}

int check_launch(const char *where) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MMS_OK : hip_fail(e, where);
}

bool grid_ok(const mms_grid *g, int radius) {
    if (!g) return false;
    if (g->nx < 0 || g->ny < 0 || g->nz < 0) return false;
    if (g->nx > (1 << 30) || g->ny > (1 << 30) || g->nz > (1 << 30)) return false;
    if (g->halo < radius || g->halo < 4 || g->halo % 4 != 0) return false;
    const int64_t nx4 = (g->nx + 3) & ~(int64_t)3;
    if (g->sy % 4 != 0 || g->sy < nx4 + 2 * (int64_t)g->halo) return false;
    if (g->sz % 4 != 0 || g->sz < g->sy * (g->ny + 2 * (int64_t)g->halo)) return false;
    return true;
}

bool overlap(const void *a, int64_t abytes, const void *b, int64_t bbytes) {
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bbytes && pb < pa + abytes;
}

}  // namespace mms

using namespace mms;

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
static bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

// A reduction's result pair and its workspace: both present, 8-byte aligned, disjoint.
static bool reduce_buffers_ok(const double *out, const double *work, int64_t work_elems) {
    if (!out || !work || !aligned8(out) || !aligned8(work)) return false;
    return !overlap(out, 2 * (int64_t)sizeof(double), work, work_elems * (int64_t)sizeof(double));
}

extern "C" {

int mms_abi_version(void) { return MMS_ABI_VERSION; }

const char *mms_strerror(int code) {
    switch (code) {
        case MMS_OK: return "ok";
        case MMS_EINVAL: return "invalid argument";
        case MMS_EUNSUPPORTED: return "unsupported radius, shape or precision";
        case MMS_EHIP: return "HIP runtime error";
        case MMS_ENOMEM: return "out of device memory";
        case MMS_EUNSTABLE: return "non-finite values (NaN or Inf) in a reduction";
        default: return "unknown error";
    }
}

const char *mms_last_error(void) { return g_last; }

int mms_grid_aligned(int64_t nx, int64_t ny, int64_t nz, int32_t halo, mms_grid *g,
                     int64_t *lead) {
    if (!g || !lead || nx < 0 || ny < 0 || nz < 0 || halo < 4 || halo % 4 != 0) return MMS_EINVAL;
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30)) return MMS_EINVAL;
    const int64_t need = ((nx + 3) & ~(int64_t)3) + 2 * (int64_t)halo;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->halo = halo;
    g->pad_ = 0;
    g->sy = (need + 31) & ~(int64_t)31;
    g->sz = g->sy * (ny + 2 * (int64_t)halo);
    *lead = (32 - halo % 32) % 32;
    return MMS_OK;
}

int mms_stencil_apply(const float *in, float *out, const mms_grid *g, int shape, int radius,
                      const float *coeffs, int ncoeffs, int precision, void *stream) {
    if (radius < 1 || radius > 4) return MMS_EUNSUPPORTED;
    if (shape < MMS_STAR || shape > MMS_BOX2D) return MMS_EUNSUPPORTED;
    if (precision < MMS_FP32 || precision > MMS_BF16X1) return MMS_EUNSUPPORTED;
    if (shape != MMS_BOX && precision != MMS_FP32) return MMS_EUNSUPPORTED;
    if (!in || !out || !coeffs || !g) return MMS_EINVAL;
    if (!grid_ok(g, radius)) return MMS_EINVAL;
    if (!aligned16(in) || !aligned16(out)) return MMS_EINVAL;
    const int w = 2 * radius + 1;
    const int need[4] = {3 * w, w * w * w, 2 * w, w * w};
    if (ncoeffs != need[shape]) return MMS_EINVAL;
    const int64_t bytes = grid_elems(g) * (int64_t)sizeof(float);
    if (overlap(in, bytes, out, bytes)) return MMS_EINVAL;
    if (grid_empty(g)) return MMS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (shape == MMS_STAR) return launch_star(in, out, g, radius, coeffs, s);
    if (shape == MMS_STAR2D || shape == MMS_BOX2D)
        return launch_plane2d(in, out, g, shape, radius, coeffs, s);
    if (precision == MMS_FP32) return launch_box_valu(in, out, g, radius, coeffs, s);
    return launch_box_mfma(in, out, g, radius, coeffs, precision, s);
}

static int wave_ok(const mms_wave *w) {
    if (!w) return MMS_EINVAL;
    if (w->radius < 1 || w->radius > 4) return MMS_EUNSUPPORTED;
    if (!grid_ok(&w->g, w->radius) || !w->c2 || !aligned16(w->c2)) return MMS_EINVAL;
    if (w->sponge_width < 0 || w->nt < 0) return MMS_EINVAL;
    if (w->acc_block < 0) return MMS_EINVAL;
    if (w->image && w->acc_block > 1 && !w->acc_part) return MMS_EINVAL;
    if (w->src_dt2f && (w->src_z < 0 || w->src_z >= w->g.nz || w->src_y < 0 ||
                        w->src_y >= w->g.ny || w->src_x < 0 || w->src_x >= w->g.nx))
        return MMS_EINVAL;
    return MMS_OK;
}

int mms_wave_step(const mms_wave *w, int n, const float *u_prev, const float *u_cur, float *u_next,
                  void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!u_prev || !u_cur || !u_next) return MMS_EINVAL;
    if (!aligned16(u_prev) || !aligned16(u_cur) || !aligned16(u_next)) return MMS_EINVAL;
    if (n < 1 || n >= w->nt) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    if (overlap(u_cur, bytes, u_next, bytes)) return MMS_EINVAL;
    if (u_prev != u_next && overlap(u_prev, bytes, u_next, bytes)) return MMS_EINVAL;
    if (grid_empty(&w->g)) return MMS_OK;
    return wave_step(w, n, u_prev, u_cur, u_next, (hipStream_t)stream);
}

int mms_vti_step(const mms_wave *w, int n, const float *a, const float *b, const float *h_prev,
                 const float *h_cur, float *h_next, const float *v_prev, const float *v_cur,
                 float *v_next, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    const float *ins[] = {a, b, h_prev, h_cur, v_prev, v_cur};
    for (const float *p : ins)
        if (!p || !aligned16(p)) return MMS_EINVAL;
    if (!h_next || !v_next || !aligned16(h_next) || !aligned16(v_next)) return MMS_EINVAL;
    if (n < 1 || n >= w->nt) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    const float *cur[] = {h_cur, v_cur, a, b, w->c2};
    for (const float *p : cur)
        if (overlap(p, bytes, h_next, bytes) || overlap(p, bytes, v_next, bytes)) return MMS_EINVAL;
    if (overlap(h_next, bytes, v_next, bytes)) return MMS_EINVAL;
    if (h_prev != h_next && overlap(h_prev, bytes, h_next, bytes)) return MMS_EINVAL;
    if (v_prev != v_next && overlap(v_prev, bytes, v_next, bytes)) return MMS_EINVAL;
    if (overlap(h_prev, bytes, v_next, bytes) || overlap(v_prev, bytes, h_next, bytes))
        return MMS_EINVAL;
    if (grid_empty(&w->g)) return MMS_OK;
    return vti_step(w, n, a, b, h_prev, h_cur, h_next, v_prev, v_cur, v_next,
                    (hipStream_t)stream);
}

int mms_tti_step(const mms_wave *w, const mms_tti *t, int n, const float *p_prev,
                 const float *p_cur, float *p_next, const float *q_prev, const float *q_cur,
                 float *q_next, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!t) return MMS_EINVAL;
    const float *ins[] = {t->eps, t->delta, t->theta, t->phi, p_prev, p_cur, q_prev, q_cur};
    for (const float *p : ins)
        if (!p || !aligned16(p)) return MMS_EINVAL;
    if (!p_next || !q_next || !t->work || !aligned16(p_next) || !aligned16(q_next) ||
        !aligned16(t->work))
        return MMS_EINVAL;
    if (n < 1 || n >= w->nt) return MMS_EINVAL;
    if (!(t->alpha > 0.f) || !(t->sigma >= 0.f)) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    // every read-only operand against both outputs and the workspace
    const float *ro[] = {t->eps, t->delta, t->theta, t->phi, p_cur, q_cur, w->c2};
    for (const float *p : ro)
        if (overlap(p, bytes, p_next, bytes) || overlap(p, bytes, q_next, bytes) ||
            overlap(p, bytes, t->work, 4 * bytes))
            return MMS_EINVAL;
    if (overlap(p_next, bytes, q_next, bytes)) return MMS_EINVAL;
    if (overlap(p_next, bytes, t->work, 4 * bytes) || overlap(q_next, bytes, t->work, 4 * bytes))
        return MMS_EINVAL;
    if (overlap(p_prev, bytes, t->work, 4 * bytes) || overlap(q_prev, bytes, t->work, 4 * bytes))
        return MMS_EINVAL;
    if (p_prev != p_next && overlap(p_prev, bytes, p_next, bytes)) return MMS_EINVAL;
    if (q_prev != q_next && overlap(q_prev, bytes, q_next, bytes)) return MMS_EINVAL;
    if (overlap(p_prev, bytes, q_next, bytes) || overlap(q_prev, bytes, p_next, bytes))
        return MMS_EINVAL;
    if (grid_empty(&w->g)) return MMS_OK;
    return tti_step(w, t, n, p_prev, p_cur, p_next, q_prev, q_cur, q_next, (hipStream_t)stream);
}

int mms_wave_record(const mms_wave *w, int n, const float *u, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!u || !w->traces || n < 0 || n >= w->nt) return MMS_EINVAL;
    if (grid_empty(&w->g)) return MMS_OK;
    return wave_record(w, n, u, (hipStream_t)stream);
}

int mms_wave_forward(const mms_wave *w, int n_begin, int n_end, float *const *states, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!states || n_begin < 1 || n_end > w->nt || n_end < n_begin) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    for (int n = n_begin; n < n_end; ++n) {
        const int i = n - n_begin;  // states[i] = u^{n-1}, states[i+1] = u^n, states[i+2] = u^{n+1}
        float *up = states[i], *uc = states[i + 1], *un = states[i + 2];
        if (!up || !uc || !un) return MMS_EINVAL;
        if (overlap(uc, bytes, un, bytes)) return MMS_EINVAL;
        if (up != un && overlap(up, bytes, un, bytes)) return MMS_EINVAL;
    }
    for (int n = n_begin; n < n_end; ++n) {
        const int i = n - n_begin;
        if (int rc = mms_wave_step(w, n, states[i], states[i + 1], states[i + 2], stream)) return rc;
    }
    return MMS_OK;
}

int mms_wave_adjoint_step(const mms_wave *w, int n, const float *lam_np2, const float *lam_np1,
                          float *lam_n, const float *resid, const float *u_n, double *grad,
                          void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (n < 0 || n >= w->nt || !lam_np2 || !lam_n) return MMS_EINVAL;
    if (n >= 1 && !lam_np1) return MMS_EINVAL;
    if (n >= 1 && grad && !u_n) return MMS_EINVAL;
    if (n >= 1 && grad && w->acc_block > 1 && !w->acc_part) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    if (lam_np1 && overlap(lam_np1, bytes, lam_n, bytes)) return MMS_EINVAL;
    if (lam_np2 != lam_n && overlap(lam_np2, bytes, lam_n, bytes)) return MMS_EINVAL;
    if (u_n && overlap(u_n, bytes, lam_n, bytes)) return MMS_EINVAL;
    if (grid_empty(&w->g)) return MMS_OK;
    return wave_adjoint_step(w, n, lam_np2, lam_np1, lam_n, resid, u_n, grad, (hipStream_t)stream);
}

int mms_wave_adjoint(const mms_wave *w, int n_hi, int n_lo, float *const *lams,
                     const float *const *us, const float *resid, double *grad, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!lams || n_lo < 0 || n_hi >= w->nt || n_hi < n_lo) return MMS_EINVAL;
    if (grad && !us) return MMS_EINVAL;
    for (int n = n_hi; n >= n_lo; --n) {
        const int i = n - n_lo;  // lams[i] = lam^n, lams[i+1] = lam^{n+1}, lams[i+2] = lam^{n+2}
        const float *un = (grad && n >= 1) ? us[i] : nullptr;
        const float *rs = resid;
        int rc = mms_wave_adjoint_step(w, n, lams[i + 2], lams[i + 1], lams[i], rs, un, grad, stream);
        if (rc) return rc;
    }
    return MMS_OK;
}

int mms_wave_adjoint_mu(const mms_wave *w, int n_hi, int n_lo, float *const *mus,
                        const float *const *us, const float *resid, double *grad, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!mus || n_lo < 0 || n_hi >= w->nt || n_hi < n_lo) return MMS_EINVAL;
    if (grad && !us) return MMS_EINVAL;
    if (grad && w->acc_block > 1 && !w->acc_part) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    // every step's buffers first, so that a bad entry changes nothing
    for (int n = n_hi; n >= n_lo; --n) {
        const int i = n - n_lo;   // mus[i] = mu^n, mus[i+1] = mu^{n+1}, mus[i+2] = mu^{n+2}
        const float *m2 = mus[i + 2], *m1 = mus[i + 1];
        float *m0 = mus[i];
        if (!m2 || !m0 || (n >= 1 && !m1)) return MMS_EINVAL;
        const float *un = (grad && n >= 1) ? us[i] : nullptr;
        if (grad && n >= 1 && !un) return MMS_EINVAL;
        if (m1 && n >= 1 && overlap(m1, bytes, m0, bytes)) return MMS_EINVAL;
        if (m2 != m0 && overlap(m2, bytes, m0, bytes)) return MMS_EINVAL;
        if (un && overlap(un, bytes, m0, bytes)) return MMS_EINVAL;
    }
    if (grid_empty(&w->g)) return MMS_OK;
    hipStream_t s = (hipStream_t)stream;
    for (int n = n_hi; n >= n_lo; --n) {
        const int i = n - n_lo;
        const float *un = (grad && n >= 1) ? us[i] : nullptr;
        int rc = wave_adjoint_mu_step(w, n, mus[i + 2], mus[i + 1], mus[i], resid, un,
                                      n >= 1 ? grad : nullptr, s);
        if (rc) return rc;
    }
    return MMS_OK;
}

int mms_wave_scale_mu(const mms_wave *w, const float *in, float *out, int dir, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!in || !out || (dir != 1 && dir != -1)) return MMS_EINVAL;
    const int64_t bytes = grid_elems(&w->g) * (int64_t)sizeof(float);
    if (in != out && overlap(in, bytes, out, bytes)) return MMS_EINVAL;
    if (grid_empty(&w->g)) return MMS_OK;
    return wave_scale_mu(w, in, out, dir, (hipStream_t)stream);
}

int mms_wave_energy_work(const mms_wave *w, int64_t *elems) {
    if (int rc = wave_ok(w)) return rc;
    if (!elems) return MMS_EINVAL;
    *elems = grid_empty(&w->g) ? 0 : 2 * wave_energy_blocks(w);
    return MMS_OK;
}

int mms_wave_energy(const mms_wave *w, const float *u_n, const float *u_np1, double *out_dev,
                    double *work, int64_t work_elems, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!u_n || !u_np1) return MMS_EINVAL;
    int64_t need = 0;
    if (int rc = mms_wave_energy_work(w, &need)) return rc;
    if (work_elems < need || need > (int64_t)0x7fffffff) return MMS_EINVAL;
    if (!out_dev || !aligned8(out_dev) || (need > 0 && !reduce_buffers_ok(out_dev, work, need)))
        return MMS_EINVAL;
    if (grid_empty(&w->g)) return fill_pair(out_dev, 0.0, (hipStream_t)stream);
    return wave_energy(w, u_n, u_np1, out_dev, work, (hipStream_t)stream);
}

int mms_dense_to_grid(const double *in, float *out, const mms_grid *g, double scale, void *stream) {
    if (!in || !out || !grid_ok(g, 1)) return MMS_EINVAL;
    if (g->ny > 65535 || g->nz > 65535) return MMS_EINVAL;
    if (grid_empty(g)) return MMS_OK;
    return dense_to_grid(in, out, g, scale, (hipStream_t)stream);
}

int mms_wave_energy_noalloc(const mms_wave *w, const float *u_n, const float *u_np1,
                            double *out_dev, void *stream) {
    if (int rc = wave_ok(w)) return rc;
    if (!u_n || !u_np1 || !out_dev || !aligned8(out_dev)) return MMS_EINVAL;
    int64_t need = 0;
    if (int rc = mms_wave_energy_work(w, &need)) return rc;
    if (need > kEnergyScratch) {
        snprintf(g_last, sizeof g_last,
                 "mms_wave_energy_noalloc: the grid needs %lld doubles of scratch, the static "
                 "scratch holds %lld (use mms_wave_energy with a workspace)",
                 (long long)need, (long long)kEnergyScratch);
        return MMS_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (grid_empty(&w->g)) return fill_pair(out_dev, 0.0, s);
    double *ptr = nullptr;
    if (int rc = scratch_address(&ptr)) return rc;
    return wave_energy(w, u_n, u_np1, out_dev, ptr, s);
}

int mms_dot_f64(const float *a, const float *b, const mms_grid *g, double *out_dev, double *work,
                void *stream) {
    if (!a || !grid_ok(g, 1)) return MMS_EINVAL;
    if (!reduce_buffers_ok(out_dev, work, MMS_REDUCE_WORK)) return MMS_EINVAL;
    return reduce_grid_dot(a, b, g, out_dev, work, (hipStream_t)stream);
}

int mms_flat_dot_f64(const float *a, const float *b, int64_t n, double *out_dev, double *work,
                     void *stream) {
    if (!a || n < 0) return MMS_EINVAL;
    if (!reduce_buffers_ok(out_dev, work, MMS_REDUCE_WORK)) return MMS_EINVAL;
    return reduce_flat(a, b, nullptr, n, 0, out_dev, work, (hipStream_t)stream);
}

int mms_flat_misfit_f64(const float *a, const float *b, float *resid, int64_t n, double *out_dev,
                        double *work, void *stream) {
    if (!a || !b || n < 0) return MMS_EINVAL;
    if (!reduce_buffers_ok(out_dev, work, MMS_REDUCE_WORK)) return MMS_EINVAL;
    return reduce_flat(a, b, resid, n, 1, out_dev, work, (hipStream_t)stream);
}

int mms_flat_scale_f32(const float *in, const double *scale_dev, float *out, int64_t n,
                       void *stream) {
    if (!scale_dev || n < 0 || !aligned8(scale_dev)) return MMS_EINVAL;
    if (n == 0) return MMS_OK;
    if (!in || !out) return MMS_EINVAL;
    const int64_t bytes = n * (int64_t)sizeof(float);
    if (in != out && overlap(in, bytes, out, bytes)) return MMS_EINVAL;
    return flat_scale(in, scale_dev, out, n, (hipStream_t)stream);
}

int mms_check_reduction(const double *result) {
    if (!result) return MMS_EINVAL;
    if (result[1] != 0.0 || !isfinite(result[0])) return MMS_EUNSTABLE;
    return MMS_OK;
}

}  // extern "C"
