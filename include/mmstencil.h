/*
 * mmstencil.h -- C ABI of the MI355X (gfx950) high-order stencil library.
 *
 * The library computes the hot path of MMStencil (arXiv 2507.11067): sweeps of
 * 3-D high-order FP32 stencils over a regular grid (the star and box patterns
 * of the problem statement in Sec. I; radius 4 is the 8th-order case of
 * Sec. II-A) and the acoustic wave time step those sweeps drive in reverse-time
 * migration (Sec. II-A, Sec. V-F), with its exact discrete adjoint and the
 * gradient of a receiver misfit with respect to C2 = (v dt / h)^2.
 *
 * Conventions shared by every entry point
 *  - Grid, field and workspace pointers are DEVICE pointers owned by the
 *    caller.  The library keeps no reference after a call returns, allocates no
 *    device memory and holds no mutable state other than the thread-local text
 *    of the last HIP error: every scratch buffer a kernel needs (partial sums,
 *    block partials, intermediate fields) is a workspace argument.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the default stream).  Errors found by the host-side checks are
 *    returned before anything is enqueued; launch failures return MMS_EHIP.
 *  - Return value 0 means success; negative values are the MMS_E* codes below.
 *    No exception crosses the ABI.  Calls from different threads or on
 *    different streams may run concurrently as long as no buffer that one of
 *    them writes (outputs and workspaces) is read or written by another.
 *  - Grid layout (mms_grid): FP32 elements, x fastest.  Interior point (z,y,x),
 *    0 <= z < nz etc., is element (z+H)*sz + (y+H)*sy + (x+H) of the array.
 *    Requirements (MMS_EINVAL otherwise): nx, ny, nz >= 0; H >= radius and
 *    H % 4 == 0; sy % 4 == 0 and sy >= roundup4(nx) + 2H; sz % 4 == 0 and
 *    sz >= sy * (ny + 2H); base pointer 16-byte aligned.  The array therefore
 *    holds (nz + 2H) * sz elements.  Halo cells are read as stored and never
 *    written; the workloads keep them zero (a zero-halo boundary).
 *  - FP64 outputs (image, gradient) are dense interior arrays [nz][ny][nx].
 */
#ifndef MMSTENCIL_H
#define MMSTENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MMS_ABI_VERSION 4   /* 4: caller-owned reduction workspaces, (sum, non-finite count)
                               result pairs, mms_flat_scale_f32, mms_check_reduction;
                               the z-chunk tuning call is gone */

/* error codes */
#define MMS_OK 0
#define MMS_EINVAL (-1)       /* null pointer, bad layout, bad sizes, aliasing   */
#define MMS_EUNSUPPORTED (-2) /* radius outside 1..4, unknown shape, split precision other than on a 3-D box,
                                 an FP32 box over rows too long for its tile offsets */
#define MMS_EHIP (-3)         /* HIP runtime or launch error (see mms_last_error)*/
#define MMS_ENOMEM (-4)       /* reserved: no call of this version allocates      */
#define MMS_EUNSTABLE (-5)    /* a reduction result reports NaN or Inf values     */
                              /* (returned by mms_check_reduction)               */

/* stencil shapes (Sec. I: star = axes only, box = full (2r+1)^d cube; the 2-D
   shapes are the 2DStar / 2DBox kernels of Table I, applied to every z-plane) */
#define MMS_STAR 0
#define MMS_BOX 1
#define MMS_STAR2D 2
#define MMS_BOX2D 3

/* arithmetic of a box sweep */
#define MMS_FP32 0     /* FP32 FMA on the vector ALUs                                 */
#define MMS_BF16X3 1   /* MFMA, BF16 hi+lo split of data and weights, 3 products,   */
                       /* FP32 accumulation                                          */
#define MMS_FP16X3S 2  /* MFMA, FP16 hi+lo split with a power-of-two scale per      */
                       /* thread block (data) and per call (weights), 3 products    */
#define MMS_BF16X1 3   /* MFMA, BF16 hi*hi only: reduced-accuracy reference variant  */

typedef struct mms_grid {
    int64_t nx, ny, nz; /* interior extent                                   */
    int32_t halo;       /* H: halo width, >= radius, multiple of 4          */
    int32_t pad_;       /* unused, keep 0                                   */
    int64_t sy, sz;     /* element strides of y and z (x stride is 1)       */
} mms_grid;

/*
 * mms_stencil_apply -- one out-of-place sweep, out = S(in) on the interior.
 * Definition (Sec. I problem statement, Fig. 1 patterns):
 *   star: out(p) = sum_{axis a} sum_{k=-r..r} coeffs[a][k+r] * in(p + k e_a),
 *         coeffs is [3][2r+1] with axis order z, y, x (ncoeffs = 3(2r+1));
 *   box:  out(p) = sum_{dz,dy,dx} coeffs[dz+r][dy+r][dx+r] * in(p + (dz,dy,dx)),
 *         ncoeffs = (2r+1)^3;
 *   star2d: out(z,y,x) = sum_k coeffs[0][k+r] in(z,y+k,x) + sum_k coeffs[1][k+r] in(z,y,x+k),
 *         ncoeffs = 2(2r+1) (axis y, then x); no z neighbour is read;
 *   box2d: out(z,y,x) = sum_{dy,dx} coeffs[dy+r][dx+r] in(z,y+dy,x+dx), ncoeffs = (2r+1)^2.
 * in, out: device grids with the same layout g; out's halo is not written; in
 * and out must not overlap (MMS_EINVAL).  coeffs: HOST pointer, read during the
 * call only.  radius: 1..4.  precision: MMS_FP32 for the star and the 2-D
 * shapes; any of the four for the box.  The box MFMA variants recast each (dz, dy) pair of the sweep as
 * a banded Toeplitz product along x, the matrix-unit mapping of Sec. IV-A, with
 * the (2r+1)^2 one-dimensional stencils of the box decomposition of Sec. IV-C.
 * An FP32 box of radius 2-4 addresses a tile of (32 + 2r + 1) rows with 32-bit
 * offsets: a pitch sy with (33 + 2r) * sy >= 2^32 gives MMS_EUNSUPPORTED.
 */
int mms_stencil_apply(const float *in, float *out, const mms_grid *g, int shape, int radius,
                      const float *coeffs, int ncoeffs, int precision, void *stream);

/*
 * Acoustic problem description for the wave entry points.  The time step is
 * the leapfrog update that RTM is built on (Sec. II-A), with an absorbing
 * sponge G and a point source:
 *   u^{n+1} = G (2 u^n - G u^{n-1} + C2 S(u^n)) + src_dt2f[n] delta_src
 * S is the star with per-axis symmetric weights lap (unit spacing), C2 =
 * (v dt / h)^2 = c2_scale * c2[cell].  G(z,y,x) = gz(z) gy(y) gx(x) with g(d) = exp(-(alpha (W-d))^2)
 * for a cell at distance d < W from a damped face and 1 elsewhere.
 */
typedef struct mms_wave {
    mms_grid g;
    int32_t radius;       /* 1..4                                                   */
    float lap[5];         /* per-axis weights: centre, then k = 1..radius           */
    const float *c2;      /* device grid (layout g), zero halo: C2 = c2_scale * c2   */
    float c2_scale;       /* 1 when c2 holds C2; dt^2 / h^2 when it holds v^2       */
    int32_t sponge_width; /* W >= 0 cells                                           */
    float sponge_alpha;   /* alpha                                                  */
    int32_t sponge_faces; /* bit mask: 1 x-lo, 2 x-hi, 4 y-lo, 8 y-hi, 16 z-lo,     */
                          /* 32 z-hi (z-lo is the top, z = 0)                       */
    int32_t nt;           /* number of time levels 0..nt-1 recorded                 */
    int64_t src_z, src_y, src_x; /* interior index of the point source              */
    const float *src_dt2f;/* device [nt]: dt^2 f(n dt), or NULL for no source       */
    float *traces;        /* device [nt][ny][nx]: d^n = u^n(z = 0), or NULL          */
    double *image;        /* device [nz][ny][nx] FP64: += (u^{n+1})^2, or NULL       */
    float *acc_part;      /* device [nz][ny][nx] FP32 workspace for acc_block > 1    */
    int32_t acc_block;    /* K for the FP64 accumulations (the image in forward steps, */
                          /* the gradient in adjoint steps): 0 or 1 adds every step's  */
                          /* term in FP64; K > 1 sums the terms of each block of K     */
                          /* consecutive steps in FP32 in acc_part and adds that sum   */
                          /* in FP64 at the block's last step                          */
    int32_t pad_;         /* unused, keep 0                                          */
} mms_wave;

/*
 * mms_wave_step -- one forward step n (1 <= n < nt): u_next = u^{n+1} from
 * u_prev = u^{n-1}, u_cur = u^n; records traces[n] = u^n(z = 0) and adds
 * (u^{n+1})^2 to image when those are set.  With acc_block = K > 1 the image holds
 * every term of steps 1..n once n is a multiple of K or n = nt-1 (forward blocks are
 * steps 1+jK .. (j+1)K; each is summed in FP32, relative error <= K 2^-24, and added
 * in FP64); the steps of a block must run in order.  u_next may equal u_prev (the update
 * reads and writes each cell in place); u_next must not overlap u_cur.
 */
int mms_wave_step(const mms_wave *w, int n, const float *u_prev, const float *u_cur,
                  float *u_next, void *stream);

/*
 * mms_wave_record -- traces[n] = u(z = 0): the receiver reading of a level that
 * no step produces from the recurrence (level 0).
 */
int mms_wave_record(const mms_wave *w, int n, const float *u, void *stream);

/*
 * mms_wave_forward -- steps n = n_begin .. n_end-1 in one call.
 * states[i] holds u^{n_begin-1+i} for i = 0 .. n_end-n_begin+1: entries 0 and 1
 * are inputs, the rest are outputs.  Entries may repeat (three buffers used in
 * rotation, or two with u_next = u_prev) as long as step n never writes the
 * buffer that holds u^n.  states is a HOST array of device pointers.
 */
int mms_wave_forward(const mms_wave *w, int n_begin, int n_end, float *const *states,
                     void *stream);

/*
 * mms_wave_adjoint_step -- one step n of the exact discrete adjoint of the
 * recurrence above (the transpose of the state map (u^n, u^{n-1}) ->
 * (u^{n+1}, u^n); the paper has no adjoint).  For n >= 1:
 *   lam^n = 2 G lam^{n+1} - G^2 lam^{n+2} + S^T(C2 G lam^{n+1}) + R^T resid[n]
 *   grad += c2_scale G lam^{n+1} S(u^n)     (FP64, dense [nz][ny][nx])
 * For n = 0: lam^0 = -G^2 lam^2 + R^T resid[0] (no gradient term).
 * R^T adds resid[n] ([ny][nx], device, may be NULL) to the plane z = 0.  u_n is
 * needed when grad is set and n >= 1.  lam_n may equal lam_np2.
 * grad is dJ/d(c2 field): dJ/dC2 for c2_scale = 1, dJ/d(v^2) for c2_scale =
 * dt^2 / h^2.  With acc_block = K > 1 the gradient terms of each block of K steps,
 * counted down from n = nt-1 (n = nt-1-jK .. nt-K-jK), are summed in FP32 in acc_part
 * and added to grad in FP64 at the block's last step and at n = 1; the steps of a
 * block must run in order.
 */
int mms_wave_adjoint_step(const mms_wave *w, int n, const float *lam_np2, const float *lam_np1,
                          float *lam_n, const float *resid, const float *u_n, double *grad,
                          void *stream);

/*
 * mms_wave_adjoint -- adjoint steps n = n_hi down to n_lo in one call.
 * lams[i] holds lam^{n_lo+i} for i = 0 .. n_hi-n_lo+2 (the last two are inputs);
 * us[i] holds u^{n_lo+i} for i = 0 .. n_hi-n_lo (read for n >= 1 when grad is
 * set).  resid is the whole [nt][ny][nx] residual (device) or NULL.  Both
 * pointer arrays live on the host; entries may repeat as for mms_wave_forward.
 */
int mms_wave_adjoint(const mms_wave *w, int n_hi, int n_lo, float *const *lams,
                     const float *const *us, const float *resid, double *grad, void *stream);

/*
 * mms_vti_step -- one step n (1 <= n < nt) of the pseudo-acoustic VTI pair that RTM
 * in VTI media runs (Sec. II-A).  The paper prints a sigma_H / sigma_V system whose
 * second equation, as printed, is ill-posed; the TTI system printed next to it
 * reduces, for zero tilt, zero shear velocity and alpha = sqrt(1 + 2 delta), to
 *   H^{n+1} = G (2 H^n - G H^{n-1} + C2 (a Sxy H^n + b Szz V^n)) + src_dt2f[n] delta_src
 *   V^{n+1} = G (2 V^n - G V^{n-1} + C2 (b Sxy H^n +   Szz V^n)) + src_dt2f[n] delta_src
 * which is what this computes.  a = 1 + 2 epsilon, b = sqrt(1 + 2 delta): device grids
 * (layout g).  Sxy = Sxx + Syy and Szz are the axis parts of the star with weights
 * w->lap; C2, G, the source and dt as in mms_wave_step; traces[n] = H^n(z = 0); the
 * image is not used.  h_next may equal h_prev and v_next may equal v_prev; neither may
 * overlap h_cur or v_cur.
 *  The H tile of (8 + 2r + 1) rows is addressed with 32-bit offsets: a pitch sy with
 * (9 + 2r) * sy >= 2^32 gives MMS_EUNSUPPORTED.
 */
int mms_vti_step(const mms_wave *w, int n, const float *a, const float *b, const float *h_prev,
                 const float *h_cur, float *h_next, const float *v_prev, const float *v_cur,
                 float *v_next, void *stream);

/*
 * Medium of the pseudo-acoustic TTI pair (Sec. II-A) for mms_tti_step.
 */
typedef struct mms_tti {
    const float *eps, *delta;  /* Thomsen parameters, device grids (layout g)             */
    const float *theta, *phi;  /* tilt of the symmetry axis from z and its azimuth from x,  */
                               /* radians, device grids (layout g); |angle| < 1600 (sine   */
                               /* and cosine come from the transcendental unit, absolute   */
                               /* error below 1e-6)                                         */
    float sigma;               /* v_sz^2 / v_pz^2 (0 gives the pure pseudo-acoustic pair)   */
    float alpha;               /* scale of q in the coupling, > 0                           */
    float d1[4];               /* first-derivative weights d_1..d_radius:                   */
                               /* D f(i) = sum_k d_k (f(i+k) - f(i-k))                       */
    float *work;               /* device workspace of 4 grids (layout g, 16-byte aligned),  */
                               /* overwritten by every call; caller-owned                   */
} mms_tti;

/*
 * mms_tti_step -- one step n (1 <= n < nt) of the pseudo-acoustic TTI pair (Sec. II-A),
 * in units of C2 = (v_pz dt / h)^2 (C2 and the rest of the problem from w):
 *   p'' = C2 [ (1+2eps) H2 p + alpha H1 q + sigma H1 (p - alpha q) ]
 *   q'' = C2 [ ((1+2delta)/alpha) H2 p + H1 q - sigma H2 (p/alpha - q) ]
 *   H1 = (n . grad)^2, n = (sin(theta) cos(phi), sin(theta) sin(phi), cos(theta)) in (x, y, z),
 *   H2 = Dxx + Dyy + Dzz - H1,
 * stepped as u^{n+1} = G (2 u^n - G u^{n-1} + u'') + src_dt2f[n] delta_src for u = p, q.
 * Dxx, Dyy, Dzz use the per-axis weights w->lap; the mixed derivatives are products of the
 * first-derivative stencil t->d1 along the two axes (the composition of one-dimensional
 * stencils of Sec. IV-G).  traces[n] = p^n(z = 0); the image is not used.  Grid cells are read
 * as stored, halo included.  p_next may equal p_prev and q_next may equal q_prev; no other
 * pair of arguments (work included) may overlap.  The second pass addresses tiles of
 * (8 + 2r + 1) rows with 32-bit offsets: a pitch sy with (9 + 2r) * sy >= 2^32 gives
 * MMS_EUNSUPPORTED before either pass runs.
 */
int mms_tti_step(const mms_wave *w, const mms_tti *t, int n, const float *p_prev,
                 const float *p_cur, float *p_next, const float *q_prev, const float *q_cur,
                 float *q_next, void *stream);

/*
 * mms_wave_adjoint_mu -- the steps n_hi .. n_lo of mms_wave_adjoint carried in the
 * scaled variable mu = C2 G lam (C2 = c2_scale c2, G the sponge factor).  The exact
 * discrete adjoint of the previous section then has the forward step's form, with one
 * stencil operand:
 *   mu^n = G (2 mu^{n+1} - G mu^{n+2} + C2 S(mu^{n+1})) + C2 G R^T resid[n]   (n >= 1)
 *   mu^0 = -G^2 mu^2 + C2 G R^T resid[0]
 * mus[i] holds mu^{n_lo+i}; entries n_hi-n_lo+1 and n_hi-n_lo+2 are inputs, the rest are
 * outputs (a HOST array of device pointers; entries may repeat as in mms_wave_adjoint).
 * With grad: grad += c2_scale G lam^{n+1} S(u^n) for n = max(n_lo, 1) .. n_hi, the same
 * terms as mms_wave_adjoint, formed as mu^{n+1} S(u^n) / c2; acc_block blocks as there.
 * The FP32 block partial holds mu^{n+1} S(u^n) sums, and the division by c2 (in FP64)
 * happens where a sum is added to grad, so the c2 field is read once per block rather
 * than every step.  A block begun by this call must therefore be finished by calls of
 * this entry point (and one begun by mms_wave_adjoint by that one).  grad holds only
 * finished terms between calls.  Requires c2 > 0 in every interior cell
 * (lam = mu / (C2 G)); results are undefined otherwise.  Buffers are checked before
 * anything is enqueued.
 */
int mms_wave_adjoint_mu(const mms_wave *w, int n_hi, int n_lo, float *const *mus,
                        const float *const *us, const float *resid, double *grad, void *stream);

/*
 * mms_wave_scale_mu -- out = C2 G in (dir = +1: lam -> mu) or out = in / (C2 G)
 * (dir = -1: mu -> lam) on the interior; out may equal in, and must not otherwise
 * overlap it.  Halo cells of out are left unchanged.  dir = -1 requires c2 > 0.
 */
int mms_wave_scale_mu(const mms_wave *w, const float *in, float *out, int dir, void *stream);

/*
 * FP64 reductions of FP32 data.  A fixed number of blocks strides over the data
 * in a fixed order and writes one (partial sum, non-finite count) pair each into
 * a caller-owned device workspace; one block then sums the pairs in a fixed tree
 * (no atomics, so a result is bit-reproducible).  Every reduction writes a result
 * PAIR to out_dev (device, 2 doubles, 8-byte aligned, disjoint from the
 * workspace): out_dev[0] = the FP64 sum, out_dev[1] = the number of terms that
 * were NaN or +-Inf, plus one if the sum itself is not finite (0 for a clean
 * result; mms_check_reduction turns the pair into MMS_OK or MMS_EUNSTABLE).
 * Two reductions may run at once (other streams, other threads) when their
 * workspaces and result pairs are distinct.
 */
#define MMS_REDUCE_WORK 2048  /* doubles of workspace for the flat and grid reductions */

/*
 *   mms_dot_f64:      sum over the interior of a*b (b == NULL: a*a)
 *   mms_flat_dot_f64: sum_i a[i]*b[i] over n contiguous elements (b == NULL: a*a)
 *   mms_flat_misfit_f64: 0.5 * sum_i (a[i]-b[i])^2, and resid[i] = a[i]-b[i]
 *                     when resid is non-NULL (may equal a)
 * work: device, MMS_REDUCE_WORK doubles, overwritten.  MMS_EINVAL for a null
 * input, result or workspace, a misaligned result or workspace, or a result that
 * overlaps the workspace.
 */
int mms_dot_f64(const float *a, const float *b, const mms_grid *g, double *out_dev, double *work,
                void *stream);
int mms_flat_dot_f64(const float *a, const float *b, int64_t n, double *out_dev, double *work,
                     void *stream);
int mms_flat_misfit_f64(const float *a, const float *b, float *resid, int64_t n, double *out_dev,
                        double *work, void *stream);

/*
 * mms_wave_energy -- FP64 discrete energy of the leapfrog scheme without
 * sponge or source, E^{n+1/2} = sum (u^{n+1}-u^n)^2 / C2 - <u^{n+1}, S u^n>,
 * which the scheme conserves exactly for a symmetric S, so growth of E is the
 * signature of an unstable run (a time step beyond the CFL limit).  The result
 * pair goes to out_dev as for the reductions above.  Cells with C2 == 0 add only
 * the second term.  work: device workspace of at least the number of doubles
 * that mms_wave_energy_work reports for w (it depends on the grid only).
 */
int mms_wave_energy_work(const mms_wave *w, int64_t *elems);
int mms_wave_energy(const mms_wave *w, const float *u_n, const float *u_np1, double *out_dev,
                    double *work, int64_t work_elems, void *stream);

/*
 * mms_wave_energy_noalloc -- mms_wave_energy for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the per-block partials go to a static device array
 * of 65536 doubles (512 KiB) that every GPU the library runs on holds until the process
 * ends.  Grids whose energy needs more than that (mms_wave_energy_work > 65536, i.e.
 * more than 32768 blocks) are refused with MMS_EINVAL before anything is enqueued, and
 * mms_last_error names the sizes.  The call allocates nothing.  Every call on one GPU
 * uses that GPU's array, so calls that overlap on one GPU (other streams, other
 * threads) race and may return wrong sums; calls in stream order are safe (each call
 * writes every partial it reads).  The first call on a device looks up the array's
 * address there (hipGetSymbolAddress).
 */
int mms_wave_energy_noalloc(const mms_wave *w, const float *u_n, const float *u_np1,
                            double *out_dev, void *stream);

/*
 * mms_check_reduction -- host helper: MMS_EUNSTABLE if a reduction's result pair
 * (copied to the host) reports non-finite terms or a non-finite sum, MMS_OK
 * otherwise, MMS_EINVAL for NULL.
 */
int mms_check_reduction(const double *result_host);

/*
 * mms_flat_scale_f32 -- out[i] = (float)(scale * in[i]) for i < n, with the FP64 scale
 * read on the device from *scale_dev (so a scale that an earlier kernel produced needs
 * no copy to the host).  This is the chain-rule step of a misfit's gradient: the
 * residual times the upstream derivative.  out may equal in; with n = 0 nothing is read
 * and in and out may be NULL.
 */
int mms_flat_scale_f32(const float *in, const double *scale_dev, float *out, int64_t n,
                       void *stream);

/*
 * mms_dense_to_grid -- out(z,y,x) = (float)(scale * in[z][y][x]) on the interior
 * of a device grid (halo untouched); in is a dense FP64 device array.  Turns an
 * FP64 gradient into the layout of the field it belongs to.
 */
int mms_dense_to_grid(const double *in, float *out, const mms_grid *g, double scale, void *stream);

/*
 * mms_grid_aligned -- host helper: fill *g with the layout whose interior rows
 * start on 128-byte boundaries, and return in *lead the number of elements to
 * place in front of the array.  sy = roundup(roundup4(nx) + 2H, 32),
 * sz = sy (ny + 2H), lead = (32 - H % 32) % 32.  An array that starts lead
 * elements after a 128-byte aligned address (device allocators return at least
 * that) has interior point (z, y, 0) on a 128-byte boundary for every z, y, so
 * a sweep's output rows cover whole cache lines whenever 4 nx is a multiple of
 * 128 (no partial-line writes).  Allocate lead + (nz + 2H) sz elements.  Any
 * other layout that meets the mms_grid requirements stays valid; this one is
 * faster for the memory-bound sweeps.  Returns MMS_EINVAL for a null output,
 * negative extents, or a halo that is not a positive multiple of 4.
 */
int mms_grid_aligned(int64_t nx, int64_t ny, int64_t nz, int32_t halo, mms_grid *g,
                     int64_t *lead);

const char *mms_strerror(int code);
const char *mms_last_error(void); /* text of the last MMS_EHIP on this thread, or of a */
                                  /* size refusal of mms_wave_energy_noalloc            */
int mms_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MMSTENCIL_H */
