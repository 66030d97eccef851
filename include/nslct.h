/*
 * nslct.h -- C ABI of the MI355X (gfx950) 2D nonseparable discrete linear
 * canonical transform by the CM-CC-CM-CC decomposition of Pei & Huang,
 * "Two-dimensional nonseparable discrete linear canonical transform based on
 * CM-CC-CM-CC decomposition".
 *
 * What is computed
 *   For a 4x4 ABCD matrix M = (A, B; C, D) with M J M^T = J (Sec. 1,
 *   eq. Intro12) the forward transform is the high-accuracy NsDLCT
 *     type 1 (CM-CC-CM-CC, Sec. 4.2.1, eq. HA28):
 *       G = CM(P1) CC(B') CM(P3) CC(H) g
 *     type 2 (CC-CM-CC-CM, Sec. 4.3, eq. CCCMCCCM40):
 *       G = CC(H1) CM(Q1) CC(B1') CM(Q3) g
 *   with the discrete chirp multiplication CM (Sec. 2.1, eq. BasicCM12) and
 *   chirp convolution CC(B) = F^-1 CM(-B) F (Sec. 2.3, eq. BasicCC20), the DFTs
 *   carrying the constants of eqs. BasicDFT16/20.  The type follows the sign of
 *   tr B (Sec. 4.4, eq. Reversible08) unless overridden; the gauge H (H1) is
 *   the minimiser of the phase-space growth product of eq. HA24.
 *   The chain equals a unitary operator L; nslct_inverse applies L^H = L^-1,
 *   the reversed chain with negated stage matrices (eq. CCCMCCCM30).
 *   On request the reduced decompositions are planned instead: CM-CC-CM for
 *   a symmetric invertible B (Sec. 4.1, eq. Bsym12) and the low-complexity
 *   LC-NsDLCT with a rank-one gauge (Sec. 4.2.2, eq. LC12), three passes
 *   over the image instead of five (see nslct_opts.type_override).
 *
 * Data layout (all entry points)
 *   An image is Nx*Ny interleaved complex numbers (re, im), row-major
 *   [Nx][Ny]: element [m][n] holds g(x_m, y_n) with n contiguous.  Sample
 *   indices are centred: x_m = (m - floor(Nx/2)) * dx, y_n = (n - floor(Ny/2)) * dy.
 *   Output uses the same grid (spacings dx, dy), as in the paper's
 *   experiments.  Precision NSLCT_C64 uses float (8 bytes per sample),
 *   NSLCT_C128 uses double (16 bytes per sample).
 *
 * Ownership and errors
 *   Device pointers are owned by the caller and must be 16-byte aligned
 *   device memory on the current HIP device.  `stream` is a hipStream_t
 *   (0 = the legacy default stream).  A plan is immutable after creation,
 *   holds no device memory and may be used from several threads and streams
 *   at once.  Every entry point returns NSLCT_OK (0) or a negative code;
 *   on error no device work has been queued and nslct_last_error() returns
 *   a message (per thread).  Launches are asynchronous: a fault inside a
 *   kernel shows up at the next synchronising HIP call.
 *
 * Sizes
 *   Nx, Ny are any length from 2 to 2048, or 2^k up to 4096 (NSLCT_E_SIZE
 *   otherwise).  2^k and 3 * 2^k (up to 768) run native mixed-radix line
 *   FFTs; every other length runs Bluestein's chirp-z form of its line DFT
 *   on a power-of-two line of at least 2N - 1 samples (about four times the
 *   arithmetic; its tables are computed on the host and uploaded on the
 *   first transform of that length on a device, so that first call must not
 *   be inside a stream capture).  The ragged batch and the backward sweep
 *   take them too (not the allocation-free backward entry point); the
 *   split-precision paths take sides 256 and 4096 only.
 */
#ifndef NSLCT_H
#define NSLCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define NSLCT_OK 0
#define NSLCT_E_ARG (-1)              /* null / misaligned pointer, bad scalar */
#define NSLCT_E_NOT_SYMPLECTIC (-2)   /* max|M J M^T - J| above the tolerance */
#define NSLCT_E_NO_DECOMPOSITION (-3) /* no symmetric gauge with invertible B' */
#define NSLCT_E_SIZE (-4)             /* unsupported Nx, Ny */
#define NSLCT_E_HIP (-5)              /* HIP runtime error (message kept) */
#define NSLCT_E_UNSUPPORTED (-6)      /* valid request the library does not implement */

/* Precision of storage and arithmetic. */
#define NSLCT_C64 0  /* complex64 storage, FP32 butterflies, FP64-exact phases */
#define NSLCT_C128 1 /* complex128 storage and arithmetic */
/* complex64 storage, line DFTs on the matrix cores with operands split into
 * high + low FP16 (or BF16) parts and FP32 accumulation; chirps as NSLCT_C64.
 * Sides 256 or 4096 (radix-16 stages only). */
#define NSLCT_C64_SPLIT_F16 2
#define NSLCT_C64_SPLIT_BF16 3

typedef struct nslct_plan_s* nslct_plan_t;
typedef struct nslct_batch_s* nslct_batch_t;

/* Planning options; initialise with nslct_opts_default. */
typedef struct {
    int precision;         /* NSLCT_C64 (default), NSLCT_C128, NSLCT_C64_SPLIT_F16/BF16 */
    int type_override;     /* 0: trace rule (eq. Reversible08), 1: CM-CC-CM-CC, 2: CC-CM-CC-CM,
                              3: CM-CC-CM (Sec. 4.1, B symmetric and invertible),
                              4: LC-NsDLCT with H = (h,0;0,0) (Sec. 4.2.2, eq. LC08),
                              5: LC-NsDLCT with H = (0,0;0,h) (eq. LC10),
                              6: LC-NsDLCT, the form with the smaller eq. HA24 objective; when neither
                                 rank-one gauge exists, the route of 7 if it applies, else the HA-NsDLCT,
                              7: for a12 = a21 = 0 (Sec. 4.2.2): (A, B; C, D) = (-B, A; -D, C)(0, -I; I, 0),
                                 the IDFT then CM-CC-CM of (-B, A; -D, C) (eq. Bsym12); needs A
                                 invertible and dx = sqrt(2 pi / Nx), dy = sqrt(2 pi / Ny) (the IDFT
                                 keeps the grid only there), native lengths, complex64 / complex128 */
    double symplectic_tol; /* accepted max|M J M^T - J|, default 1e-9 */
    double det_min;        /* a middle CC matrix B' is accepted when |det B'| >= det_min * max(1, max|B_ij|^2)
                              (the invertibility conditions of eqs. Bsym08 and Bnonsym32), default 1e-6 */
} nslct_opts;

/* Stage description of a plan (and input of nslct_plan_from_stages).
 *   type 1: mats = {P1, B', P3, H}    -> CM(P1) CC(B') CM(P3) CC(H)
 *   type 2: mats = {H1, Q1, B1', Q3}  -> CC(H1) CM(Q1) CC(B1') CM(Q3)
 *   type 0: mats[0] = C (pure chirp multiplication, B = 0, A = D = I)
 *   type 3: mats = {P1, B, P3, 0}     -> CM(P1) CC(B) CM(P3)        (eq. Bsym12)
 *   type 4: mats = {P1, B', P3, H}, H = (h, 0; 0, 0), LC along x   (eq. LC12)
 *   type 5: mats = {P1, B', P3, H}, H = (0, 0; 0, h), LC along y
 *   type 7: mats = {P1', A, P3', 0} of M' = (-B, A; -D, C):
 *           G = j^phase_q CM(P1') CC(A) CM(P3') U^H g, with U^H the unitary
 *           centred 2D IDFT and the CC unitary; phase_q makes the route the
 *           operator of the CM-CC-CM-CC / CC-CM-CC-CM chain of M (the paper
 *           leaves the constant of a product open; it is derived by
 *           propagating a Gaussian through both factorisations in closed form).
 *           Four passes (64 B per sample for complex64).
 * Each symmetric 2x2 matrix is stored as (x11, x12, x22).  Types 3-5 have one
 * 2D CC; their overall constant is +1 like the two-CC chains' (the paper's
 * DFT constants taken literally would give -1 there), and their 1D CC uses
 * the unitary 1D DFT pair (a 1D CC with h = 0 is the identity).  They run as
 * three passes (48 B per sample for complex64) on the single-image path at
 * native lengths, and as their five-slot form (the same chain, a CC with a
 * zero or rank-one matrix in place of the missing one) at other lengths. */
typedef struct {
    int type;
    double mats[4][3];
    double h[3];               /* gauge (h11, h12, h22), zero for type 0 */
    double gauge_objective;    /* value of the eq. HA24 product at h */
    double symplectic_residual;/* max|M J M^T - J| of the planned matrix */
    double dx, dy;             /* space sampling intervals */
    double dwx, dwy;           /* frequency intervals 2 pi / (N dx), 2 pi / (N dy) */
    int phase_q;               /* type 7: overall constant j^phase_q (0..3); 0 otherwise */
} nslct_stages;

/* Fills *opts with the defaults. */
void nslct_opts_default(nslct_opts* opts);

/* Plans the transform of an Nx x Ny image for ABCD matrix `abcd` (16 doubles,
 * row-major 4x4) with sampling intervals dx, dy > 0 (host only, FP64).
 * Validates M (eq. Intro12), picks the type (eq. Reversible08) and solves the
 * gauge problem of eq. HA24.  B = 0 with A = D = I gives a pure CM; B = 0
 * otherwise is an affine map (eq. Intro20): NSLCT_E_NO_DECOMPOSITION. */
int nslct_plan(const double abcd[16], int Nx, int Ny, double dx, double dy, nslct_plan_t* out);
int nslct_plan_ex(const double abcd[16], int Nx, int Ny, double dx, double dy,
                  const nslct_opts* opts, nslct_plan_t* out);

/* Plans M = M0 expm(J S(theta)) for differentiation (Sec. 6.2 with the
 * parameterisation of the configs: theta holds the 10 coordinates of the Lie
 * algebra of the ABCD group, the upper triangle, row by row, of the symmetric
 * 4x4 S; J S is a general element of that algebra, so M satisfies eq. Intro12
 * whenever M0 does).  The plan records (M0, theta) for nslct_backward_theta.
 * With type_override 0 the type follows the trace rule (eq. Reversible08)
 * even when B is symmetric: the CM-CC-CM form does not exist at perturbed
 * matrices, so a differentiable plan keeps the CM-CC-CM-CC / CC-CM-CC-CM
 * form.  Other options as nslct_plan_ex; host only. */
int nslct_plan_lie(const double abcd0[16], const double theta[10], int Nx, int Ny, double dx, double dy,
                   const nslct_opts* opts, nslct_plan_t* out);

/* Plans from explicit stage matrices (type and mats read from *st; dx, dy
 * read from *st; other fields ignored).  Used to run the chain at fixed
 * stages (Secs. 4.2-4.3). */
int nslct_plan_from_stages(const nslct_stages* st, int Nx, int Ny, const nslct_opts* opts,
                           nslct_plan_t* out);

/* Copies the plan's stage description into *out. */
int nslct_plan_get_stages(nslct_plan_t plan, nslct_stages* out);

/* Phase-space growth check of the plan (Sec. 4.2.1, eqs. HA12-HA20): the box
 * |x|,|y| <= frac*N*d/2, |w| <= frac*pi/d pushed through the four stages in
 * application order stays inside the grid.  Host only.  *ok = 1 or 0. */
int nslct_plan_box_check(nslct_plan_t plan, double frac, int* ok);

void nslct_plan_destroy(nslct_plan_t plan);

/* Forward transform of one image; in == out (in place) is allowed. */
int nslct_forward(nslct_plan_t plan, const void* in, void* out, void* stream);

/* Inverse (= adjoint) transform, eq. CCCMCCCM30; in == out allowed. */
int nslct_inverse(nslct_plan_t plan, const void* in, void* out, void* stream);

/* `count` images of the plan's shape stored back to back (image stride
 * Nx*Ny samples), all with the plan's matrix.  in == out allowed.  For
 * complex64 passes over lines of length 64, 192, 256, 384, 512, 768 or 1024
 * the split of a line over threads is chosen by the number of lines in
 * flight (lines of the pass times count), so one image's result may differ
 * in its last bits with `count` (every result within the complex64 bar);
 * complex128 passes over lines of length 64, 192, 256, 384 or 768 always
 * take the alternative split.
 * Square 32 x 32 images, and 64 x 64 images from 32 (complex64) or 128
 * (complex128) per call, run the whole chain in one launch with each image
 * held in LDS (one workgroup per image, the passes' own line split). */
int nslct_forward_many(nslct_plan_t plan, int count, const void* in, void* out, void* stream);
int nslct_inverse_many(nslct_plan_t plan, int count, const void* in, void* out, void* stream);

/* One of the five fused passes of the forward (direction 0) or inverse
 * (direction 1) chain, pass = 0 .. nslct_plan_passes - 1, on `count` images:
 * pass 0 reads `in`, every pass writes `out`; chaining all passes with
 * in = out after the first equals nslct_forward_many / nslct_inverse_many.
 * A column pass over 4096-long columns (complex64 / complex128) is three
 * kernel launches over 64 x 64 blocks of each column.  For profiling. */
int nslct_launch_pass(nslct_plan_t plan, int direction, int pass, int count,
                      const void* in, void* out, void* stream);

/* Makes, on the current device, every device table the plan's transforms
 * use (the library's twiddle tables, and the Bluestein tables of a side
 * without a native line plan), which the first transform would otherwise
 * make.  After it, transforms of the plan on this device allocate nothing
 * and may be captured into a HIP graph.  Synchronous; idempotent. */
int nslct_plan_prepare(nslct_plan_t plan);

/* Number of passes of the single-image path of `plan`: 3 for the reduced
 * chains (types 3-5) in complex64 / complex128 at native lengths (2^k,
 * 3 * 2^k), else 5.  Host only. */
int nslct_plan_passes(nslct_plan_t plan, int* npasses);

/* Ragged batch: `count` plans (each with its own matrix and size) over one
 * packed buffer in which image i occupies samples [off_i, off_i + Nx_i Ny_i),
 * off_0 = 0, images back to back in plan order.  All plans must share one
 * precision (complex64 or complex128); sides must be 64, 128, 192, 256, 384,
 * 512, 768, 1024, or any length up to 2048 without a native plan (Bluestein
 * line DFTs, as in the single-image path; their tables are made here).  The
 * batch copies the plans (they may be destroyed afterwards), uploads a
 * table of pass arguments per (image, direction, pass) and an XCD-balanced
 * work list to the current device.  Its passes run one launch per group
 * (pass axis, line length); each group's schedule, the line plan (0: the
 * single-image split of a line over threads and radices; 1: an
 * alternative split, e.g. 1024 = 16 x 4 x 16 on 32 instead of 64 threads),
 * the tile width (lines per work item: 256, 512 or 1024 threads' worth, as
 * LDS allows) and the grid (1, 2, 4 or 8 persistent workgroups per CU, or
 * one workgroup per item), is taken from the schedule cache or chosen by
 * timing every candidate on scratch images (device work and allocation
 * happen here, once).  The schedule cache is a text file keyed by (GPU architecture,
 * precision, axis, line length, lines of the group rounded up to a power of
 * two): NSLCT_TUNE_CACHE names it (off: no cache), default
 * $HOME/.cache/nslct/batch_schedule.txt; unwritable paths only disable it.
 * Not reentrant: calls on one batch from several threads are serialised
 * internally. */
int nslct_batch_create(const nslct_plan_t* plans, int count, nslct_batch_t* out);

/* Packed buffer length in samples, the grid set by nslct_batch_set_grid
 * (workgroups per CU; 0 = one workgroup per work item; -1 = per-group
 * schedules as tuned) and the forward time of the whole batch measured
 * after tuning, in microseconds (0 when every schedule came from the cache;
 * any pointer may be NULL). */
int nslct_batch_info(nslct_batch_t batch, size_t* total_samples, int* mult, double* tuned_us);

/* Schedule of the group of pass axis `col` (0: row passes, lines of length
 * Ny; 1: column passes, lines of length Nx) and line length N: line plan,
 * lines per work item, grid (workgroups per CU, 0 = one per item) and
 * whether it came from the schedule cache (any output pointer may be NULL).
 * NSLCT_E_ARG when the batch has no such group. */
int nslct_batch_group(nslct_batch_t batch, int col, int N, int* plan, int* lines, int* mult, int* cached);

/* Sets one group's line plan (0 or 1), tile width (`lines`, a candidate of
 * that plan) and grid (mult as nslct_batch_set_grid); synchronises the
 * batch's device and drops the captured graphs.  Results agree across
 * schedules to rounding (bitwise across tile widths and grids of one line
 * plan; the two line plans order their additions differently). */
int nslct_batch_set_group(nslct_batch_t batch, int col, int N, int plan, int lines, int mult);

/* Puts every group on `mult` persistent workgroups per CU (1, 2, 4 or 8) or
 * on one workgroup per work item (0), keeping the tile widths; any other
 * value is NSLCT_E_ARG.  Synchronises the batch's device, then drops the
 * captured graphs (the next graph run captures again).  Results do not
 * depend on the grid (each work item is computed by the same code whatever
 * the grid). */
int nslct_batch_set_grid(nslct_batch_t batch, int mult);

/* Forward / inverse of every image of the batch: the five passes, each one
 * persistent launch per line length over all images of that length (the
 * launches of one pass run concurrently), captured once per (in, out) pair
 * into a HIP graph that is then replayed on `stream`.  When the row and
 * column line lengths pair up (the images whose rows have length a all have
 * columns of length b, and no other image has either; square images
 * always), each pair's five launches form an independent sequence on its
 * own fork stream, joined once at the end, instead of joining every pass.
 * in == out allowed. */
int nslct_forward_batched(nslct_batch_t batch, const void* in, void* out, void* stream);
int nslct_inverse_batched(nslct_batch_t batch, const void* in, void* out, void* stream);

/* Same work with an explicit execution mode: 0 graph replay (as above),
 * 1 the five batched launches without a graph, 2 one chain of launches per
 * image (the reference loop).  direction 0 forward, 1 inverse. */
int nslct_batch_run(nslct_batch_t batch, int direction, int mode, const void* in, void* out, void* stream);

void nslct_batch_destroy(nslct_batch_t batch);

/* Backward sweep for a loss of G = forward(x) (Sec. 6.2: the operator is
 * unitary, so its adjoint is the inverse chain, eq. CCCMCCCM30).  G is the
 * forward output and grad_out = dLoss/dRe(G) + j dLoss/dIm(G), both `count`
 * images.  Runs the inverse chain on G (into `work`) and on grad_out (into
 * grad_x) together and at each of the five chirp points adds to the device
 * array sums[15] (caller-zeroed, accumulated over images; must not be read
 * before the stream reaches this call) the sums of Im(conj(adjoint) signal)
 * weighted by x^2, x y, y^2.  On return grad_x = L^H grad_out = dLoss/dx.
 * Sides 8..1024 (2^k), 48, 96, 192, 384, 768, or any length up to 2048
 * without a native plan (Bluestein lines; their tables are made on the first
 * call with that length on a device); work, grad_x distinct buffers. */
int nslct_backward(nslct_plan_t plan, int count, const void* G, const void* grad_out, void* work, void* grad_x,
                   double* sums, void* stream);

/* Gradients of a real loss of G = forward(x) with respect to x and to the
 * plan's 10 Lie coordinates theta (plans from nslct_plan_lie, or nslct_plan /
 * nslct_plan_ex, whose theta is 0 around M itself):
 *   grad_x     = L^H grad_out = dLoss/dx (device, `count` images; L is
 *                unitary, Sec. 6.2, and L^H is the inverse chain, eq.
 *                CCCMCCCM30),
 *   grad_theta = dLoss/dtheta (host, 10 doubles; may be NULL),
 * where G is the forward output and grad_out = dLoss/dRe(G) + j dLoss/dIm(G)
 * (device, `count` images each).  The sweep of nslct_backward runs on a work
 * image and 15 sums that the library allocates on `stream`
 * (hipMallocAsync) and frees after use; grad_theta chains the stage gradient
 * (nslct_plan_stage_gradient) with d(stage entries)/d(theta)
 * (nslct_plan_theta_jacobian) and the sum over images.  With grad_theta the
 * call returns after `stream` has finished the sweep; without it the call is
 * asynchronous.  grad_x must differ from G; sizes as nslct_backward.  Plans
 * made from stage matrices have no theta: NSLCT_E_UNSUPPORTED when
 * grad_theta is requested. */
int nslct_backward_theta(nslct_plan_t plan, int count, const void* G, const void* grad_out, void* grad_x,
                         double grad_theta[10], void* stream);

/* nslct_backward_theta for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same results without any allocation.  The work image and
 * the 15 sums live in a static device array of the library, 16 MiB + 256
 * bytes per device (held from the library's first use of that device until
 * the process ends); images are swept in chunks of up to 16 MiB, so any
 * count is accepted, and a single image above 16 MiB is NSLCT_E_SIZE
 * (unreachable with its sizes, whose largest image is 1024 x 1024
 * complex128 = 16 MiB).  Native sides only: a side without a native line
 * plan is NSLCT_E_SIZE (its Bluestein table would be allocated).  The sums
 * are cleared by a kernel at the start of
 * every call.  Every call on one device shares that device's array: calls
 * that overlap in time on one device (several host threads, or streams
 * that run concurrently) race and give wrong results. */
int nslct_backward_theta_noalloc(nslct_plan_t plan, int count, const void* G, const void* grad_out,
                                 void* grad_x, double grad_theta[10], void* stream);

/* Host: d(stage entries)/d(theta) of the plan at its own (M0, theta),
 * jac[12][10] row-major (entries in the order of nslct_stages.mats), the
 * planner differentiated as nslct_plan_jacobian does with its step chosen by
 * the decomposition type (1e-4 for a searched gauge, 1e-5 for closed-form
 * stages).  Computed once per plan and kept. */
int nslct_plan_theta_jacobian(nslct_plan_t plan, double jac[12 * 10]);

/* Host: the 15 sums of nslct_backward -> dLoss / d(stage-matrix entries),
 * 12 doubles in the order of nslct_stages.mats (x11, x12, x22 each).  The
 * derivative of CM(P) g = exp(j phi) g with respect to an entry of P is
 * j (d phi / d entry) CM(P) g (eq. BasicCM12); CC chirps enter with -B. */
int nslct_plan_stage_gradient(nslct_plan_t plan, const double sums[15], double grad_stages[12]);

/* Host: out = M expm(J S(theta)), S symmetric 4x4 whose upper triangle,
 * row by row, is theta (s11, s12, s13, s14, s22, s23, s24, s33, s34, s44);
 * J S is a general element of the Lie algebra of the ABCD group, so every
 * output satisfies eq. Intro12 when M does. */
int nslct_lie_point(const double abcd[16], const double theta[10], double out[16]);

/* Host: d(stage entries)/d(theta) at theta0, jac[12][10] row-major, for
 * M(theta) = M expm(J S(theta)): central differences of the planner with
 * step h in (0, 1e-2], decomposition type held; at theta0 +- h the eq. HA24
 * minimiser is followed from the one at theta0 (local Nelder-Mead and kink
 * snapping instead of the full grid search).  Valid where the minimiser
 * moves smoothly (its set of vanishing stage entries does not change within
 * +-h). */
int nslct_plan_jacobian(const double abcd[16], const double theta0[10], int Nx, int Ny, double dx, double dy,
                        const nslct_opts* opts, double h, double jac[12 * 10]);

/* Plain device-to-device copy kernel of `bytes` bytes (multiple of 16): the
 * bandwidth reference the transform is measured against. */
int nslct_device_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* nslct_last_error(void);
const char* nslct_strerror(int code);

/* Library version string. */
const char* nslct_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NSLCT_H */
