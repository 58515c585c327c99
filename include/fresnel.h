/* fresnel.h - C ABI of libfresnel.so, the gfx950 (MI355X) Fresnel + matrix-Fourier-transform
 * propagation library.
 *
 * The operations are those of Douglas & Perrin, "Accelerated Modeling of Near and Far-Field
 * Diffraction for Coronagraphic Optical Systems" (SPIE 2018, arXiv:1806.06467):
 *   - fresnel_step: one plane-to-plane step, i.e. the optic multiply of Eq. (3) (and a thin
 *     lens, Sec. 1.1 after Goodman Eq. 5-10) followed by angular-spectrum propagation
 *     (Sec. 1.1, after Lawrence Eqs. 82-89): 2-D FFT, transfer function, inverse 2-D FFT;
 *   - fresnel_direct: the direct Fresnel step (Sec. 1.1; the quadratic phase of Sec. 2.3):
 *     quadratic phase, one 2-D FFT, quadratic phase, to a grid of pitch lambda z / (n dx);
 *   - mft_forward / mft_adjoint: the matrix Fourier transform between pupil and focal planes
 *     used by the semi-analytic Lyot coronagraph (Sec. 1.1, Soummer et al.; Sec. 2.3, the
 *     sin/cos arrays of the matrix DFT);
 *   - propagate_train: a complete coronagraph train repeated over wavelengths (Sec. 1.2),
 *     with an optional adjoint pass giving deformable-mirror gradients.
 *
 * Conventions (all entry points):
 *   - complex data are interleaved float pairs (fr_c64), row-major [y][x], in DEVICE memory;
 *     real maps (amplitude, OPD, masks) are float, row-major, device memory;
 *   - the optical axis of an n x n plane sits on pixel (n/2, n/2) (integer division);
 *   - forward transforms use exp(-2 pi i ...); the angular-spectrum transfer function is the
 *     paraxial H(fx, fy) = exp(-i pi lambda z (fx^2 + fy^2)) with no e^{ikz} piston;
 *   - lengths are SI metres, angles on focal planes are in lambda/D;
 *   - every call is asynchronous on `stream` (a hipStream_t; NULL = the null stream); device
 *     buffers are owned by the caller and must stay valid until the stream reaches the call;
 *   - return value: FR_OK (0), a negative FR_E* error (nothing was launched and no output
 *     was touched), or a positive FR_W_* bitmask (results were written; a sampling warning).
 *   - an fr_ctx caches per-geometry tables (FFT roots, transfer functions, lens chirps, MFT
 *     matrices, DM influence matrices). The first call with new parameters builds them
 *     (allocating device memory and waiting on `stream` for the upload); later calls with the
 *     same parameters allocate nothing (the cache bound: fr_set_cache_limit). One fr_ctx may be
 *     used by one host thread at a time.
 */
#ifndef FRESNEL_H
#define FRESNEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status ------------------------------------------------------------------------ */
#define FR_OK 0
#define FR_EINVAL (-1)        /* bad argument: null pointer, non-positive size, bad flag   */
#define FR_EUNSUPPORTED (-2)  /* size or combination the kernels do not implement          */
#define FR_EWORKSPACE (-3)    /* workspace missing or smaller than the *_workspace_bytes   */
#define FR_EHIP (-4)          /* a HIP runtime call or a kernel launch failed              */
#define FR_ENOMEM (-5)        /* device allocation for a cached table failed               */
#define FR_ESTATE (-6)        /* a table was missing while a graph was being recorded      */

#define FR_W_AS_UNDERSAMPLED 1 /* |z| > n dx^2 / lambda: the transfer function aliases     */
#define FR_W_MFT_ALIASED 2     /* du > n_d / n_in: focal sampling beyond the input lattice */
#define FR_W_DIRECT_UNDERSAMPLED 4 /* z < n dx^2 / lambda: the direct step's input chirp aliases */

/* flags of fresnel_step and fresnel_direct */
#define FR_ADJOINT 1 /* apply the adjoint: the step's adjoint first, then the conjugate optic */
#define FR_INVERSE 2 /* fresnel_direct only: the inverse of the optic-free step             */

typedef struct fr_ctx fr_ctx;
typedef struct {
  float re, im;
} fr_c64;
typedef struct {
  double re, im;
} fr_c128;

/* Create a context bound to HIP device `device`. *ctx receives the handle. autotune_path, when
 * not NULL, names a tuning file (fr_autotune_save's format) whose choices the context takes at
 * once, as fr_autotune_load would; a file it cannot read or parse fails the call (FR_EINVAL,
 * *ctx left NULL). */
int fr_create(fr_ctx **ctx, int device, const char *autotune_path);
/* Free every cached table and the context (synchronises the device). NULL is accepted. */
int fr_destroy(fr_ctx *ctx);
/* Bound of the context's table cache (default 4096 tables; max_tables >= 1, else FR_EINVAL).
 * The bound is applied when an entry point starts: a call that finds max_tables or more tables
 * cached first waits for the device (hipDeviceSynchronize) and frees every table and recorded
 * graph, then builds what it needs; tables are never freed in the middle of a call. So a long
 * scan over distances or wavelengths holds at most max_tables plus one call's tables. */
int fr_set_cache_limit(fr_ctx *ctx, int32_t max_tables);
/* Static text for a status code (never NULL). For FR_EHIP the last HIP error is appended. */
const char *fr_status_string(int status);
/* 1 if n is a plane edge fresnel_step implements, else 0. */
int fr_fft_size_supported(int32_t n);

/* ---- one Fresnel plane (Sec. 1.1; Eq. 3) ----------------------------------------------
 * field  : n x n c64, in place. On return field <- AS_z( field * optic ), where
 *          optic = amp * exp(2 pi i opd / lambda) * exp(-i pi r^2 / (lambda f)),
 *          r^2 = ((x - n/2)^2 + (y - n/2)^2) dx^2 and the two-dimensional AS step is
 *          U <- IDFT2( H . DFT2(U) ), H[ky][kx] = exp(-i pi lambda z (kx^2 + ky^2)/(n dx)^2),
 *          kx, ky the signed frequency indices.
 *          With FR_ADJOINT: field <- conj(optic) * AS_{-z}(field), the exact adjoint.
 * amp    : n x n float or NULL (= 1).   opd_m : n x n float OPD in metres or NULL (= 0).
 * lens_focal_m : thin-lens focal length, 0 = no lens.
 * Implemented edges: fr_fft_size_supported(n). Errors: FR_EINVAL (null field, n <= 0,
 * dx/lambda <= 0, unknown flag), FR_EUNSUPPORTED (edge). Warning: FR_W_AS_UNDERSAMPLED.
 * Uses no workspace: each sweep owns whole rows/columns, so the update is in place. */
int fresnel_step(fr_ctx *ctx, fr_c64 *field, int32_t n, double dx_m, double wavelength_m,
                 double z_m, const float *amp, const float *opd_m, double lens_focal_m,
                 int32_t flags, void *stream);

/* ---- one Fresnel plane in float64 (Sec. 2.2: the paper's benchmarks are double precision) ----
 * fresnel_step with complex float64 fields (fr_c128, interleaved, row-major, n x n, in place)
 * and float64 maps (amp, opd_m: n x n or NULL): the same optic, transfer function, lens, flags,
 * conventions, errors and warning. Tables (transfer function, lens chirp, twiddles) are built
 * and kept in float64. Implemented edges: powers of two from 64 to 8192. Uses no workspace. */
int fresnel_step_f64(fr_ctx *ctx, fr_c128 *field, int32_t n, double dx_m, double wavelength_m,
                     double z_m, const double *amp, const double *opd_m, double lens_focal_m,
                     int32_t flags, void *stream);

/* ---- angular-spectrum step with the exact transfer function (Sec. 1.1: the angular-spectrum
 * method after Lawrence, without the paraxial approximation) ----------------------------------
 * As fresnel_step (same optic, same conventions, same flags), with
 *   H[ky][kx] = exp(2 pi i z (sqrt(1/lambda^2 - f^2) - 1/lambda)),  f^2 = (kx^2 + ky^2)/(n dx)^2,
 * the piston exp(2 pi i z / lambda) left out as in the paraxial form (which is this phase to
 * second order in lambda f); evanescent components (f > 1/lambda) decay as
 * exp(-2 pi |z| sqrt(f^2 - 1/lambda^2)) in either direction. H is not separable, so a plane takes
 * three sweeps (row FFT, column FFT * H * inverse FFT, inverse row FFT). H's phase is formed per
 * element in float64 and reduced before the float32 sine and cosine; on a grid with no evanescent
 * frequency whose phase differs from the paraxial one by at most a quarter turn, H is formed
 * instead as its paraxial factors along x and y (built in float64) times exp(2 pi i c) with that
 * difference c in float32, to the same accuracy. Implemented edges:
 * powers of two from 64 to 8192. Errors: FR_EINVAL (null field, n <= 0, dx / lambda <= 0, a
 * non-finite value, unknown flag), FR_EUNSUPPORTED (edge). Warning: FR_W_AS_UNDERSAMPLED. Uses no
 * workspace. */
int fresnel_step_exact(fr_ctx *ctx, fr_c64 *field, int32_t n, double dx_m, double wavelength_m,
                       double z_m, const float *amp, const float *opd_m, double lens_focal_m,
                       int32_t flags, void *stream);

/* ---- direct (single-transform) Fresnel step (Sec. 1.1: the direct Fresnel method beside the
 * angular spectrum; Sec. 2.3, Eq. 2: the quadratic phase factor, read as
 * exp(+i pi (x^2 + y^2) / (lambda z))) -----------------------------------------------------
 * field : n x n c64, in place. With U = field * optic (optic exactly as for fresnel_step,
 *         lens included), on return
 *           field[ky][kx] <- dx^2 / (i lambda z) q2(kx) q2(ky) sum_{y, x} U[y][x] q1(x) q1(y)
 *                            exp(-2 pi i ((x - n/2)(kx - n/2) + (y - n/2)(ky - n/2)) / n),
 *         q1(i) = exp(i pi ((i - n/2) dx)^2 / (lambda z)) on the input grid and
 *         q2(k) = exp(i pi ((k - n/2) dx2)^2 / (lambda z)) on the output grid of pitch
 *         dx2 = lambda |z| / (n dx): the Fresnel integral over z evaluated with one 2-D FFT (no
 *         e^{ikz} piston, as for fresnel_step). The output plane is centred on pixel n/2 too.
 *         Over z < 0 (towards the source) the same formula holds with the signed z (the
 *         transform's kernel sign flips): the step over -z is the conjugate of the step over z
 *         applied to the conjugate field.
 * flags : 0, or FR_ADJOINT: the exact adjoint of the call with the same arguments, from the
 *         output grid back to the input grid: field <- conj(optic) D^H(field), with D^H the
 *         conjugate transpose of the step above (conjugate phases and constant, exp(+2 pi i ...)).
 *         Scaled by (dx2 / dx)^2 it undoes the forward step (the step is unitary up to the
 *         pitch change), i.e. it propagates a far-field plane back over -z.
 *         FR_INVERSE: that scaled adjoint, the inverse of the step (no optic: amp, opd_m NULL and
 *         lens_focal_m 0, else FR_EINVAL).
 * z_m   : nonzero.   dx_out_m : receives dx2 (written only on success), for either direction.
 * Implemented edges: powers of two from 64 to 8192. Errors: FR_EINVAL (null field or dx_out_m,
 * n <= 0, dx / lambda <= 0, z = 0, a non-finite value, unknown flag), FR_EUNSUPPORTED (edge).
 * Warning: FR_W_DIRECT_UNDERSAMPLED (|z| < n dx^2 / lambda, where the angular-spectrum step is
 * the sampled one). Uses no workspace (in place, two sweeps). */
int fresnel_direct(fr_ctx *ctx, fr_c64 *field, int32_t n, double dx_m, double wavelength_m, double z_m,
                   const float *amp, const float *opd_m, double lens_focal_m, int32_t flags,
                   double *dx_out_m, void *stream);

/* ---- Gaussian pilot-beam planner (Sec. 1.1: both the direct and the angular-spectrum method
 * propagate a wavefront; which one a step takes follows a Gaussian pilot beam, after Lawrence) --
 * The beam has its waist (radius w0_m) at z_waist_m; its Rayleigh distance is
 * z_R = pi w0^2 / lambda. A plane within z_R of the waist (|z - z_waist| <= z_R) is near: its
 * field is held on the waist-plane pitch dx_w and moved by the angular-spectrum step. A farther
 * plane is far: its field is held on the pitch lambda |d| / (n dx_w), d = z - z_waist, and is the
 * direct step over d of the waist-plane field. fr_plan_route writes into steps[] (capacity >= 2)
 * the steps that carry the field from z_from_m to z_to_m and returns their count (0, 1 or 2):
 *   near -> near: one FR_ROUTE_AS step over z_to - z_from;
 *   otherwise through the waist plane: leaving a far plane by FR_ROUTE_DIRECT_INVERSE, moving
 *   between near planes and the waist by FR_ROUTE_AS, reaching a far plane by FR_ROUTE_DIRECT
 *   (steps of zero length are left out).
 * Each step gives the call to make: FR_ROUTE_AS: fresnel_step over z_m at pitch dx_in_m;
 * FR_ROUTE_DIRECT: fresnel_direct over z_m from pitch dx_in_m (it returns dx_out_m);
 * FR_ROUTE_DIRECT_INVERSE: fresnel_direct(..., FR_INVERSE) with dx = dx_out_m over z_m. dx_m is
 * the pitch of the field at z_from_m (near or far as
 * that plane is). Host-only arithmetic (no device call). Errors: FR_EINVAL (w0, lambda, dx <= 0,
 * n <= 0, a non-finite value, steps NULL or capacity < 2). */
#define FR_ROUTE_AS 1
#define FR_ROUTE_DIRECT 2
#define FR_ROUTE_DIRECT_INVERSE 3
typedef struct {
  int32_t kind;     /* FR_ROUTE_* */
  double z_m;       /* signed distance of the call */
  double dx_in_m;   /* pitch of the field before the step */
  double dx_out_m;  /* pitch after it */
} fr_route_step;
int fr_plan_route(double w0_m, double z_waist_m, double wavelength_m, int32_t n, double dx_m,
                  double z_from_m, double z_to_m, fr_route_step *steps, int32_t capacity);

/* ---- a multi-optic system (App. B: the paper's benchmark relay of optics -- aperture, primary,
 * relay mirrors as thin lenses, a shaped pupil, a focal-plane mask, a final focus -- with Fresnel
 * propagation between them, about 19 FFTs per wavelength; Sec. 1.2) ----------------------------
 * optics[0] sits on the input plane; optics[i] (i > 0) sits z_m >= 0 after optics[i - 1]. At each
 * plane the field is multiplied by its optic: amp (transmission) and opd_m (OPD, phasor
 * exp(2 pi i opd / lambda), Eq. 3), n x n float maps sampled on the pitch fr_plan_system gives
 * that plane (NULL = none), and a thin lens exp(-i pi r^2 / (lambda f)) (lens_focal_m, 0 =
 * none). Between planes the field travels by the steps of fr_plan_route under a Gaussian pilot
 * beam that starts collimated with waist radius beam_radius_m on the input plane and changes at
 * every lens by the q-law 1/q' = 1/q - 1/f (q = z - z_waist - i z_R): the angular spectrum
 * between near planes, the direct step (or its inverse) to (or from) far planes, so the pitch
 * changes where the field crosses a focus. fr_plan_system (host arithmetic, no device call)
 * writes each plane's pitch into plane_dx_m[count] (where masks must be sampled; the first is
 * dx_m) and the number of 2-D transforms the system takes into *transforms (two per
 * angular-spectrum step, one per direct step); either output may be NULL. propagate_system runs
 * it on field (n x n c64, in place, pitch dx_m on the input plane) and leaves the field at the
 * last plane, after its optic, with its pitch in *dx_out_m. Power-of-two edges 64..8192.
 * Errors: FR_EINVAL (a NULL or non-finite argument, count <= 0, a negative distance, a lens
 * that leaves no beam), FR_EUNSUPPORTED (edge); warnings of the steps are ORed. */
typedef struct {
  double z_m;           /* distance from the previous optic's plane (ignored for optics[0]) */
  double lens_focal_m;  /* thin lens at this plane, 0 = none                                  */
  const float *amp;     /* n x n transmission on this plane's pitch, or NULL                   */
  const float *opd_m;   /* n x n OPD [m] on this plane's pitch, or NULL                        */
} fr_optic;
int fr_plan_system(int32_t n, double dx_m, double wavelength_m, double beam_radius_m, const fr_optic *optics,
                   int32_t count, double *plane_dx_m, int32_t *transforms);
int propagate_system(fr_ctx *ctx, fr_c64 *field, int32_t n, double dx_m, double wavelength_m,
                     double beam_radius_m, const fr_optic *optics, int32_t count, double *dx_out_m,
                     void *stream);

/* Many independent planes in one launch per sweep (e.g. the wavelengths of a broadband
 * model, Sec. 1.2). Each entry has the meaning of the fresnel_step arguments. `planes` is a
 * HOST array read during the call. Planes may have different edges (e.g. one grid per
 * wavelength): the planes of each power-of-two edge take the two-sweep kernels together, the
 * planes of other edges the persistent mixed-radix sweeps together; each plane's result is the
 * one fresnel_step gives. The fields must not overlap. Planes go in groups that fit the
 * last-level cache (both sweeps of a group before the next). Returns the OR of the per-plane
 * warnings, or the first error (then nothing was launched). */
typedef struct {
  fr_c64 *field;
  const float *amp;
  const float *opd_m;
  double dx_m, wavelength_m, z_m, lens_focal_m;
  int32_t n, flags;
} fr_plane;
int fresnel_step_batched(fr_ctx *ctx, const fr_plane *planes, int32_t count, void *stream);
/* The same batched step (Sec. 1.2: the planes of the wavelengths of one broadband model), with
 * the whole call's launch sequence held as one instantiated HIP graph: the first call with a given
 * set of entry values (every field of every fr_plane, count and stream) runs as
 * fresnel_step_batched and then records that sequence; a later call with the same values replays
 * the recording (no table lookups, no host work per plane). Field contents, amp and opd_m may
 * change between calls, their addresses may not. The context keeps at most 8 recordings (the
 * oldest is dropped); fr_set_cache_limit's trim drops them all. Same errors and warnings as
 * fresnel_step_batched; FR_EHIP if recording fails. */
int fresnel_step_batched_graph(fr_ctx *ctx, const fr_plane *planes, int32_t count, void *stream);

/* Many planes of the exact-transfer-function step (fresnel_step_exact; e.g. the wavelengths of
 * a broadband model, Sec. 1.2) in one call. Each fr_plane entry has the meaning of the
 * fresnel_step_exact arguments; all planes share one power-of-two edge n (64..8192). Planes go
 * in groups that fit the last-level cache together, each of the three sweeps over a group in one
 * launch. `planes` is a HOST array read during the call. Returns the OR of the per-plane
 * warnings, or an error; argument errors (FR_EINVAL: count <= 0, mixed edges, any plane's
 * fresnel_step_exact error; FR_EUNSUPPORTED: edge) are found before anything is launched. */
int fresnel_step_exact_batched(fr_ctx *ctx, const fr_plane *planes, int32_t count, void *stream);

/* ---- matrix Fourier transform (Sec. 1.1, Soummer et al.; Sec. 2.3) ---------------------
 * Pupil sample m of an n_in-wide window sits at x_m = (m - n_in/2)/n_d  [D];
 * focal sample k of an m_out grid sits at u_k = (k - m_out/2) du      [lambda/D].
 *   mft_forward: out[ky][kx] = (du/n_d) sum_{y,x} W[ky][y] in[y][x] W[kx][x] (* out_mask),
 *                W[k][m] = exp(-2 pi i u_k x_m); phases are formed from the exact integer
 *                (k - m_out/2)(m - n_in/2) times du/n_d in float64 turns.
 *   mft_adjoint: out = alpha (du/n_d) W^H in conj(W) + beta out, then out *= out_mask;
 *                the exact adjoint of mft_forward for alpha = 1, beta = 0; alpha = -1,
 *                beta = 1 is the Babinet subtraction of an occulting spot.
 * ld_in / ld_out: row strides in elements (>= width), so a window of a larger plane can be
 * read or updated in place. out_mask: float, same shape as out, or NULL.
 * ws: device workspace of at least mft_workspace_bytes(n_in, m_out) bytes (forward) or
 * mft_workspace_bytes(n_out, m_in) bytes (adjoint); contents on entry are ignored.
 * Errors: FR_EINVAL, FR_EWORKSPACE. Warning: FR_W_MFT_ALIASED. */
size_t mft_workspace_bytes(int32_t n_pupil, int32_t m_focal);
int mft_forward(fr_ctx *ctx, const fr_c64 *in, int32_t n_in, int32_t ld_in, fr_c64 *out,
                int32_t m_out, int32_t ld_out, double n_d, double du, const float *out_mask,
                void *ws, size_t ws_bytes, void *stream);
int mft_adjoint(fr_ctx *ctx, const fr_c64 *in, int32_t m_in, int32_t ld_in, fr_c64 *out,
                int32_t n_out, int32_t ld_out, double n_d, double du, float alpha, float beta,
                const float *out_mask, void *ws, size_t ws_bytes, void *stream);

/* ---- mft_forward for callers that cannot allocate device memory -----------------------------
 * For code under HIP graph capture, tight serving loops and harnesses that forbid allocation: the
 * same transform, arguments and kernels as mft_forward without the workspace arguments. The
 * working memory (the n_in x m_out product T, then split-K partial sums in what is left) is a
 * library-owned array of 64 MiB per device (2^26 bytes, a static device array held until the
 * process ends; its address is taken once per device by fr_create). The call allocates and frees
 * nothing: it neither trims the table cache nor builds tables, so the MFT matrix of the geometry
 * (m_out, n_in, n_d, du) must already be cached in the context by an earlier mft_forward (or
 * propagate_train) call with that geometry; if it is not, FR_ESTATE and nothing is launched.
 * Sizes whose product T exceeds the array (8 n_in m_out bytes, 256-aligned, above 2^26) give
 * FR_EWORKSPACE. Calls on one device share the array: calls that overlap on one device (several
 * streams or host threads) race and must be ordered by the caller; the array needs no clearing
 * (every byte read is written by the same call first). Results equal mft_forward's up to the
 * split-K factor, which the smaller array may reduce (float32 rounding order). Errors: FR_EINVAL
 * (as mft_forward), FR_EWORKSPACE, FR_ESTATE, FR_EHIP (the array's address could not be taken).
 * Warning: FR_W_MFT_ALIASED. */
int mft_forward_noalloc(fr_ctx *ctx, const fr_c64 *in, int32_t n_in, int32_t ld_in, fr_c64 *out,
                        int32_t m_out, int32_t ld_out, double n_d, double du, const float *out_mask,
                        void *stream);

/* ---- the MFT in float64 (Sec. 1.1, after Soummer et al.; the paper benchmarks float64) -------
 * Forward (flags 0): in is the n_pupil x n_pupil pupil field, out the m_focal x m_focal focal
 *   field, out = (du/n_d) W in W^T with W as for mft_forward (phases from the exact integer
 *   index product times du/n_d, reduced in float64 turns).
 * Adjoint (FR_ADJOINT): in is m_focal x m_focal, out n_pupil x n_pupil,
 *   out = (du/n_d) W^H in conj(W), the exact adjoint of the forward.
 * in, out: dense row-major fr_c128 in DEVICE memory, not overlapping. ws: device workspace of
 * ws_bytes >= mft_f64_workspace_bytes(n_pupil, m_focal) bytes (the intermediate product, in
 * split-K partial sums where the first product's K is long), for either direction; contents
 * on entry ignored; the caller owns every buffer. The matrix W is built once per (shape, n_d,
 * du) and cached in the context. Errors: FR_EINVAL (null buffer, a size <= 0, n_d or du not
 * positive and finite, unknown flag), FR_EWORKSPACE (ws_bytes too small). */
size_t mft_f64_workspace_bytes(int32_t n_pupil, int32_t m_focal);
int mft_f64(fr_ctx *ctx, const fr_c128 *in, fr_c128 *out, int32_t n_pupil, int32_t m_focal, double n_d,
            double du, int32_t flags, fr_c128 *ws, size_t ws_bytes, void *stream);

/* ---- Lyot coronagraph train over wavelengths (Sec. 1.1 and 1.2) ------------------------
 * Per wavelength lambda_j on an n_pad[j]-wide grid (dx = d_m / n_d):
 *   E   = embed( pupil_amp * exp(2 pi i pupil_opd / lambda) )  [* DM1 phasor if n_dm == 2]
 *   E   = AS_z(E) * exp(4 pi i s / lambda)      (last DM; s = G A G^T, Gaussian influence
 *         G[i][a] = exp(-(i - n/2 - xi_a)^2 / (2 p^2)), xi_a = (a - (n_act-1)/2) p, p = n_d/n_act)
 *   Eo  = MFT(E: whole padded plane -> occ_m^2, du = occ_du_c lambda_c / lambda)
 *   EL  = lyot * ( window_{n_d}(E) - MFT^H(occ_mask * Eo -> n_d^2) )
 *   Ed  = MFT(EL -> det_m^2, du = det_du_c lambda_c / lambda)
 *   psf = sum_j weight_j |Ed_j|^2    (det_m^2 float, overwritten; summed in float64, rounded once)
 * FR_TRAIN_NO_OCCULTER skips the occulter term (the reference PSF).
 * FR_TRAIN_GRAD additionally takes grad_psf = dL/dpsf (det_m^2 float) and writes
 * grad_heights = dL/dA (n_dm * n_act^2 float, DM1 first), the chain rule through every
 * adjoint above. Arrays lambda_m, n_pad, weight are HOST arrays of n_lambda entries.
 * FR_TRAIN_BATCHED keeps one field plane per wavelength in the workspace and runs the Fresnel
 * steps of a group of wavelengths (grids of different edges allowed) in one launch per sweep;
 * groups are as many wavelengths as fit the last-level cache together (one 4096^2 plane,
 * several smaller ones), each followed by its focal-plane chains; all sums still go in
 * wavelength order. Each plane takes the same kernels as in the plain (wavelength after
 * wavelength) mode (power-of-two edges the two-sweep kernels, other edges the mixed-radix
 * sweeps), so psf and grad_heights are bit-identical to that mode. Its workspace grows with
 * sum_j n_pad[j]^2.
 * FR_TRAIN_GRAPH records the whole call as one graph the first time a given set of argument
 * values (descriptor bytes, host arrays, device pointers, stream) is seen, after running it
 * normally, and replays that graph on later identical calls; the device inputs may change
 * between calls, their addresses may not. At most 8 graphs are kept per context.
 * The gradient in two calls (for an autograd forward / backward pair): FR_TRAIN_FWD_SAVE runs
 * the forward (psf written, as without it) and keeps in the caller's checkpoint `ckpt` what the
 * adjoint needs: per wavelength the field at the last DM plane (n_pad[j]^2 c64) and the detector
 * field (det_m^2 c64), ckpt_bytes >= propagate_train_ckpt_bytes(desc, n_lambda, n_pad). A later
 * FR_TRAIN_BWD call with the same descriptor, heights, wavelengths, grids, weights and occulter
 * bit takes grad_psf, reads that checkpoint and writes grad_heights without running the forward
 * again (psf is not touched and may be NULL); its grad_heights are bit-identical to those of one
 * FR_TRAIN_GRAD call. The checkpoint is owned by the caller and only read by FR_TRAIN_BWD; the
 * caller keeps its contents between the two calls. At most one of FR_TRAIN_GRAD,
 * FR_TRAIN_FWD_SAVE, FR_TRAIN_BWD per call (else FR_EINVAL); ckpt / ckpt_bytes are ignored (may
 * be NULL / 0) without the last two, FR_EWORKSPACE when they are too small.
 * ws: device workspace of propagate_train_workspace_bytes(...) bytes (same mode bits). */
#define FR_TRAIN_NO_OCCULTER 1
#define FR_TRAIN_GRAD 2
#define FR_TRAIN_BATCHED 4
#define FR_TRAIN_GRAPH 8
#define FR_TRAIN_FWD_SAVE 16
#define FR_TRAIN_BWD 32
typedef struct {
  int32_t n_d;               /* pupil pixels across D                                   */
  double d_m;                /* pupil diameter [m]                                      */
  const float *pupil_amp;    /* n_d x n_d                                               */
  const float *pupil_opd_m;  /* n_d x n_d or NULL                                       */
  int32_t n_dm;              /* 0, 1 (after the step) or 2 (pupil and after the step)   */
  int32_t n_act;             /* actuators per DM edge                                   */
  const float *dm_heights_m; /* n_dm x n_act x n_act surface heights [m]                */
  double z_m;                /* pupil -> last-DM distance [m]                           */
  int32_t occ_m;             /* occulter grid edge                                      */
  double occ_du_c;           /* occulter pitch [lambda_c/D]                             */
  const float *occ_mask;     /* occ_m x occ_m, 1 where the spot blocks                  */
  const float *lyot;         /* n_d x n_d                                               */
  int32_t det_m;             /* detector grid edge                                      */
  double det_du_c;           /* detector pitch [lambda_c/D]                             */
  double lambda_c_m;         /* reference wavelength of the focal grids [m]             */
} fr_train_desc;
size_t propagate_train_workspace_bytes(const fr_train_desc *desc, int32_t n_lambda,
                                       const int32_t *n_pad, int32_t mode);
size_t propagate_train_ckpt_bytes(const fr_train_desc *desc, int32_t n_lambda, const int32_t *n_pad);
int propagate_train(fr_ctx *ctx, const fr_train_desc *desc, int32_t n_lambda,
                    const double *lambda_m, const int32_t *n_pad, const float *weight,
                    int32_t mode, float *psf, const float *grad_psf, float *grad_heights,
                    void *ckpt, size_t ckpt_bytes, void *ws, size_t ws_bytes, void *stream);

/* ---- autotuner (Sec. 2.1: measurement decides among equivalent implementations) ---------
 * fr_autotune times the candidate kernel configurations of one workload shape on `stream` and
 * keeps the fastest in the context; later calls of every entry point use it:
 *   FR_TUNE_FRESNEL, a = plane edge n (b unused): the tile variants of the power-of-two sweeps
 *     (rows per block, columns per tile) and the pass orders of the mixed-radix plan of n (the
 *     orders of its greedy radices and, for the per-wavelength grids of a broadband model, the
 *     plan of the register-resident sweeps, which is also their default);
 *   FR_TUNE_MFT, a = pupil-side edge n, b = focal edge m: the GEMM tile configuration and split-K
 *     factor of each of the two GEMMs of mft_forward (n -> m) and mft_adjoint (m -> n). Tiles
 *     0-3 form each complex k-step from four real products, tiles 4-5 from three (Gauss; the
 *     three sums are combined in float64 at every 32-deep group), tile 6 from four real products
 *     each summed from six products of exact bfloat16 pieces of the float32 operands on the
 *     bf16 matrix cores.
 * Every candidate computes the same result up to the order of float32 roundings. fr_autotune and
 * fr_autotune_load drop every recorded graph (fresnel_step_batched_graph, FR_TRAIN_GRAPH), after
 * waiting for the device, since a recording holds the kernel choices of its time. The call
 * allocates scratch device memory for its duration, synchronises `stream`, and is not meant for
 * a hot loop or a graph capture. Errors: FR_EINVAL, FR_EUNSUPPORTED, FR_ENOMEM, FR_EHIP.
 * fr_autotune_save / fr_autotune_load write / read the tuned choices as a text file (one
 * "sweep n variant [planes]" (planes: the power-of-two sweeps' planes per launch in batched calls,
 * 1..64, or 0 = as many as fit the last-level cache together), "plan n packed_order" (radices
 * 2-10, 12, 14, 15 or 16, 5 bits each from the first pass up, at most 6, product n),
 * "gemm M N K transA transB tile [split]" or
 * "gemm_default tile split" per line; the default applies to GEMM shapes without their own line,
 * tile -1 restoring the choice by shape); a malformed or inconsistent line makes load return
 * FR_EINVAL (valid lines are still taken). */
#define FR_TUNE_FRESNEL 1
#define FR_TUNE_MFT 2
int fr_autotune(fr_ctx *ctx, int32_t kind, int32_t a, int32_t b, void *stream);
int fr_autotune_save(fr_ctx *ctx, const char *path);
int fr_autotune_load(fr_ctx *ctx, const char *path);

/* ---- kernel timing (profiling aid; Sec. 2.1: profiling decides what to optimise) -------
 * While enabled, every kernel the context launches is bracketed by two HIP events recorded
 * on the launch stream. fr_profile_read waits for the recorded events, returns per-kernel
 * totals (names "kernel/tag", NUL-terminated, name_len bytes each; total milliseconds;
 * launch counts; at most max_entries rows, *n_entries written) and forgets them.
 * Errors: FR_EINVAL (null ctx or outputs), FR_EHIP (an event failed). */
int fr_profile_enable(fr_ctx *ctx, int enable);
int fr_profile_read(fr_ctx *ctx, int32_t max_entries, char *names, int32_t name_len,
                    double *total_ms, int64_t *launches, int32_t *n_entries);

#ifdef __cplusplus
}
#endif
#endif /* FRESNEL_H */
