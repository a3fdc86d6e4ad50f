/*
 * gsm.h - C ABI of libgsm: the Generalized Source Method (GSM) solve for 3D
 * periodic dielectric composites on AMD Instinct MI355X (gfx950).
 *
 * Method: A. A. Shcherbakov, A. V. Tishchenko, "3D periodic dielectric
 * composite homogenization based on the Generalized Source Method",
 * arXiv 1501.01752.  The library solves the truncated Fourier-space system of
 * the paper's Eq.(4),
 *
 *   E_am - sum_b G_ab(k_m) sum_m' (Delta eps / eps_b)_{m-m'} E_bm' = E^inc_am,
 *   G_ab(k) = (k_b^2 delta_ab - k_a k_b) / (|k|^2 - k_b^2),  k_b^2 = k0^2 eps_b,
 *   k_m = k_inc + (m_x K_x, m_y K_y, m_z K_z),  K_a = 2 pi / Lambda_a,
 *   E^inc_am = delta_m0 a_a,
 *
 * with a restarted Krylov method (GMRES, the method the paper settles on in
 * its "Calculation details" section) whose matrix-vector product applies the
 * Toeplitz contrast matrix by FFT (the step the truncation section singles out
 * as the most costly): inverse 3D FFT of the three field components, point-wise product
 * with the band-limited contrast on the real-space grid, forward 3D FFT, then
 * the per-harmonic 3x3 Green tensor.  All of it runs in HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Per-axis arrays are ordered (x, y, z).  Lengths use any one unit:
 *   period, wavelength and 1/|k_inc| must agree.  k0 = 2 pi / wavelength.
 * - Voxel permittivities: real, Vz*Vy*Vx values, x fastest; voxel
 *   (ix, iy, iz) fills [ix, ix+1) x [iy, iy+1) x [iz, iz+1) in units of
 *   Lambda_a / V_a.  The plan takes the exact Fourier image of this
 *   piecewise-constant body (the paper prefers exact Fourier images to mesh
 *   samples, "Calculation details").
 * - Field vectors ("systems"): one per (instance, drive), in instance order
 *   and drive order; each is 3 * N1z * N1y * N1x complex128 values
 *   (interleaved re, im) laid out [component][mz][my][mx] with index
 *   m_a + M_a, N1_a = 2 M_a + 1.  Systems are concatenated without padding.
 * - Device pointers are HIP device memory of the plan's device unless a
 *   GSM_OUT_HOST flag says otherwise.  `stream` is a hipStream_t (NULL: the
 *   default stream).  Calls returning results synchronise that stream
 *   before they return.
 * - The library is linked against the HIP runtime libamdhip64.so.7.  Device
 *   pointers and streams passed in must belong to the runtime instance it is
 *   bound to; in a process that also uses PyTorch, load PyTorch first (its
 *   wheel carries its own copy of that runtime) so that the two share it.
 * - No call throws or aborts; every failure is a negative status and
 *   gsm_last_error() (thread-local) holds a message.  On error the outputs
 *   are left untouched, except GSM_W_* results, which are written.
 * - A plan is used by one host thread / stream at a time; different plans
 *   may be used from different host threads at once.
 */
#ifndef GSM_H
#define GSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSM_VERSION 100

/* status codes */
enum {
  GSM_OK = 0,
  GSM_W_NOT_CONVERGED = 1, /* tolerance not met within the caps; best iterate returned */
  GSM_E_ARG = -1,          /* invalid argument (sizes, pointers, ranges) */
  GSM_E_NONFINITE = -2,    /* NaN or Inf in an input */
  GSM_E_NOMEM = -3,        /* device allocation failed */
  GSM_E_DEVICE = -4,       /* HIP runtime error or no device */
  GSM_E_SINGULAR = -5,     /* |k_m|^2 too close to k_b^2 for some m, or singular E0 */
  GSM_E_WORKSPACE = -6,    /* workspace pointer NULL or smaller than gsm_workspace_size */
  GSM_E_UNSUPPORTED = -7   /* order count beyond the largest supported FFT grid */
};

/* precision of the Krylov iterations (the FP64 residual is always FP64) */
enum { GSM_MIXED = 0, GSM_FP64 = 1 };
/* Krylov method: restarted GMRES (default), or BiCGStab (two operator
 * applications per iteration, six vectors per system; needs restart >= 5,
 * which then only sizes the workspace) */
enum { GSM_GMRES = 0, GSM_BICGSTAB = 1 };
/* gsm_solver_opts.flags */
enum {
  GSM_OUT_HOST = 1,    /* E_out / eps_eff / grad are host pointers */
  GSM_SOLVE_GRAPH = 2, /* issue GMRES steps as captured launch graphs (see below) */
  GSM_SOLVE_REORTH = 4 /* GMRES: a second Gram-Schmidt pass at every Arnoldi step
                          (classical Gram-Schmidt twice) instead of only where the
                          first pass removed nearly all of the new vector; see below */
};
/* Second Gram-Schmidt passes.  A system whose step needs a second pass makes
 * it in the slot of its next step (the other systems of its launch group go
 * on), so it runs one slot behind; the host adds up to four slots past the
 * restart length for the systems it has seen fall behind.  With
 * GSM_SOLVE_REORTH every step takes two slots, so a cycle completes about
 * (restart + 4) / 2 steps: a reference mode (tests, badly conditioned
 * systems), not a fast one.  info.reorth counts the second passes. */
/* Launch graphs.  With GSM_SOLVE_GRAPH (and launch profiling off) the
 * Arnoldi steps of a GMRES cycle are issued as captured HIP graphs of four
 * steps each (one graph launch instead of six kernel launches per step; a
 * cycle issued so ends after the restart length, without slots added for
 * systems running behind).  A plan keeps the instantiated graphs of its recent groups and
 * reuses one when a later call would issue exactly the same launches (same
 * kernel arguments: same plan, workspace address, group composition and
 * options), so repeated solves of one batch pay the capture once.  Results
 * are identical to those of separate launches.  BiCGStab steps are always
 * separate launches.  Off by default: on the MI355X with ROCm 7.2 the graph
 * launches ran 1-9 % slower than separate launches for these kernels. */
/* gsm_apply modes: the E-field operator of Eq.(4) or its adjoint, or the
 * H-field operator of Eq.(5) */
enum { GSM_APPLY_FORWARD = 0, GSM_APPLY_ADJOINT = 1, GSM_APPLY_FORWARD_H = 2 };
/* gsm_solver_opts.formulation.  GSM_FORM_E: the electric-field system,
 * Eq.(4).  GSM_FORM_H: the magnetic-field system of Eq.(5),
 *   H_m = H^inc_m + q_m x w_m / (eps_b - |q_m|^2),
 *   w_m = sum_m' [delta_mm' - eps_b eta_{m-m'}] (q_m' x H_m'),
 * q_m = k_m / k0, eta_n the Fourier image of 1/eps (the paper's (eps_b/eps)
 * Toeplitz matrix, taken from the exact image of 1/eps, not by inverting
 * that of eps: "Calculation details"), H^inc_m = delta_m0 a.  Same passes:
 * the curl q x is applied per harmonic before the contrast product, the
 * plane pass multiplies by 1 - eps_b eta(r), and the last pass applies
 * q x / (eps_b - |q|^2).  The H system is solved (gsm_solve) and searched
 * for poles (gsm_pole_search); the effective tensor, the adjoint and the
 * gradient are defined on the E system only (GSM_E_ARG otherwise). */
enum { GSM_FORM_E = 0, GSM_FORM_H = 1 };

typedef struct gsm_plan_s* gsm_plan_t;

/* Geometry of one unit cell (the periodic permittivity of the section on
 * artificial dielectric structures): periods and a voxel body. */
typedef struct gsm_geometry {
  double period[3];  /* Lambda_x, Lambda_y, Lambda_z > 0 (orthogonal lattice) */
  int32_t nvox[3];   /* Vx, Vy, Vz >= 1 */
  const double* eps; /* host, Vz*Vy*Vx real values > 0, x fastest; copied */
} gsm_geometry;

/* gsm_plan_opts.flags */
enum {
  GSM_PLAN_AUTOTUNE = 1 /* time the codelet families of each FFT stage at the
                           first use of an (M, P, precision) and keep the
                           fastest (else fixed defaults) */
};

typedef struct gsm_plan_opts {
  int32_t m_max[3];       /* largest order count M_a any instance will use (0..127) */
  int32_t device;         /* HIP device ordinal */
  int32_t flags;          /* GSM_PLAN_AUTOTUNE or 0 */
  int32_t reserved;       /* must be 0 */
  const char* tune_cache; /* NULL, or a text file of tuning results: read at
                             plan creation (entries of this device's
                             architecture), extended with each new tuning */
} gsm_plan_opts;

/* One (omega, k) point.  Harmonics m_a run over [-M_a, M_a] (the paper's
 * truncation to N_a = 2 M_a + 1 harmonics per axis). */
typedef struct gsm_instance {
  double wavelength; /* lambda > 0 */
  double k_inc[3];   /* incident Bloch wave-vector k^inc (absolute; |k^inc| = n_i k0) */
  int32_t M[3];      /* order counts, 0 <= M_a <= plan m_max[a] */
  int32_t n_drive;   /* number of drives 1..3 (gsm_eff_tensor ignores it and uses 3) */
  double pol[3][6];  /* drive d: incident amplitude a (re, im of x, y, z) */
  double eps_b;      /* basis permittivity; <= 0 selects the policy below */
} gsm_instance;

typedef struct gsm_solver_opts {
  double tol;         /* stop when ||b - A x||_2 / ||b||_2 <= tol (FP64); default 1e-9 */
  double inner_tol;   /* GSM_MIXED: residual reduction asked of each FP32 Krylov
                         cycle; default 1e-5 */
  int32_t restart;    /* Krylov dimension per cycle, 1..64; default 30 */
  int32_t max_iter;   /* cap on Krylov iterations per system; default 5000 */
  int32_t max_refine; /* cap on FP64 residual evaluations per system; default 200 */
  int32_t precision;  /* GSM_MIXED (complex64 Krylov inside FP64 refinement) or GSM_FP64 */
  int32_t method;     /* GSM_GMRES or GSM_BICGSTAB */
  int32_t flags;      /* GSM_OUT_HOST | GSM_SOLVE_GRAPH | GSM_SOLVE_REORTH */
  const double* x0;   /* NULL or an initial guess (device, layout of E_out) */
  int32_t group_max;  /* systems per launch group, >= 0 (0: no limit); default 32.
                         The systems of a call that share (M, P) are split into
                         groups of at most this many, which the scheduler runs
                         concurrently on its streams, so that the last steps of
                         one group's Krylov cycles, when few of its systems still
                         work, overlap with another group's launches.  The
                         workspace query must be given the same value. */
  int32_t formulation; /* GSM_FORM_E (default) or GSM_FORM_H */
} gsm_solver_opts;

/* Result of one system (instance, drive). */
typedef struct gsm_solve_info {
  int32_t status;      /* GSM_OK, GSM_W_NOT_CONVERGED, GSM_E_SINGULAR */
  int32_t iterations;  /* Krylov iterations (matrix-vector products in the Krylov precision) */
  int32_t refinements; /* FP64 residual evaluations */
  int32_t fft_size;    /* P, the FFT grid per axis */
  int32_t reorth;      /* Arnoldi steps that asked for a second Gram-Schmidt pass */
  int32_t reserved;
  double rel_residual; /* final ||b - A x||_2 / ||b||_2 evaluated in FP64 */
  double eps_b;        /* basis permittivity used */
} gsm_solve_info;

/* ---------------------------------------------------------------- helpers */

int gsm_version(void);
const char* gsm_strerror(int status);
const char* gsm_last_error(void); /* thread-local message of the last failure */

/* Fill opts with the defaults listed above. */
void gsm_solver_opts_default(gsm_solver_opts* opts);

/* FFT grid size P used for order counts M (the smallest supported size with
 * P >= 4 max_a M_a + 1, the condition under which the cropped FFT product
 * equals the truncated Toeplitz product).  Supported: the powers of two 4 ..
 * 512 (M up to 127, the paper's largest Table 1 size); from 256 on the plane
 * pass runs as three kernels with the column-expanded planes in HBM (a plane
 * no longer fits in LDS).  Returns P > 0, or GSM_E_UNSUPPORTED. */
int gsm_fft_size(const int32_t M[3]);

/* CPU-only validation of a geometry, plan options and instances (no device
 * call).  Checks sizes, finiteness, positivity, M ranges and drive counts,
 * and the basis-permittivity choice (GSM_E_SINGULAR if an explicit eps_b
 * gives min_m | |k_m|^2/k0^2 - eps_b | < 1e-3 eps_b).  Any pointer may be NULL
 * to skip its checks (n_inst = 0 skips the instances). */
int gsm_plan_validate(const gsm_geometry* geo, const gsm_plan_opts* opts, int32_t n_inst,
                      const gsm_instance* inst);

/* Basis permittivity the library uses for `inst` with plan `plan`: the
 * instance's eps_b if > 0; otherwise the voxel mean <eps>, unless that comes
 * within 1e-3 eps_b of some |k_m|^2/k0^2, in which case the value in
 * [0.5 eps_min, 2 eps_max] with the largest such margin on a fixed scan. */
int gsm_basis_eps(gsm_plan_t plan, const gsm_instance* inst, double* eps_b);

/* ------------------------------------------------------------------ plan */

/* Build a plan on opts->device: copies the voxels to the device and computes
 * there the exact Fourier coefficients c_n, |n_a| <= 2 m_max[a], of the voxel
 * body (voxel DFT times the box factor sinc(pi n/V) exp(-i pi n/V) per axis).
 * Band-limited real-space contrast grids for each (M, P) are derived from c_n
 * on first use.  The plan owns its device memory. */
int gsm_plan(const gsm_geometry* geo, const gsm_plan_opts* opts, gsm_plan_t* out);
int gsm_plan_destroy(gsm_plan_t plan);

/* Analytic bodies.  The paper builds its Toeplitz matrices from exact
 * Fourier images of simple shapes, spheres and polyhedra combined into a
 * structure ("Calculation details"), rather than from mesh samples.  A
 * shape body is a host permittivity eps_host holding inclusions that overlap
 * neither each other nor their own periodic copies (the caller's
 * responsibility; each inclusion's extent must not exceed the period on any
 * axis, else GSM_E_ARG).  Its coefficients are
 *   c_n = eps_host delta_n0 + sum_i (eps_i - eps_host) S_i(G_n),
 *   S_i(G) = (1/|cell|) integral over inclusion i of exp(-i G.r) dr,
 * G_n = 2 pi (n_x/Lambda_x, n_y/Lambda_y, n_z/Lambda_z), evaluated in FP64
 * on the device: for a sphere of radius R, or an axis-aligned ellipsoid
 * with semi-axes (a, b, c), (volume/|cell|) 3 (sin u - u cos u)/u^3
 * exp(-i G.r0) with u = |(a G_x, b G_y, c G_z)|; for an axis-aligned box with
 * half-sides (a, b, c), (8abc/|cell|) sinc(a G_x) sinc(b G_y) sinc(c G_z)
 * exp(-i G.r0), sinc(x) = sin(x)/x. */
enum { GSM_SHAPE_SPHERE = 0, GSM_SHAPE_ELLIPSOID = 1, GSM_SHAPE_BOX = 2 };
typedef struct gsm_shape {
  int32_t kind;     /* GSM_SHAPE_* */
  int32_t reserved; /* must be 0 */
  double centre[3]; /* r0, in the period's length unit */
  double size[3];   /* sphere: radius in size[0] (others ignored); ellipsoid:
                       semi-axes; box: half-sides; all > 0 */
  double eps;       /* permittivity inside, > 0 */
} gsm_shape;

typedef struct gsm_shape_body {
  double period[3];
  double eps_host;          /* > 0 */
  int32_t n_shapes;         /* >= 0 */
  int32_t reserved;         /* must be 0 */
  const gsm_shape* shapes;  /* host, n_shapes entries; copied */
} gsm_shape_body;

/* Plan of an analytic shape body: as gsm_plan, with the coefficients above
 * in place of the voxel image.  The basis-permittivity policy uses the mean
 * c_0 and the range of eps_host and the inclusions' values.  Gradients with
 * respect to voxels (gsm_eff_tensor_vjp) are refused on such a plan. */
int gsm_plan_shapes(const gsm_shape_body* body, const gsm_plan_opts* opts, gsm_plan_t* out);

/* Coefficients given directly (an image computed elsewhere). */
typedef struct gsm_coeff_body {
  double period[3];
  int32_t n_max[3];     /* the array covers |n_a| <= n_max[a]; needs n_max[a] >= 2 m_max[a] */
  int32_t reserved;     /* must be 0 */
  const double* coef;   /* host complex128 (re, im) [2 n_max z + 1][2 n_max y + 1][2 n_max x + 1],
                           index n_a + n_max[a]; the Fourier image of a real permittivity
                           (c_-n = conj(c_n) to 1e-12 of the largest entry, c_0 > 0), else
                           GSM_E_ARG; copied */
  double eps_min;       /* range of the permittivity, 0 < eps_min <= eps_max: the basis- */
  double eps_max;       /* permittivity policy scans [0.5 eps_min, 2 eps_max] */
  const double* coef_inv; /* NULL, or the image of 1/eps in the layout of coef (needed by the
                             H-field system); copied */
} gsm_coeff_body;

/* Plan from given coefficients: the |n_a| <= 2 m_max[a] block is taken.  As
 * gsm_plan_shapes otherwise (no voxel gradient). */
int gsm_plan_from_coeffs(const gsm_coeff_body* body, const gsm_plan_opts* opts, gsm_plan_t* out);

/* Copy the plan's coefficients c_n to host memory: (4 m_max[2]+1) x
 * (4 m_max[1]+1) x (4 m_max[0]+1) complex128, [nz][ny][nx], index n_a + 2 m_max[a]. */
int gsm_plan_coefficients(gsm_plan_t plan, double* c_out);

/* Copy the plan's coefficients of 1/eps (the H-field system's), layout of
 * gsm_plan_coefficients.  GSM_E_ARG if the plan holds none (a coefficient
 * plan made without coef_inv).  Voxel plans take the exact image of the
 * piecewise-constant 1/eps, shape plans the analytic images with the
 * weights 1/eps_i - 1/eps_host. */
int gsm_plan_inverse_coefficients(gsm_plan_t plan, double* c_out);

/* Copy the band-limited permittivity grid used for order counts M and grid
 * P: eps_M(r_j) = sum_{|n_a| <= 2 M_a} c_n exp(2 pi i n.j / P), real,
 * P^3 doubles [z][y][x] (host). */
int gsm_plan_contrast_grid(gsm_plan_t plan, const int32_t M[3], int32_t P, double* g_out);

/* ------------------------------------------------------------- workspace */

/* Bytes of device workspace gsm_solve, gsm_apply, gsm_solve_adjoint,
 * gsm_eff_tensor and gsm_eff_tensor_vjp need for these instances and options
 * (the caller allocates it, e.g. as a torch uint8 tensor, and may reuse it
 * across calls).  The size covers three drives per instance and the
 * effective-tensor calls' own buffers (solved fields, adjoint right-hand
 * sides and solutions, the correlation grids of the gradient), so none of
 * these calls allocates device memory for its arithmetic.  Plan state is
 * allocated on first need and then kept: the real-space contrast grids of a
 * new (M, P), and the scheduler's pinned host words when a call has more
 * systems than any before (see gsm_allocation_stats). */
int gsm_workspace_size(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst,
                       const gsm_solver_opts* opts, size_t* bytes);

/* ----------------------------------------------------------------- solve */

/* Solve Eq.(4) for every (instance, drive).  Systems of equal (M, P) are
 * batched into the same kernel launches.  E_out receives the fields
 * (complex128, layout above); info (host, one per system) the per-system
 * results.  Returns the worst status.  Synchronises `stream` before
 * returning.  n_inst must be >= 1 (GSM_E_ARG otherwise, nothing launched);
 * with opts->x0 the refinement starts from that field, and one that already
 * meets the tolerance is returned unchanged after one FP64 residual check. */
int gsm_solve(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst,
              const gsm_solver_opts* opts, void* ws, size_t ws_bytes, double* E_out,
              gsm_solve_info* info, void* stream);

/* Apply the operator of Eq.(4) once: y = A x (GSM_APPLY_FORWARD) or
 * y = A^H x (GSM_APPLY_ADJOINT), or that of Eq.(5) (GSM_APPLY_FORWARD_H, see
 * GSM_FORM_H), for every (instance, drive) vector, in
 * complex128 (precision GSM_FP64) or complex64 (GSM_MIXED: x and y are then
 * interleaved float pairs).  Device pointers.  For parity tests and timing. */
int gsm_apply(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst, int32_t precision,
              int32_t mode, const void* x, void* y, void* ws, size_t ws_bytes, void* stream);

/* gsm_apply without a workspace, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same operation, arguments, kernels and results as
 * gsm_apply; the intermediate buffers (per-system parameters, the staged
 * input and output vectors, the FFT pass planes) live instead in a static
 * device array of GSM_APPLY_STATIC_BYTES that the library holds on each
 * device it runs on until the process ends.  The call allocates no device
 * or pinned memory: it never calls hipMalloc or hipFree.
 * - Limit: the systems of one (M, P) group must fit in the array; a larger
 *   call fails with GSM_E_WORKSPACE (split it).  At M = 15 that is about
 *   ten systems in complex128 or twenty in complex64.
 * - The contrast grid of each (M, P) used must already exist on the plan
 *   (made by any earlier gsm_apply, gsm_solve, gsm_eff_tensor or
 *   gsm_plan_contrast_grid with those orders); otherwise GSM_E_ARG.
 * - Every call on one device shares that device's array: calls that overlap
 *   on one device (several host threads or streams) race and must be
 *   serialised by the caller.  The array keeps the last call's contents.
 * Synchronises `stream` before returning, like gsm_apply. */
#define GSM_APPLY_STATIC_BYTES ((size_t)64 << 20)
int gsm_apply_static(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst, int32_t precision,
                     int32_t mode, const void* x, void* y, void* stream);

/* Effective permittivity tensor of each instance (field-averaged form): the
 * three drives a = x, y, z are solved, and with E0 and D0 the zeroth Fourier
 * orders of E and of eps E, eps_eff = D0 E0^-1 (3x3 complex128, row-major,
 * [inst][3][3]).  Its Fresnel zeros det(|k|^2 I - k k^T - k0^2 eps_eff) = 0
 * are the resonances the paper's pole search finds (Eqs.(6)-(10)).  E_save,
 * if not NULL, receives the three solved fields per instance (device, layout
 * of E_out with 3 drives per instance) for gsm_eff_tensor_vjp.  info: 3 per
 * instance. */
int gsm_eff_tensor(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst,
                   const gsm_solver_opts* opts, double* eps_eff, double* E_save, void* ws,
                   size_t ws_bytes, gsm_solve_info* info, void* stream);

/* Adjoint solve A^H lambda = rhs for every (instance, drive); rhs and
 * lambda_out device, layout of E_out.  A^H = I - V^H G^H applies the Green
 * tensor before the contrast convolution (G is real symmetric for real
 * k_inc and eps_b; V is Hermitian for real eps). */
int gsm_solve_adjoint(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst,
                      const gsm_solver_opts* opts, const double* rhs, double* lambda_out,
                      void* ws, size_t ws_bytes, gsm_solve_info* info, void* stream);

/* Vector-Jacobian product of gsm_eff_tensor with respect to the voxel
 * permittivities: given gbar = dL/d conj(eps_eff) per instance (3x3 complex128,
 * host) and the saved fields (device, from gsm_eff_tensor), accumulates
 * dL/d eps_v = 2 Re sum <...> into grad_vox (device, Vz*Vy*Vx doubles).  Runs
 * three adjoint solves per instance; eps_b is held fixed (eps_eff does not
 * depend on it). */
int gsm_eff_tensor_vjp(gsm_plan_t plan, int32_t n_inst, const gsm_instance* inst,
                       const gsm_solver_opts* opts, const double* E_save,
                       const double* eps_eff, const double* gbar, double* grad_vox, void* ws,
                       size_t ws_bytes, gsm_solve_info* info, void* stream);

/* ---------------------------------------------------------- pole search */

/* Mode propagation constants by the pole search of the paper's section on
 * mode propagation, Eqs.(6)-(10).  For one direction k_hat and drive a, the
 * zeroth-order field component xi(kappa) = E_{component, m = 0} of the solve
 * with k_inc = kappa k_hat (all else fixed) is meromorphic in kappa; its
 * poles eta_j are the modes' propagation constants, n_eff = eta / k0.
 * - The mesh: N_d + N_p equidistant kappa over [kappa_min, kappa_max] (one
 *   batched solve of all of them).  Eq.(9) takes one equation from each of
 *   the N_p windows of N_d + 1 consecutive mesh points, with xi_i
 *   multiplying the divided-difference weights 1/prod_{j != i}(kappa_i -
 *   kappa_j) (the printed equation shows it in a denominator); the monic
 *   polynomial's zeros (Eq.(7)) are the eigenvalues of its companion matrix;
 *   the amplitudes zeta_j follow from Eq.(10) with the middle window's nodes.
 * - The basis permittivity is one value for the whole mesh (xi must be one
 *   function of kappa): the query's eps_b if > 0 (GSM_E_SINGULAR if some mesh
 *   point violates the 1e-3 margin), else the plan's mean permittivity if it
 *   keeps the margin at every mesh point, else the value of [0.5 eps_min,
 *   2 eps_max] with the largest smallest margin over the mesh.
 * - The fit (Eq.(9) by Gaussian elimination, the companion matrix by shifted
 *   QR, Eq.(10)) runs in FP64 in a HIP kernel, one thread per query. */
#define GSM_POLE_MAX_NP 8
#define GSM_POLE_MAX_ND 32

typedef struct gsm_pole_query {
  double wavelength;
  double k_hat[3];    /* direction of k_inc (normalised by the library; nonzero) */
  int32_t M[3];       /* order counts */
  int32_t n_poles;    /* N_p, 1 .. GSM_POLE_MAX_NP (the paper suggests about 5) */
  int32_t n_div;      /* N_d, N_p < N_d <= GSM_POLE_MAX_ND (the paper suggests about 10) */
  int32_t component;  /* 0, 1, 2: the x, y or z component of the zeroth order */
  double pol[6];      /* drive a (re, im of x, y, z) */
  double kappa_min;   /* mesh interval of |k_inc|, absolute (1/length), 0 < min < max */
  double kappa_max;
  double eps_b;       /* <= 0: the policy above */
} gsm_pole_query;

typedef struct gsm_pole_result {
  int32_t status;            /* worst status of the mesh solves; GSM_E_SINGULAR if Eq.(9)
                                or the eigenvalue iteration failed */
  int32_t n_poles;
  int32_t best;              /* index of the pole of largest |zeta| among those with real
                                part in [kappa_min, kappa_max] and |imaginary part| at most
                                (kappa_max - kappa_min) / 2 (the modes of a lossless medium
                                are real; poles far off the axis model the regular part of
                                xi); -1 if none */
  int32_t iterations;        /* Krylov iterations summed over the mesh */
  double eta[GSM_POLE_MAX_NP][2];   /* poles (re, im), ascending real part */
  double zeta[GSM_POLE_MAX_NP][2];  /* amplitudes */
  double n_eff;              /* Re eta[best] / k0, 0 if best < 0 */
  double eps_b;              /* the basis permittivity of the mesh */
  double max_rel_residual;   /* over the mesh solves */
} gsm_pole_result;

/* Workspace bytes of gsm_pole_search for these queries and options. */
int gsm_pole_workspace_size(gsm_plan_t plan, int32_t n_q, const gsm_pole_query* q,
                            const gsm_solver_opts* opts, size_t* bytes);

/* Run the mesh solves of every query in one batched call (queries of equal
 * orders share launches) and fit the poles.  out: host, n_q results.
 * Returns the worst status.  Synchronises `stream`. */
int gsm_pole_search(gsm_plan_t plan, int32_t n_q, const gsm_pole_query* q,
                    const gsm_solver_opts* opts, void* ws, size_t ws_bytes, gsm_pole_result* out,
                    void* stream);

/* The fit alone, on samples already on the device: n problems of N_d + N_p
 * points each; kappa [n][N_d + N_p] doubles, xi [n][N_d + N_p] complex128;
 * eta and zeta [n][N_p] complex128 out; status [n] int32 out (GSM_OK or
 * GSM_E_SINGULAR; eta, zeta zero then).  Device pointers, stream-ordered
 * (no synchronisation). */
int gsm_pole_fit(int32_t n, int32_t n_poles, int32_t n_div, const double* kappa, const double* xi,
                 double* eta, double* zeta, int32_t* status, void* stream);

/* ------------------------------------------------ Fresnel normal surface
 * The paper reads the effective tensor off the propagation constants: a
 * direction of the effective medium carries two refractive indices, the
 * roots of the Fresnel normal equation ("Modes in 3D crystals"; in its
 * uniaxial and biaxial examples the principal axes are the lattice axes).
 * A plane wave of unit normal k and index n in a medium of real symmetric
 * permittivity eps obeys (eps - n^2 (I - k k^T)) E = 0, whose determinant is
 * the quadratic (k^T eps k) n^4 - (tr C - k^T C k) n^2 + det(eps), C the
 * adjugate of eps.  Host functions: no device work, any thread. */

/* The two indices of direction k_hat (nonzero, need not be normalised) for
 * eps [3][3] row-major (symmetric; the upper triangle is read), ascending,
 * into n_out[2].  GSM_E_ARG for NULL pointers or a zero direction,
 * GSM_E_NONFINITE for NaN/Inf, GSM_E_SINGULAR when the roots are not both
 * real and positive (eps not positive definite across k). */
int gsm_fresnel_indices(const double* eps, const double* k_hat, double* n_out);

/* Real symmetric tensor whose normal surface passes closest to n_dir
 * observed directions k_hat [n_dir][3] with their two indices each,
 * n_pair [n_dir][2] (either order).  diagonal != 0: principal axes along
 * x, y, z, three values (n_dir >= 3); else all six components (n_dir >= 6).
 * Method: the product of a direction's two roots n1^2 n2^2 is
 * det(eps) / (k^T eps k), linear in eps / det(eps), which gives a linear
 * least-squares estimate; Levenberg-Marquardt steps on the residuals
 * det(eps - n^2 (I - k k^T)) / n^6 (analytic Jacobian from the adjugate)
 * refine it.  eps_out [3][3] row-major; rms_out (may be NULL) the root mean
 * square of those residuals.  GSM_E_ARG for NULL pointers, too few
 * directions, a zero direction or a non-positive index; GSM_E_NONFINITE for
 * NaN/Inf; GSM_E_SINGULAR when the directions do not determine the tensor
 * or the estimate is not positive definite. */
int gsm_fresnel_fit(int32_t n_dir, const double* k_hat, const double* n_pair, int32_t diagonal, double* eps_out,
                    double* rms_out);

/* Launch graphs of a plan so far: *captured = graphs captured and
 * instantiated, *launched = graph launches (each runs a few Krylov steps of
 * one group).  Either pointer may be NULL.  GSM_E_ARG for a NULL plan. */
int gsm_plan_graph_stats(gsm_plan_t plan, int64_t* captured, int64_t* launched);

/* Allocations the library has made since it was loaded: *count calls and
 * *bytes in total of hipMalloc (device) and hipHostMalloc (pinned host).
 * Either pointer may be NULL.  Repeated calls on a plan whose contrast grids
 * and pinned words exist leave both unchanged. */
int gsm_allocation_stats(int64_t* count, int64_t* bytes);

/* Codelet families (0: fewest operations, 1: plain radix 4) used for the
 * orders M with the precision given, per FFT stage: fam[0] pass A (z),
 * fam[1] pass B rows (x), fam[2] pass B columns (y), fam[3] pass C (z).
 * *tuned = 1 when they come from timing (this plan or its cache file),
 * 0 for the fixed defaults. */
int gsm_plan_tuning(gsm_plan_t plan, const int32_t M[3], int32_t precision, int32_t fam[4], int32_t* tuned);

/* ------------------------------------------------------------ profiling */

/* Per-kernel-class statistics of the launches made between
 * gsm_profile_begin and gsm_profile_end on any stream: launch count, summed
 * duration from a hipEvent pair recorded around each launch on its stream,
 * and summed algorithmic bytes (what each launch must read and write by the
 * definition of its step, counted only for the systems that work in it). */
typedef struct gsm_kernel_stat {
  char name[40];    /* e.g. "pass_b_c64", "gs_update1_c64" */
  int64_t launches;
  double ms;
  double bytes;
  double flops;     /* algorithmic real floating-point operations (FFT passes) */
  double bytes_min; /* algorithmic bytes with each launch's grid replaced by the
                       smallest admissible one, P >= 4 max M + 1 with no prime
                       factor above 5 (the bytes model's grid; equal to `bytes`
                       outside the FFT passes) */
} gsm_kernel_stat;

/* Start collecting (clears earlier records).  Calls on different plans may
 * run on several host threads meanwhile; start and end are made from one. */
int gsm_profile_begin(void);
/* The same, recording only the launches of one kernel class, given by its
 * name without the precision suffix (e.g. "pass_b"), so that a timed run
 * carries one event pair per launch of that class only.  GSM_E_ARG for an
 * unknown name. */
int gsm_profile_begin_only(const char* kernel_class);
/* The same (kernel_class may be NULL: every class), timing only one launch
 * in `every` of each class, counted in launch order from this call (the
 * first launch of a class is timed); the statistics cover the timed launches
 * only.  GSM_E_ARG for every < 1 or an unknown name. */
int gsm_profile_begin_sampled(const char* kernel_class, int32_t every);
/* Stop, synchronise the device, write up to `max` entries to out and the
 * number of classes seen to *n_out. */
int gsm_profile_end(gsm_kernel_stat* out, int32_t max, int32_t* n_out);

#ifdef __cplusplus
}
#endif
#endif /* GSM_H */
