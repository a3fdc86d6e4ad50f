// Internal declarations of libgsm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gsm {

constexpr int kMaxRestart = 64;   // largest Krylov dimension per cycle
constexpr int kMaxOrder = 127;    // largest M_a (P = 512)
constexpr int kGsThreads = 256;   // block size of the Gram-Schmidt kernels
#ifndef GSM_GS_PER_THREAD
#define GSM_GS_PER_THREAD 8
#endif
constexpr int kGsPerThread = GSM_GS_PER_THREAD;  // vector elements per thread in those kernels
constexpr int kGsChunk = kGsThreads * kGsPerThread;

template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cplx = typename cplx_t<T>::type;

// Per-system constants (device memory, written once per solve).
struct SysParam {
  double q0[3];      // k_inc / k0
  double b[3];       // lambda / Lambda_a  (= K_a / k0)
  double eps_b;      // basis permittivity
  double inv_eps_b;
  double a[6];       // drive amplitude (re, im) x 3  (incident field at m = 0)
  double bnorm;      // ||a||_2 = ||b||_2 of the right-hand side
  double tol;        // outer relative residual target
  double inner_tol;  // relative reduction asked of one Krylov cycle
  int max_iter;
  int max_refine;
  int pad[2];
  // the plane pass multiplies by conv_a g(r) + conv_b: g = eps, (1/eps_b, -1)
  // for Eq.(4); g = 1/eps, (-eps_b, 1) for Eq.(5)
  double conv_a;
  double conv_b;
};

// Per-system solver state (device memory).
struct SysState {
  int active;        // outer refinement still running
  int inner_active;  // current Krylov cycle still running
  int j;             // Arnoldi steps completed in the current cycle
  int iters;         // total Krylov iterations
  int refinements;   // FP64 residual evaluations
  int status;        // 0 running/converged, 1 not converged
  int reorth;        // step j awaits its second Gram-Schmidt pass (made in the next step's slot)
  int nreorth;       // second passes requested (diagnostics)
  int lag;           // second passes requested in the current cycle: slots the system runs behind
  int pad[3];
  double rho;        // ||r|| of the last FP64 residual
  double rel;        // rho / bnorm
  double vscale;     // scale of the newest basis vector, applied as pass A reads it
  double inner_target;
  double xscale;     // factor applied to the Krylov correction (rho)
  double pad2;
  double2 w0[3];     // zeroth order of the contrast convolution (last FP64 pass)
  double2 brho[2];   // BiCGStab: (rh, r) of iterations of even / odd index
  double2 balpha;    // BiCGStab: alpha of the current iteration
  double2 bomega;    // BiCGStab: omega of the current iteration
  double2 g[kMaxRestart + 1];
  double2 H[(kMaxRestart + 1) * kMaxRestart];  // column j at H[j * (kMaxRestart+1) + i]
  double cs[kMaxRestart];
  double2 sn[kMaxRestart];
  double2 y[kMaxRestart];
  double2 hw[kMaxRestart + 2];   // first-pass Q^H w of the current step, then ||w||^2
  double2 hw2[kMaxRestart + 2];  // second-pass coefficients (when one is made)
  double sigma[kMaxRestart + 1];  // the basis is stored unnormalised: q_k = sigma[k] V_k
};

// Shape of a group: systems sharing (M, P).
struct GroupShape {
  int S;            // systems in the group
  int M[3];
  int N1[3];
  int P;
  int npencil;      // N1x * N1y
  int tstride;      // pencils per intermediate plane: npencil rounded up to 64, so the
                    // pencil segments of pass C blocks (16-64 pencils) start on whole
                    // cache lines and the last block's segment stays inside the plane
  long long n;      // 3 * N1x * N1y * N1z complex values per system
  long long tsize;  // 3 * tstride * P complex values per system (intermediate)
  int nchunk;       // ceil(n / kGsChunk)
  int nblk_c;       // pass C blocks per system
  int form;         // FORM_E: the E-field system of Eq.(4); FORM_H: the H-field system of Eq.(5)
  int reserved;     // zero (no padding bytes in kernel arguments)
};
enum { FORM_E = 0, FORM_H = 1 };

// pass A modes
enum { PA_NORMALIZE = 1, PA_GREEN_PRE = 2 };
// pass C modes
// PC_FWD y = x - G w; PC_RESID r = b - (x - G w) and |r|^2; PC_ADJ y = x - w
// (Green applied in pass A); PC_ADJ_RESID r = rhs - (x - w); PC_CONV y = w;
// PC_GREEN y = G w (the part B = G V of A = I - B, x not read).
enum { PC_FWD = 0, PC_RESID = 1, PC_ADJ = 2, PC_ADJ_RESID = 3, PC_CONV = 4, PC_GREEN = 5 };
// gating of blocks by state
enum { GATE_NONE = 0, GATE_INNER = 1, GATE_OUTER = 2 };

template <typename T>
struct PassArgs {
  GroupShape g;
  const SysParam* par;
  SysState* st;
  cplx<T>* x;           // pass A input / pass C "x"
  cplx<T>* t;           // intermediate (per system stride g.tsize)
  cplx<T>* y;           // pass C output
  const cplx<T>* rhs;   // PC_ADJ_RESID right-hand side, else unused
  long long xs, ys, rs; // per-system strides (complex values) of x, y, rhs
  const T* grid;        // band-limited permittivity, P^3 real [z][y][x]
  double* partial;      // pass C residual partials [S][nblk_c]
  int mode;
  int gate;
  hipEvent_t ev0, ev1;  // when set: stamped at the start and end of the launch
  int fam[4];           // codelet family per stage: pass A, pass B rows, pass B columns, pass C
  int xnorm;            // passes A and C read x scaled by the system's vscale
  int xstep;            // GMRES basis: x and y advance by the system's own step
                        // (x = V_j, y = V_j+1 with j = st.j; x scaled when j > 0)
  cplx<T>* u;           // P >= 256: the plane pass's column-expanded planes [S][3][P][P][N1x]
  long long us;         // per-system stride of u (complex values)
};

// ---- launchers (passes.hip) ----
template <typename T> hipError_t launch_pass_a(const PassArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_pass_b(const PassArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_pass_c(const PassArgs<T>& a, hipStream_t s);
int pass_c_pencils_per_block(int P, bool dbl);
bool fft_size_supported(int P);

// ---- Krylov / refinement kernels (krylov.hip) ----
template <typename T>
struct KrylovArgs {
  GroupShape g;
  const SysParam* par;
  SysState* st;
  cplx<T>* V;          // basis [S][restart+1][n]
  int restart;
  int reorth_all;      // second Gram-Schmidt pass at every step (GSM_SOLVE_REORTH); the int
                       // also keeps the struct free of padding bytes (its bytes key cached launch graphs)
  double2* part1;      // [S][nchunk][restart+2] Gram-Schmidt partial sums
  double* partn;       // [S][nchunk]
  double2* x64;        // [S][n] FP64 iterate
  double2* r64;        // [S][n] FP64 residual
  double* partc;       // [S][nblk_c] pass C residual partials
  int* host_inner;     // pinned host flags, per system (may be null): 0 when the cycle has
                       // ended for it, else 1 + the slots it runs behind (st.lag)
};
template <typename T> hipError_t launch_cgs_dot(const KrylovArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_cgs_update(const KrylovArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_cgs_finish(const KrylovArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_lsq_update(const KrylovArgs<T>& a, hipStream_t s);
template <typename T> hipError_t launch_cast_v0(const KrylovArgs<T>& a, hipStream_t s);
// BiCGStab kernels (bicgstab.inc), selected by `kernel`; its vectors sit in
// these slots of the system's Krylov storage
enum { BI_RH = 0, BI_R = 1, BI_P = 2, BI_V = 3, BI_S = 4, BI_T = 5 };
enum { BICG_INIT, BICG_DOT_RV, BICG_S, BICG_DOT_TS, BICG_XR, BICG_P, BICG_END };
template <typename T>
hipError_t launch_bicg(const KrylovArgs<T>& a, int kernel, int it, int it_cap, hipStream_t s);
hipError_t launch_resid_finalize(const KrylovArgs<double>& a, int fp64_inner, int* flags, hipStream_t s);
hipError_t launch_state_init(const GroupShape& g, SysState* st, double2* x64, const double2* x0,
                             hipStream_t s);

// ---- adjoint of the effective tensor (adjoint.inc) ----
struct AdjInst {
  int M[3];
  int N1[3];
  long long n;          // 3 * N1^3
  int mmax[3];          // plan order bounds (coefficient array is (4 mmax + 1)^3)
  double q0[3], b[3];
  double eps_b;
  double2 w[3][3];      // w_p, p = drive
  double2 u[3][3];      // eps_eff^H w_p
};
hipError_t launch_adjoint_rhs(const double2* coef, const AdjInst& ai, double2* rhs, hipStream_t s);
hipError_t launch_adjoint_weight(const AdjInst& ai, double2* lam, hipStream_t s);
hipError_t launch_conj_mul_acc(const double2* a, const double2* e, double2* y, long long n, hipStream_t s);
hipError_t launch_acc_real(const double2* in, double* out, long long n, double scale, hipStream_t s);
hipError_t launch_rhs_norm(const GroupShape& g, const double2* rhs, SysParam* par, hipStream_t s);
hipError_t launch_zero_start(const GroupShape& g, const SysParam* par, double2* r64, const double2* rhs,
                             double* partc, hipStream_t s);

// ---- plan kernels (plan.hip) ----
// out[o][j][i] = sum_{k<nin} in[o][k][i] * exp(sign 2 pi i ((k+koff)(j+joff) mod Q) / Q)
hipError_t launch_dft_axis(const double2* in, double2* out, int nouter, int nin, int nout,
                           int ninner, int koff, int joff, int Q, int sign, hipStream_t s);
hipError_t launch_real_to_complex(const double* in, double2* out, long long n, hipStream_t s);
hipError_t launch_box_factor(double2* c, const int nc[3], const int vox[3], hipStream_t s);
hipError_t launch_extract_grid(const double2* in, double* g64, float* g32, long long n,
                               hipStream_t s);
hipError_t launch_copy_block(const double2* src, double2* dst, const int src_n[3],
                             const int dst_n[3], const int off[3], hipStream_t s);
// ---- pole search (poles.hip) ----
struct PoleFitArgs {
  int n;              // problems
  int n_poles;        // N_p
  int n_div;          // N_d
  int pad;
  const double* kappa;  // [n][N_d + N_p] mesh
  const double* xi;     // [n][N_d + N_p] complex samples (re, im)
  double* eta;          // [n][N_p] complex poles, ascending real part
  double* zeta;         // [n][N_p] complex amplitudes
  int* status;          // [n] GSM_OK or GSM_E_SINGULAR
};
hipError_t launch_pole_fit(const PoleFitArgs& a, hipStream_t s);
hipError_t launch_gather_zero_order(const double2* E, const long long* idx, double* xi, int n, hipStream_t s);

// one inclusion of an analytic body: kind, centre, radius / semi-axes /
// half-sides, and its weight in the image (eps_i - eps_h, or the difference
// of the inverses)
enum { SHAPE_SPHERE = 0, SHAPE_ELLIPSOID = 1, SHAPE_BOX = 2 };
struct ShapeDesc {
  int kind;
  int pad;
  double centre[3];
  double size[3];
  double weight;
};
// c[nz][ny][nx] (dims nc, index n + (nc-1)/2) = host delta_n0 + sum_k weight_k S_k(G_n)
hipError_t launch_shape_image(double2* c, const int nc[3], const double period[3], double host,
                              const ShapeDesc* sh, int nsh, hipStream_t s);

}  // namespace gsm
