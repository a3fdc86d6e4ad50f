// Host side of libgsm: the C ABI declared in include/gsm.h.
//
// Validation, the basis-permittivity policy, grouping of (instance, drive)
// systems by (M, P), workspace carving, and the solve loop that drives the
// HIP kernels (FP64 residual -> Krylov cycle -> FP64 update, see refine.inc).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gsm.h"
#include "fft_opcount.h"
#include "gsm_internal.h"

using namespace gsm;

// Scratch memory of the allocation-free operator application
// (gsm_apply_static), 64 MiB per device, held until the process ends.
constexpr size_t kScratchBytes = GSM_APPLY_STATIC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? GSM_E_NOMEM : GSM_E_DEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                       \
  } while (0)

constexpr int kSupportedP[] = {4, 8, 16, 32, 36, 40, 48, 64, 72, 128, 256, 512};

int fft_size_for(const int32_t M[3]) {
  int mm = std::max(M[0], std::max(M[1], M[2]));
  for (int p : kSupportedP)
    if (p >= 4 * mm + 1) return p;
  return GSM_E_UNSUPPORTED;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Every device (hipMalloc) and pinned host (hipHostMalloc) allocation of the
// library goes through these, so that gsm_allocation_stats can show which
// calls allocate: plan set-up, the first use of an (M, P) grid and slot
// buffers do; repeated solves on a plan do not.
std::atomic<long long> g_alloc_count{0}, g_alloc_bytes{0};
hipError_t dev_malloc(void** p, size_t bytes) {
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) {
    ++g_alloc_count;
    g_alloc_bytes += (long long)bytes;
  }
  return e;
}
template <typename T> hipError_t dev_malloc(T** p, size_t bytes) { return dev_malloc((void**)p, bytes); }
hipError_t pinned_malloc(void** p, size_t bytes) {
  const hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e == hipSuccess) {
    ++g_alloc_count;
    g_alloc_bytes += (long long)bytes;
  }
  return e;
}

struct Grid {
  double* g64 = nullptr;
  float* g32 = nullptr;
  // codelet families per FFT stage (pass A, pass B rows, pass B columns,
  // pass C) for complex64 [0] and complex128 [1]; tuned[k] once timed
  int fam[2][4] = {};
  bool tuned[2] = {false, false};
};

// Fixed families when not tuned (measured at M = 15, P = 64): the
// fewest-operation codelets everywhere except complex128 pass C, which is
// faster with the plain radix-4 ones.
void default_families(int P, bool dbl, int* fam) {
  (void)P;
  fam[0] = 0;
  fam[1] = 0;
  fam[2] = 0;
  fam[3] = dbl ? 1 : 0;
}

}  // namespace

// Host-side resources of one group in flight: its stream, the events the
// host polls, pinned words the kernels and copies write for the host.
constexpr int kSlots = 4;  // groups of one call in flight at once
constexpr int kRing = 8;   // step events per slot (more than the host's lead)
struct RunSlot {
  hipStream_t stream = nullptr;
  hipEvent_t step_ev[kRing] = {};
  hipEvent_t phase_ev = nullptr;  // residual check or export done
  int* h_flags = nullptr;         // pinned [2 cap]: active flags | steps of the last cycle
  int* h_inner = nullptr;         // pinned [cap]: cycle still running (written by kernels)
  void* h_exp = nullptr;          // pinned [cap] per-system results
  int cap = 0;
  // instantiated launch graphs of Krylov steps, keyed by the bytes of every
  // kernel argument they were captured with (least recently used evicted)
  struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    unsigned long long used = 0;
  };
  std::vector<GraphEntry> graphs;
};
constexpr size_t kGraphsPerSlot = 32;

struct gsm_plan_s {
  int device = 0;
  double period[3]{};
  int vox[3]{1, 1, 1};
  bool voxel_body = false;  // coefficients from voxels (gradients with respect to them are defined)
  int mmax[3]{};
  int nc[3]{};  // 4 m_max + 1
  double eps_mean = 0, eps_min = 0, eps_max = 0;
  double2* d_coef = nullptr;
  double2* d_coef_inv = nullptr;  // image of 1/eps (the H-field system); null if not given
  // real-space grids per (M, P, kind): kind 0 the permittivity (Eq.(4)),
  // kind 1 its inverse (Eq.(5))
  std::map<std::array<int, 5>, Grid> grids;
  RunSlot slots[kSlots];
  bool autotune = false;
  std::string tune_cache;  // file of tuning results ("" = none)
  std::string arch;        // device architecture name, the cache's key
  // cached tuning results by (M, P, precision)
  std::map<std::array<int, 5>, std::array<int, 4>> tune_known;
  // basis permittivities already resolved for an instance: key = the bytes
  // of (wavelength, k_inc, M, requested eps_b); the result also depends only
  // on the plan's periods and permittivity statistics
  std::map<std::array<unsigned char, 60>, double> eps_b_known;
  long long graph_captures = 0, graph_launches = 0;
  unsigned long long graph_clock = 0;  // use counter for the graph caches
  bool graph_off = false;              // set if a capture ever fails: separate launches from then on
};

namespace {

// ----------------------------------------------------------- validation ----

int check_geometry(const gsm_geometry* geo) {
  if (!geo) return fail(GSM_E_ARG, "geometry is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(geo->period[a])) return fail(GSM_E_NONFINITE, "period[%d] is not finite", a);
    if (!(geo->period[a] > 0)) return fail(GSM_E_ARG, "period[%d] must be > 0", a);
    if (geo->nvox[a] < 1 || geo->nvox[a] > 4096) return fail(GSM_E_ARG, "nvox[%d]=%d out of range", a, geo->nvox[a]);
  }
  if (!geo->eps) return fail(GSM_E_ARG, "eps is NULL");
  const long long nv = (long long)geo->nvox[0] * geo->nvox[1] * geo->nvox[2];
  if (nv > (1LL << 28)) return fail(GSM_E_ARG, "too many voxels");
  for (long long i = 0; i < nv; ++i) {
    if (!std::isfinite(geo->eps[i])) return fail(GSM_E_NONFINITE, "eps[%lld] is not finite", i);
    if (!(geo->eps[i] > 0)) return fail(GSM_E_ARG, "eps[%lld] must be > 0", i);
  }
  return GSM_OK;
}

int check_plan_opts(const gsm_plan_opts* o) {
  if (!o) return fail(GSM_E_ARG, "plan options are NULL");
  for (int a = 0; a < 3; ++a)
    if (o->m_max[a] < 0 || o->m_max[a] > kMaxOrder)
      return fail(GSM_E_UNSUPPORTED, "m_max[%d]=%d outside [0, %d]", a, o->m_max[a], kMaxOrder);
  if (o->flags & ~GSM_PLAN_AUTOTUNE) return fail(GSM_E_ARG, "unknown plan flags");
  if (o->reserved != 0) return fail(GSM_E_ARG, "reserved plan field must be 0");
  return GSM_OK;
}

int check_shape_body(const gsm_shape_body* b) {
  if (!b) return fail(GSM_E_ARG, "shape body is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(b->period[a])) return fail(GSM_E_NONFINITE, "period[%d] is not finite", a);
    if (!(b->period[a] > 0)) return fail(GSM_E_ARG, "period[%d] must be > 0", a);
  }
  if (!std::isfinite(b->eps_host)) return fail(GSM_E_NONFINITE, "eps_host is not finite");
  if (!(b->eps_host > 0)) return fail(GSM_E_ARG, "eps_host must be > 0");
  if (b->n_shapes < 0 || (b->n_shapes > 0 && !b->shapes)) return fail(GSM_E_ARG, "bad shape list");
  if (b->reserved != 0) return fail(GSM_E_ARG, "reserved shape-body field must be 0");
  for (int k = 0; k < b->n_shapes; ++k) {
    const gsm_shape& sh = b->shapes[k];
    if (sh.kind != GSM_SHAPE_SPHERE && sh.kind != GSM_SHAPE_ELLIPSOID && sh.kind != GSM_SHAPE_BOX)
      return fail(GSM_E_ARG, "shape %d: unknown kind %d", k, sh.kind);
    if (sh.reserved != 0) return fail(GSM_E_ARG, "shape %d: reserved field must be 0", k);
    if (!std::isfinite(sh.eps)) return fail(GSM_E_NONFINITE, "shape %d: eps is not finite", k);
    if (!(sh.eps > 0)) return fail(GSM_E_ARG, "shape %d: eps must be > 0", k);
    const int nsz = sh.kind == GSM_SHAPE_SPHERE ? 1 : 3;
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(sh.centre[a])) return fail(GSM_E_NONFINITE, "shape %d: centre is not finite", k);
      const double sz = sh.size[a < nsz ? a : 0];
      if (!std::isfinite(sz)) return fail(GSM_E_NONFINITE, "shape %d: size is not finite", k);
      if (!(sz > 0)) return fail(GSM_E_ARG, "shape %d: size must be > 0", k);
      // the image formula needs the body apart from its own periodic copies
      if (2.0 * sz > b->period[a])
        return fail(GSM_E_ARG, "shape %d: extent %g along axis %d exceeds the period %g", k, 2.0 * sz, a,
                    b->period[a]);
    }
  }
  return GSM_OK;
}

int check_coeff_body(const gsm_coeff_body* b, const gsm_plan_opts* o) {
  if (!b) return fail(GSM_E_ARG, "coefficient body is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(b->period[a])) return fail(GSM_E_NONFINITE, "period[%d] is not finite", a);
    if (!(b->period[a] > 0)) return fail(GSM_E_ARG, "period[%d] must be > 0", a);
    if (b->n_max[a] < 2 * o->m_max[a])
      return fail(GSM_E_ARG, "n_max[%d]=%d < 2 m_max[%d]=%d: the Toeplitz matrix needs |n| <= 2 M", a, b->n_max[a], a,
                  2 * o->m_max[a]);
  }
  if (b->reserved != 0) return fail(GSM_E_ARG, "reserved coefficient-body field must be 0");
  if (!b->coef) return fail(GSM_E_ARG, "coefficients are NULL");
  if (!(std::isfinite(b->eps_min) && std::isfinite(b->eps_max)))
    return fail(GSM_E_NONFINITE, "eps_min / eps_max not finite");
  if (!(b->eps_min > 0 && b->eps_max >= b->eps_min)) return fail(GSM_E_ARG, "need 0 < eps_min <= eps_max");
  const long long sx = 2LL * b->n_max[0] + 1, sy = 2LL * b->n_max[1] + 1, sz = 2LL * b->n_max[2] + 1;
  const long long n = sx * sy * sz;
  const long long i0 = (long long)(b->n_max[2] * sy + b->n_max[1]) * sx + b->n_max[0];
  // the image of a real function: c_{-n} = conj(c_n) (the real-space grid
  // keeps only the real part), c_0 real and positive
  auto check = [&](const double* c, const char* what) -> int {
    double big = 0;
    for (long long i = 0; i < 2 * n; ++i) {
      if (!std::isfinite(c[i])) return fail(GSM_E_NONFINITE, "%s: coefficient %lld is not finite", what, i / 2);
      big = std::max(big, std::fabs(c[i]));
    }
    for (long long i = 0; i < n; ++i) {
      const long long j = n - 1 - i;  // index of -n
      if (std::fabs(c[2 * i] - c[2 * j]) > 1e-12 * big || std::fabs(c[2 * i + 1] + c[2 * j + 1]) > 1e-12 * big)
        return fail(GSM_E_ARG, "%s are not those of a real function (c_-n != conj(c_n) at entry %lld)", what, i);
    }
    if (!(c[2 * i0] > 0)) return fail(GSM_E_ARG, "%s: c_0 (the mean) must be > 0", what);
    return GSM_OK;
  };
  int rc;
  if ((rc = check(b->coef, "coefficients"))) return rc;
  if (b->coef_inv && (rc = check(b->coef_inv, "inverse-permittivity coefficients"))) return rc;
  return GSM_OK;
}

int check_instance(const gsm_instance& in, const int* mmax, int i, bool need_drives) {
  if (!std::isfinite(in.wavelength)) return fail(GSM_E_NONFINITE, "instance %d: wavelength not finite", i);
  if (!(in.wavelength > 0)) return fail(GSM_E_ARG, "instance %d: wavelength must be > 0", i);
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(in.k_inc[a])) return fail(GSM_E_NONFINITE, "instance %d: k_inc not finite", i);
    if (in.M[a] < 0 || in.M[a] > kMaxOrder) return fail(GSM_E_UNSUPPORTED, "instance %d: M[%d]=%d", i, a, in.M[a]);
    if (mmax && in.M[a] > mmax[a])
      return fail(GSM_E_ARG, "instance %d: M[%d]=%d exceeds plan m_max %d", i, a, in.M[a], mmax[a]);
  }
  if (!std::isfinite(in.eps_b)) return fail(GSM_E_NONFINITE, "instance %d: eps_b not finite", i);
  if (need_drives) {
    if (in.n_drive < 1 || in.n_drive > 3) return fail(GSM_E_ARG, "instance %d: n_drive=%d", i, in.n_drive);
    for (int d = 0; d < in.n_drive; ++d) {
      double nn = 0;
      for (int c = 0; c < 6; ++c) {
        if (!std::isfinite(in.pol[d][c])) return fail(GSM_E_NONFINITE, "instance %d: pol not finite", i);
        nn += in.pol[d][c] * in.pol[d][c];
      }
      if (nn == 0) return fail(GSM_E_ARG, "instance %d: drive %d is zero", i, d);
    }
  }
  return GSM_OK;
}

int check_solver_opts(const gsm_solver_opts* s) {
  if (!s) return fail(GSM_E_ARG, "solver options are NULL");
  if (!std::isfinite(s->tol) || !std::isfinite(s->inner_tol)) return fail(GSM_E_NONFINITE, "tolerance not finite");
  if (s->restart < 1 || s->restart > kMaxRestart) return fail(GSM_E_ARG, "restart=%d outside [1, %d]", s->restart, kMaxRestart);
  if (s->max_iter < 1) return fail(GSM_E_ARG, "max_iter must be >= 1");
  if (s->max_refine < 1) return fail(GSM_E_ARG, "max_refine must be >= 1");
  if (s->precision != GSM_MIXED && s->precision != GSM_FP64) return fail(GSM_E_ARG, "unknown precision %d", s->precision);
  if (s->method != GSM_GMRES && s->method != GSM_BICGSTAB) return fail(GSM_E_ARG, "unknown method %d", s->method);
  if (s->method == GSM_BICGSTAB && s->restart < 5)
    return fail(GSM_E_ARG, "BiCGStab keeps six vectors per system: restart must be >= 5");
  if (s->flags & ~(GSM_OUT_HOST | GSM_SOLVE_GRAPH | GSM_SOLVE_REORTH)) return fail(GSM_E_ARG, "unknown solver flags");
  if (s->group_max < 0) return fail(GSM_E_ARG, "group_max must be >= 0");
  if (s->formulation != GSM_FORM_E && s->formulation != GSM_FORM_H)
    return fail(GSM_E_ARG, "unknown formulation %d", s->formulation);
  return GSM_OK;
}

// -------------------------------------------------- basis permittivity ----

// min over the truncated harmonic set of | |q_m|^2 - eb |.  For fixed
// (my, mz), g(mx) = (q0x + mx bx)^2 + r is a convex quadratic in mx, so over
// the integers of [-Mx, Mx] |g| is smallest next to a root of g, next to its
// vertex (g > 0 everywhere), or at an end of the range (the roots outside
// it): at most eight candidates per (my, mz) instead of the whole row, each
// evaluated as in a full scan, so the minimum is the same number.
double margin_scan(const gsm_instance& in, const double* period, double eb) {
  const double k0 = 2.0 * M_PI / in.wavelength;
  double q0[3], b[3];
  for (int a = 0; a < 3; ++a) {
    q0[a] = in.k_inc[a] / k0;
    b[a] = in.wavelength / period[a];  // > 0
  }
  const int Mx = in.M[0];
  auto clampi = [&](double v) { return v < -Mx ? -Mx : (v > Mx ? Mx : (int)v); };
  const double fv = std::floor(-q0[0] / b[0]);  // the vertex lies in [fv, fv + 1]
  double m = INFINITY;
  for (int mz = -in.M[2]; mz <= in.M[2]; ++mz) {
    const double qz = q0[2] + mz * b[2];
    for (int my = -in.M[1]; my <= in.M[1]; ++my) {
      const double qy = q0[1] + my * b[1];
      const double r = qy * qy + qz * qz - eb;
      int c[8] = {-Mx, Mx, clampi(fv), clampi(fv + 1), 0, 0, 0, 0};
      int nc = 4;
      if (r < 0) {
        const double sr = std::sqrt(-r);
        const double f1 = std::floor((sr - q0[0]) / b[0]), f2 = std::floor((-sr - q0[0]) / b[0]);
        c[nc++] = clampi(f1);
        c[nc++] = clampi(f1 + 1);
        c[nc++] = clampi(f2);
        c[nc++] = clampi(f2 + 1);
      }
      for (int i = 0; i < nc; ++i) {
        const double qx = q0[0] + c[i] * b[0];
        m = std::min(m, std::fabs(qx * qx + r));
      }
    }
  }
  return m;
}

// sorted |q_m|^2 over the truncated harmonic set
std::vector<double> shell_values(const gsm_instance& in, const double* period) {
  const double k0 = 2.0 * M_PI / in.wavelength;
  double q0[3], b[3];
  for (int a = 0; a < 3; ++a) {
    q0[a] = in.k_inc[a] / k0;
    b[a] = in.wavelength / period[a];
  }
  std::vector<double> v;
  v.reserve((size_t)(2 * in.M[0] + 1) * (2 * in.M[1] + 1) * (2 * in.M[2] + 1));
  for (int mz = -in.M[2]; mz <= in.M[2]; ++mz)
    for (int my = -in.M[1]; my <= in.M[1]; ++my)
      for (int mx = -in.M[0]; mx <= in.M[0]; ++mx) {
        const double qx = q0[0] + mx * b[0], qy = q0[1] + my * b[1], qz = q0[2] + mz * b[2];
        v.push_back(qx * qx + qy * qy + qz * qz);
      }
  std::sort(v.begin(), v.end());
  return v;
}

double margin_of(const std::vector<double>& sorted, double eb) {
  auto it = std::lower_bound(sorted.begin(), sorted.end(), eb);
  double m = INFINITY;
  if (it != sorted.end()) m = std::min(m, std::fabs(*it - eb));
  if (it != sorted.begin()) m = std::min(m, std::fabs(*(it - 1) - eb));
  return m;
}

constexpr double kSingularRel = 1e-3;

int resolve_eps_b(const double* period, double eps_mean, double eps_min, double eps_max, const gsm_instance& in,
                  int idx, double* out) {
  if (in.eps_b > 0) {
    if (margin_scan(in, period, in.eps_b) < kSingularRel * in.eps_b)
      return fail(GSM_E_SINGULAR, "instance %d: |k_m|^2 = k_b^2 within 1e-3 for eps_b=%g", idx, in.eps_b);
    *out = in.eps_b;
    return GSM_OK;
  }
  if (margin_scan(in, period, eps_mean) >= kSingularRel * eps_mean) {
    *out = eps_mean;
    return GSM_OK;
  }
  const std::vector<double> sh = shell_values(in, period);
  const double lo = 0.5 * eps_min, hi = 2.0 * eps_max;
  double best = -1, best_eb = eps_mean;
  const int n = 4001;
  for (int i = 0; i < n; ++i) {
    const double eb = lo + (hi - lo) * i / (n - 1);
    const double r = margin_of(sh, eb) / eb;
    if (r > best) {
      best = r;
      best_eb = eb;
    }
  }
  if (best < kSingularRel) return fail(GSM_E_SINGULAR, "instance %d: no admissible eps_b", idx);
  *out = best_eb;
  return GSM_OK;
}

// ------------------------------------------------------------- systems ----

struct SysDesc {
  int inst, drive;
  int form;  // FORM_E or FORM_H
  int M[3];
  int P;
  long long n;        // complex values
  long long out_off;  // complex offset in E_out
  SysParam par;
};

struct Group {
  GroupShape shape{};
  std::vector<int> sys;
  // workspace
  SysParam* par = nullptr;
  SysState* st = nullptr;
  int* flags = nullptr;
  double2* x64 = nullptr;
  double2* r64 = nullptr;
  double2* rhs64 = nullptr;  // general right-hand sides (adjoint solve)
  void* V = nullptr;
  double2* T = nullptr;
  double2* U = nullptr;  // P >= 256: the plane pass's column-expanded planes
  double2* part1 = nullptr;
  double* partn = nullptr;
  double* partc = nullptr;
  long long* off = nullptr;   // [S] offsets of the systems in the caller's flat layout (complex values)
  void* exp = nullptr;        // [S] per-system results read back at the end
};

struct SysExport {
  int status, iters, refinements, reorth;
  double rel;
  double2 e0[3];
  double2 w0[3];
};

int build_systems(gsm_plan_s* plan, int n_inst, const gsm_instance* inst, const gsm_solver_opts* so,
                  bool three_drives, std::vector<SysDesc>& sys) {
  sys.clear();
  long long off = 0;
  for (int i = 0; i < n_inst; ++i) {
    const gsm_instance& in = inst[i];
    int rc = check_instance(in, plan->mmax, i, !three_drives);
    if (rc) return rc;
    double eb;
    std::array<unsigned char, 60> key;
    std::memcpy(key.data(), &in.wavelength, 8);
    std::memcpy(key.data() + 8, in.k_inc, 24);
    std::memcpy(key.data() + 32, in.M, 12);
    std::memcpy(key.data() + 44, &in.eps_b, 8);
    std::memset(key.data() + 52, 0, 8);
    const auto known = plan->eps_b_known.find(key);
    if (known != plan->eps_b_known.end()) {
      eb = known->second;
    } else {
      rc = resolve_eps_b(plan->period, plan->eps_mean, plan->eps_min, plan->eps_max, in, i, &eb);
      if (rc) return rc;
      if (plan->eps_b_known.size() >= 65536) plan->eps_b_known.clear();
      plan->eps_b_known[key] = eb;
    }
    const int P = fft_size_for(in.M);
    if (P < 0) return fail(GSM_E_UNSUPPORTED, "instance %d: order count too large", i);
    const int nd = three_drives ? 3 : in.n_drive;
    for (int d = 0; d < nd; ++d) {
      SysDesc s{};
      s.inst = i;
      s.drive = d;
      for (int a = 0; a < 3; ++a) s.M[a] = in.M[a];
      s.P = P;
      s.n = 3LL * (2 * in.M[0] + 1) * (2 * in.M[1] + 1) * (2 * in.M[2] + 1);
      s.out_off = off;
      off += s.n;
      const double k0 = 2.0 * M_PI / in.wavelength;
      for (int a = 0; a < 3; ++a) {
        s.par.q0[a] = in.k_inc[a] / k0;
        s.par.b[a] = in.wavelength / plan->period[a];
      }
      s.par.eps_b = eb;
      s.par.inv_eps_b = 1.0 / eb;
      s.form = (so && so->formulation == GSM_FORM_H) ? FORM_H : FORM_E;
      s.par.conv_a = s.form == FORM_H ? -eb : 1.0 / eb;
      s.par.conv_b = s.form == FORM_H ? 1.0 : -1.0;
      double nn = 0;
      for (int c = 0; c < 3; ++c) {
        double re, im;
        if (three_drives) {
          re = (c == d) ? 1.0 : 0.0;
          im = 0.0;
        } else {
          re = in.pol[d][2 * c];
          im = in.pol[d][2 * c + 1];
        }
        s.par.a[2 * c] = re;
        s.par.a[2 * c + 1] = im;
        nn += re * re + im * im;
      }
      s.par.bnorm = std::sqrt(nn);
      if (so) {
        s.par.tol = so->tol;
        s.par.inner_tol = so->inner_tol;
        s.par.max_iter = so->max_iter;
        s.par.max_refine = so->max_refine;
      }
      sys.push_back(s);
    }
  }
  return GSM_OK;
}

// Systems sharing (M, P) form a group, split into groups of at most
// group_max systems (0: no limit).
void build_groups(const std::vector<SysDesc>& sys, std::vector<Group>& groups, int group_max) {
  groups.clear();
  std::map<std::array<int, 4>, int> key2g;
  for (int i = 0; i < (int)sys.size(); ++i) {
    const SysDesc& s = sys[i];
    std::array<int, 4> key{s.M[0], s.M[1], s.M[2], s.P};
    auto it = key2g.find(key);
    if (it == key2g.end() || (group_max > 0 && (int)groups[it->second].sys.size() >= group_max)) {
      Group g;
      GroupShape& sh = g.shape;
      for (int a = 0; a < 3; ++a) {
        sh.M[a] = s.M[a];
        sh.N1[a] = 2 * s.M[a] + 1;
      }
      sh.P = s.P;
      sh.form = s.form;
      sh.npencil = sh.N1[0] * sh.N1[1];
      sh.n = 3LL * sh.npencil * sh.N1[2];
      sh.tstride = (sh.npencil + 63) / 64 * 64;
      sh.tsize = 3LL * sh.tstride * s.P;
      sh.nchunk = (int)((sh.n + kGsChunk - 1) / kGsChunk);
      key2g[key] = (int)groups.size();
      groups.push_back(g);
      it = key2g.find(key);
    }
    groups[it->second].sys.push_back(i);
  }
  for (auto& g : groups) g.shape.S = (int)g.sys.size();
}

// Complex values per system of the plane pass's intermediate U[c][z][y][mx]
// on the grids whose planes do not fit in LDS (P >= 256), else 0.
long long plane_split_size(const GroupShape& sh) {
  return sh.P >= 256 ? 3LL * sh.P * sh.P * sh.N1[0] : 0;
}

// Carve one group's buffers from base (base == nullptr: size only).
size_t layout_group(Group& g, char* base, int restart, size_t vbytes, int nblk_c) {
  const long long S = g.shape.S, n = g.shape.n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return (void*)p;
  };
  g.par = (SysParam*)take(S * sizeof(SysParam));
  g.st = (SysState*)take(S * sizeof(SysState));
  g.flags = (int*)take(2 * S * sizeof(int));  // [active flags | steps of the last cycle]
  g.x64 = (double2*)take(S * n * sizeof(double2));
  g.r64 = (double2*)take(S * n * sizeof(double2));
  g.rhs64 = (double2*)take(S * n * sizeof(double2));
  g.V = take(S * (restart + 1) * n * vbytes);
  g.T = (double2*)take(S * g.shape.tsize * sizeof(double2));
  g.U = (double2*)take(S * plane_split_size(g.shape) * sizeof(double2));
  g.part1 = (double2*)take(S * g.shape.nchunk * (restart + 2) * sizeof(double2));
  g.partn = (double*)take(S * g.shape.nchunk * sizeof(double));
  g.partc = (double*)take(S * nblk_c * sizeof(double));
  g.off = (long long*)take(S * sizeof(long long));
  g.exp = take(S * sizeof(SysExport));
  return off;
}

int nblk_c_for(const GroupShape& sh, bool dbl) {
  const int npb = pass_c_pencils_per_block(sh.P, dbl);
  return (sh.npencil + npb - 1) / npb;
}

size_t workspace_for(std::vector<Group>& groups, int restart, bool fp64) {
  size_t total = 0;
  for (auto& g : groups) {
    // the pass C partials are written by the FP64 residual pass
    g.shape.nblk_c = nblk_c_for(g.shape, true);
    total += layout_group(g, nullptr, restart, fp64 ? sizeof(double2) : sizeof(float2),
                          std::max(nblk_c_for(g.shape, true), nblk_c_for(g.shape, false)));
  }
  return total + 256;
}

int carve(std::vector<Group>& groups, void* ws, size_t ws_bytes, int restart, bool fp64) {
  const size_t need = workspace_for(groups, restart, fp64);
  if (!ws) return fail(GSM_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(GSM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  char* p = (char*)(((uintptr_t)ws + 255) & ~uintptr_t(255));
  for (auto& g : groups) {
    const size_t sz = layout_group(g, p, restart, fp64 ? sizeof(double2) : sizeof(float2),
                                   std::max(nblk_c_for(g.shape, true), nblk_c_for(g.shape, false)));
    p += sz;
  }
  return GSM_OK;
}

// ----------------------------------------------- effective-tensor region --
// Workspace of gsm_eff_tensor and gsm_eff_tensor_vjp beyond the groups'
// solve buffers: two field arrays over the three-drive systems of the call
// (the solved fields when the caller keeps none; the adjoint right-hand sides
// and solutions), and the correlation buffers of one instance at a time
// (sized for the largest): two DFT staging arrays, the two expanded fields,
// the real-space product on the P^3 grid, the |n| <= 2M coefficients and the
// voxel-space result.
enum { AUX_T1, AUX_T2, AUX_AH, AUX_EH, AUX_Y, AUX_X, AUX_GV, AUX_NTMP };

void vjp_tmp_counts(const gsm_plan_s* plan, const SysDesc& s0, long long cnt[AUX_NTMP]) {
  const long long P = s0.P, P3 = P * P * P;
  const long long N1[3] = {2LL * s0.M[0] + 1, 2LL * s0.M[1] + 1, 2LL * s0.M[2] + 1};
  const long long nc[3] = {4LL * s0.M[0] + 1, 4LL * s0.M[1] + 1, 4LL * s0.M[2] + 1};
  const long long ncn = nc[0] * nc[1] * nc[2];
  const long long nvox = (long long)plan->vox[0] * plan->vox[1] * plan->vox[2];
  const long long tsz = std::max<long long>({P3, N1[2] * N1[1] * P, N1[2] * P * P, P * P * nc[0], P * nc[1] * nc[0],
                                             nc[2] * nc[1] * plan->vox[0], nc[2] * plan->vox[1] * plan->vox[0]});
  cnt[AUX_T1] = cnt[AUX_T2] = tsz;
  cnt[AUX_AH] = cnt[AUX_EH] = cnt[AUX_Y] = P3;
  cnt[AUX_X] = ncn;
  cnt[AUX_GV] = std::max(nvox, ncn);
}

struct Aux {
  double2* f[2] = {nullptr, nullptr};
  double2* tmp[AUX_NTMP] = {};
};

// Bytes of the region for three-drive systems `sys` (base == nullptr: size only).
size_t aux_layout(const gsm_plan_s* plan, const std::vector<SysDesc>& sys, char* base, Aux* out) {
  long long total = 0;
  for (auto& s : sys) total += s.n;
  size_t off = 0;
  auto take = [&](long long count) {
    double2* q = base ? (double2*)(base + off) : nullptr;
    off += align256((size_t)std::max<long long>(count, 1) * sizeof(double2));
    return q;
  };
  Aux a;
  a.f[0] = take(total);
  a.f[1] = take(total);
  long long cmax[AUX_NTMP] = {};
  for (size_t i = 0; i < sys.size(); i += 3) {
    long long c[AUX_NTMP];
    vjp_tmp_counts(plan, sys[i], c);
    for (int k = 0; k < AUX_NTMP; ++k) cmax[k] = std::max(cmax[k], c[k]);
  }
  for (int k = 0; k < AUX_NTMP; ++k) a.tmp[k] = take(cmax[k]);
  if (out) *out = a;
  return off;
}

// The region follows the groups' buffers in the caller's workspace.
int carve_aux(const gsm_plan_s* plan, std::vector<Group>& groups, const std::vector<SysDesc>& sys, void* ws,
              size_t ws_bytes, int restart, bool fp64, Aux* out) {
  const size_t gbytes = workspace_for(groups, restart, fp64);
  const size_t need = gbytes + aux_layout(plan, sys, nullptr, nullptr);
  if (!ws) return fail(GSM_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(GSM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  // gbytes holds 256 bytes of slack for aligning the start of the groups
  char* p = (char*)(((uintptr_t)ws + 255) & ~uintptr_t(255)) + (gbytes - 256);
  aux_layout(plan, sys, p, out);
  return GSM_OK;
}

// ------------------------------------------------------------ plan grids --

int ensure_grid(gsm_plan_s* plan, const int M[3], int P, hipStream_t st, Grid** out, int kind = FORM_E) {
  std::array<int, 5> key{M[0], M[1], M[2], P, kind};
  auto it = plan->grids.find(key);
  if (it != plan->grids.end()) {
    *out = &it->second;
    return GSM_OK;
  }
  Grid g;
  const long long P3 = (long long)P * P * P;
  const int nb[3] = {4 * M[0] + 1, 4 * M[1] + 1, 4 * M[2] + 1};
  const long long nbt = (long long)nb[0] * nb[1] * nb[2];
  double2 *blk = nullptr, *t1 = nullptr, *t2 = nullptr;
  HIP_TRY(dev_malloc(&g.g64, P3 * sizeof(double)));
  HIP_TRY(dev_malloc(&g.g32, P3 * sizeof(float)));
  HIP_TRY(dev_malloc(&blk, nbt * sizeof(double2)));
  HIP_TRY(dev_malloc(&t1, std::max((long long)P * nb[1] * nb[2], P3) * sizeof(double2)));
  HIP_TRY(dev_malloc(&t2, P3 * sizeof(double2)));
  const int off[3] = {2 * plan->mmax[0] - 2 * M[0], 2 * plan->mmax[1] - 2 * M[1], 2 * plan->mmax[2] - 2 * M[2]};
  const double2* src = kind == FORM_H ? plan->d_coef_inv : plan->d_coef;
  if (!src) {
    hipFree(g.g64);
    hipFree(g.g32);
    hipFree(blk);
    hipFree(t1);
    hipFree(t2);
    return fail(GSM_E_ARG, "the plan holds no inverse-permittivity coefficients (the H-field system needs them)");
  }
  HIP_TRY(launch_copy_block(src, blk, plan->nc, nb, off, st));
  // x: blk[nz][ny][nbx] -> t1[nz][ny][P]
  HIP_TRY(launch_dft_axis(blk, t1, nb[2] * nb[1], nb[0], P, 1, -2 * M[0], 0, P, +1, st));
  // y: t1[nz][nby][P] -> t2[nz][P][P]
  HIP_TRY(launch_dft_axis(t1, t2, nb[2], nb[1], P, P, -2 * M[1], 0, P, +1, st));
  // z: t2[nbz][P*P] -> t1[P][P*P]
  HIP_TRY(launch_dft_axis(t2, t1, 1, nb[2], P, P * P, -2 * M[2], 0, P, +1, st));
  HIP_TRY(launch_extract_grid(t1, g.g64, g.g32, P3, st));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipFree(blk));
  HIP_TRY(hipFree(t1));
  HIP_TRY(hipFree(t2));
  for (int d = 0; d < 2; ++d) {
    default_families(P, d == 1, g.fam[d]);
    auto tk = plan->tune_known.find({M[0], M[1], M[2], P, d});
    if (tk != plan->tune_known.end()) {
      for (int k = 0; k < 4; ++k) g.fam[d][k] = tk->second[k];
      g.tuned[d] = true;
    }
  }
  plan->grids[key] = g;
  *out = &plan->grids[key];
  return GSM_OK;
}

int ensure_slot(gsm_plan_s* plan, int k, int S, size_t exp_bytes) {
  RunSlot& sl = plan->slots[k];
  if (!sl.stream) {
    HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    for (int j = 0; j < kRing; ++j) HIP_TRY(hipEventCreateWithFlags(&sl.step_ev[j], hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&sl.phase_ev, hipEventDisableTiming));
  }
  if (sl.cap >= S) return GSM_OK;
  if (sl.h_flags) HIP_TRY(hipHostFree(sl.h_flags));
  if (sl.h_inner) HIP_TRY(hipHostFree(sl.h_inner));
  if (sl.h_exp) HIP_TRY(hipHostFree(sl.h_exp));
  sl.h_flags = sl.h_inner = nullptr;
  sl.h_exp = nullptr;
  sl.cap = 0;
  const int cap = std::max(S, 64);
  HIP_TRY(pinned_malloc((void**)&sl.h_flags, 2 * cap * sizeof(int)));
  HIP_TRY(pinned_malloc((void**)&sl.h_inner, cap * sizeof(int)));
  HIP_TRY(pinned_malloc(&sl.h_exp, cap * exp_bytes));
  sl.cap = cap;
  return GSM_OK;
}

// ---------------------------------------------------------------- kernels --

// Copies between a group's contiguous [S][n] field array and the places of
// its systems in the caller's flat layout (offsets in complex values).
__global__ void __launch_bounds__(256) k_move_fields(double2* grp, double2* flat, const long long* off, long long n,
                                                     int to_flat) {
  const int s = blockIdx.y;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double2* a = grp + (long long)s * n + i;
  double2* b = flat + off[s] + i;
  if (to_flat)
    *b = *a;
  else
    *a = *b;
}

hipError_t move_fields(const Group& g, double2* grp, const double* flat, bool to_flat, hipStream_t st) {
  hipLaunchKernelGGL(k_move_fields, dim3((unsigned)((g.shape.n + 255) / 256), g.shape.S), dim3(256), 0, st, grp,
                     (double2*)flat, g.off, g.shape.n, to_flat ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
PassArgs<T> pass_args(const Group& g, const Grid* grid) {
  PassArgs<T> a{};
  a.g = g.shape;
  a.par = g.par;
  a.st = g.st;
  a.t = (cplx<T>*)g.T;
  a.grid = sizeof(T) == 8 ? (const T*)grid->g64 : (const T*)grid->g32;
  for (int k = 0; k < 4; ++k) a.fam[k] = grid->fam[sizeof(T) == 8 ? 1 : 0][k];
  a.partial = g.partc;
  a.u = (cplx<T>*)g.U;
  a.us = plane_split_size(g.shape);
  return a;
}

template <typename T>
KrylovArgs<T> krylov_args(const Group& g, int restart) {
  KrylovArgs<T> k{};
  k.g = g.shape;
  k.par = g.par;
  k.st = g.st;
  k.V = (cplx<T>*)g.V;
  k.restart = restart;
  k.part1 = g.part1;
  k.partn = g.partn;
  k.x64 = g.x64;
  k.r64 = g.r64;
  k.partc = g.partc;
  return k;
}

// ------------------------------------------------------------- profiler --
// Optional per-launch timing: a hipEvent pair around each launch on the
// launching stream, and the launch's algorithmic bytes (what the step must
// read and write by its definition, counted for the systems that do work in
// that launch).  Systems that finish a Krylov cycle early are only known at
// the next host synchronisation, so step launches are attributed then.

enum KClass { K_PASS_A, K_PASS_B, K_PASS_C, K_CGS_DOT, K_CGS_UPD, K_CGS_FIN, K_LSQ, K_CAST, K_FINAL,
              K_BICG_INIT, K_BICG_DOT, K_BICG_UPD, K_NBASE };
const char* kClassNames[K_NBASE] = {"pass_a",     "pass_b",     "pass_c",         "cgs_dot",
                                    "cgs_update", "cgs_finish", "lsq_update",     "cast_v0",
                                    "resid_finalize", "bicg_init", "bicg_dot", "bicg_update"};

struct ProfRec {
  int cls;        // base class * 2 + (complex128 ? 1 : 0)
  hipEvent_t a, b;
  double bytes;   // resolved algorithmic bytes
  int step;       // Arnoldi step (>= 0) to resolve later, -1 resolved, -2 lsq
  double unit;    // bytes per working system (step records)
  int group;
  double flops;   // resolved algorithmic floating-point operations
  double funit;   // operations per working system (step records)
  double pmin_ratio;  // bytes on the smallest admissible grid over bytes on the grid used
};

// Shared by every host thread that calls the library (calls on different
// plans may run concurrently): records are guarded by a mutex; the tag of the
// group whose work a thread is issuing is the thread's own.
struct Profiler {
  std::atomic<bool> on{false};
  int only = -1;  // record only this base class (-1: all)
  int every = 1;  // time one launch in `every` of each class
  std::atomic<unsigned> seq[K_NBASE] = {};  // launches of each class seen
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::atomic<int> tag_counter{0};  // source of group tags
  std::mutex mu;
} g_prof;
thread_local int t_group_tag = 0;  // tag of the group whose work this thread issues
thread_local bool t_capturing = false;  // this thread is capturing a launch graph: no timing events

// a pair of pooled events (callers hold g_prof.mu)
hipEvent_t prof_event() {
  if (g_prof.used == g_prof.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_prof.pool.push_back(e);
  }
  return g_prof.pool[g_prof.used++];
}

template <class F>
hipError_t timed(int cls, bool dbl, double bytes, int step, double unit, hipStream_t st, F&& f,
                 double flops = 0.0, double funit = 0.0) {
  if (t_capturing || !g_prof.on || (g_prof.only >= 0 && g_prof.only != cls)) return f();
  if (g_prof.every > 1 && g_prof.seq[cls].fetch_add(1) % g_prof.every != 0) return f();
  ProfRec r{cls * 2 + (dbl ? 1 : 0), nullptr, nullptr, bytes, step, unit, t_group_tag, flops, funit, 1.0};
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    r.a = prof_event();
    r.b = prof_event();
  }
  if (r.a) hipEventRecord(r.a, st);
  const hipError_t e = f();
  if (r.b) hipEventRecord(r.b, st);
  if (r.a && r.b) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.recs.push_back(r);
  }
  return e;
}

// The same for launchers that take the event pair themselves (the pass
// kernels: extended launches stamped by the dispatch packet).
template <class F>
hipError_t timed_ext(int cls, bool dbl, double bytes, int step, double unit, hipStream_t st, F&& f, double flops,
                     double funit, double pmin_ratio) {
  if (t_capturing || !g_prof.on || (g_prof.only >= 0 && g_prof.only != cls)) return f(nullptr, nullptr);
  if (g_prof.every > 1 && g_prof.seq[cls].fetch_add(1) % g_prof.every != 0) return f(nullptr, nullptr);
  ProfRec r{cls * 2 + (dbl ? 1 : 0), nullptr, nullptr, bytes, step, unit, t_group_tag, flops, funit, pmin_ratio};
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    r.a = prof_event();
    r.b = prof_event();
  }
  if (!r.a || !r.b) return f(nullptr, nullptr);
  const hipError_t e = f(r.a, r.b);
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.recs.push_back(r);
  return e;
}

// Resolve the step records of the cycle that just ended: jdone[s] Arnoldi
// steps were done by system s.
void prof_resolve(const int* jdone, int S, long long n, size_t vb) {
  if (!g_prof.on) return;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& r : g_prof.recs) {
    if (r.group != t_group_tag || r.step == -1) continue;
    double tot = 0;
    if (r.step == -2) {
      for (int s = 0; s < S; ++s)
        if (jdone[s] > 0) tot += (double)jdone[s] * n * vb + 2.0 * n * sizeof(double2);
    } else {
      int cnt = 0;
      for (int s = 0; s < S; ++s) cnt += jdone[s] > r.step;
      tot = cnt * r.unit;
      r.flops = cnt * r.funit;
    }
    r.bytes = tot;
    r.step = -1;
  }
}

// Algorithmic bytes of the three passes per system (C = 3 components):
//   pass A: read x (C N1^3 b_c), write the intermediate (C N1x N1y P b_c)
//   pass B: read + write the intermediate, read the contrast grid (P^3 b_r)
//   pass C: read the intermediate, read x, write y (2 C N1^3 b_c)
struct PassBytes {
  double a, b, c;
};
PassBytes pass_bytes(const GroupShape& g, size_t bc, int P = 0) {
  if (P <= 0) P = g.P;
  const double vec = (double)g.n * bc, mid = 3.0 * g.npencil * P * bc;  // padding not counted
  const double grid = (double)P * P * P * (bc / 2);
  return {vec + mid, 2 * mid + grid, mid + 2 * vec};
}

// The smallest grid the exact product admits, P >= 4 max_a M_a + 1, among
// sizes with no prime factor above 5: the grid of the bytes model, so that a
// larger grid in use does not inflate the algorithmic bytes.
int pmin_smooth(const int M[3]) {
  int p = 4 * std::max(M[0], std::max(M[1], M[2])) + 1;
  for (;; ++p) {
    int r = p;
    for (int f : {2, 3, 5})
      while (r % f == 0) r /= f;
    if (r == 1) return p;
  }
}

// Algorithmic floating-point operations of the three passes per system: the
// pruned length-P transforms (their real add, sub and mul counts), the real
// contrast multiply (2 per complex point) and, in pass C, the real symmetric
// 3x3 Green tensor times the complex field plus the subtraction (36 per
// harmonic).  Pass B expands x on N1y rows, then y on P columns, and crops
// in the reverse order.
PassBytes pass_flops(const GroupShape& g) {
  const int row = pruned_ops_row(g.P);
  // beyond the generated table (P >= 256): the 5 P log2 P real operations of
  // a full radix-2 transform, an upper estimate of the pruned one
  const double full = 5.0 * g.P * std::log2((double)g.P);
  auto fe = [&](int ax) { return row >= 0 ? (double)kPrunedOps[row][g.M[ax]][0] : full; };
  auto fc = [&](int ax) { return row >= 0 ? (double)kPrunedOps[row][g.M[ax]][1] : full; };
  const double P = g.P, nx = g.N1[0], ny = g.N1[1], nz = g.N1[2];
  const double plane = ny * (fe(0) + fc(0)) + P * (fe(1) + fc(1)) + 2.0 * P * P;
  return {3.0 * nx * ny * fe(2), 3.0 * P * plane, 3.0 * nx * ny * fc(2) + 36.0 * nx * ny * nz};
}

template <typename T>
int apply_passes(PassArgs<T> a, int pa_mode, hipStream_t st, int nwork, int step = -1) {
  a.xnorm = (pa_mode & PA_NORMALIZE) ? 1 : 0;
  PassArgs<T> aa = a;
  aa.mode = pa_mode;
  const bool dbl = sizeof(T) == 8;
  PassBytes pb = pass_bytes(a.g, sizeof(cplx<T>));
  const PassBytes pf = pass_flops(a.g);
  const double nf = step >= 0 ? 0.0 : (double)nwork;
  const double vec = (double)a.g.n * sizeof(cplx<T>);
  if (a.mode == PC_GREEN || a.mode == PC_CONV) pb.c -= vec;  // x is not read
  if (a.mode == PC_ADJ_RESID) pb.c += vec;                   // rhs is read
  // the contrast grid is shared by the systems of a launch: counted once
  const double grid = (double)a.g.P * a.g.P * a.g.P * sizeof(T);
  const double nb_b = step >= 0 ? 0.0 : nwork * (pb.b - grid) + grid;
  // the same bytes on the smallest admissible grid, as ratios per class
  const int pm = pmin_smooth(a.g.M);
  PassBytes pbm = pass_bytes(a.g, sizeof(cplx<T>), pm);
  if (a.mode == PC_GREEN || a.mode == PC_CONV) pbm.c -= vec;
  if (a.mode == PC_ADJ_RESID) pbm.c += vec;
  const double gridm = (double)pm * pm * pm * sizeof(T);
  const double nsys_b = step >= 0 ? (double)std::max(1, a.g.S) : (double)std::max(1, nwork);
  const double rb = (nsys_b * (pbm.b - gridm) + gridm) / (nsys_b * (pb.b - grid) + grid);
  auto with_ev = [](PassArgs<T> q, hipEvent_t e0, hipEvent_t e1) {
    q.ev0 = e0;
    q.ev1 = e1;
    return q;
  };
  HIP_TRY(timed_ext(K_PASS_A, dbl, step >= 0 ? 0.0 : nwork * pb.a, step, pb.a, st,
                    [&](hipEvent_t e0, hipEvent_t e1) { return launch_pass_a<T>(with_ev(aa, e0, e1), st); },
                    nf * pf.a, pf.a, pbm.a / pb.a));
  HIP_TRY(timed_ext(K_PASS_B, dbl, nb_b, step, pb.b - grid + grid / std::max(1, a.g.S), st,
                    [&](hipEvent_t e0, hipEvent_t e1) { return launch_pass_b<T>(with_ev(a, e0, e1), st); },
                    nf * pf.b, pf.b, rb));
  HIP_TRY(timed_ext(K_PASS_C, dbl, step >= 0 ? 0.0 : nwork * pb.c, step, pb.c, st,
                    [&](hipEvent_t e0, hipEvent_t e1) { return launch_pass_c<T>(with_ev(a, e0, e1), st); },
                    nf * pf.c, pf.c, pbm.c / pb.c));
  return GSM_OK;
}

// ----------------------------------------------------------- autotuner --
// At the first use of an (M, P, precision) by a plan made with
// GSM_PLAN_AUTOTUNE: time every codelet family of each FFT stage on the
// group's own batch (zeroed buffers: the kernels' speed does not depend on
// the data), the best of five launches each, and keep the fastest, leaving
// the default unless another family is at least 3 % faster (single launches
// of a few tens of microseconds vary by about that much); record the result
// in the plan's cache file if it has one.
template <typename T>
int tune_families(gsm_plan_s* plan, Group& g, Grid* grid, int restart, hipStream_t st) {
  const int d = sizeof(T) == 8 ? 1 : 0;
  if (!plan->autotune || grid->tuned[d]) return GSM_OK;
  const long long n = g.shape.n;
  const int S = g.shape.S;
  HIP_TRY(hipMemsetAsync(g.V, 0, (size_t)S * (restart + 1) * n * sizeof(cplx<T>), st));
  HIP_TRY(hipMemsetAsync(g.T, 0, (size_t)S * g.shape.tsize * sizeof(cplx<T>), st));
  PassArgs<T> a = pass_args<T>(g, grid);
  a.g.nblk_c = nblk_c_for(g.shape, d == 1);
  a.x = (cplx<T>*)g.V;
  a.xs = (long long)(restart + 1) * n;
  a.y = a.x + n;
  a.ys = a.xs;
  a.gate = GATE_NONE;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto best_of = [&](auto launch, float* ms) -> int {
    *ms = 1e30f;
    for (int r = 0; r < 5; ++r) {
      HIP_TRY(hipEventRecord(e0, st));
      HIP_TRY(launch());
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float t = 0;
      HIP_TRY(hipEventElapsedTime(&t, e0, e1));
      *ms = std::min(*ms, t);
    }
    return GSM_OK;
  };
  int fam[4];
  float tA[2], tB[4], tC[2];
  int rc = GSM_OK;
  for (int f = 0; f < 2 && !rc; ++f) {
    PassArgs<T> q = a;
    q.mode = 0;
    q.fam[0] = f;
    rc = best_of([&] { return launch_pass_a<T>(q, st); }, &tA[f]);
  }
  for (int f = 0; f < 4 && !rc; ++f) {
    PassArgs<T> q = a;
    q.fam[1] = f / 2;
    q.fam[2] = f % 2;
    rc = best_of([&] { return launch_pass_b<T>(q, st); }, &tB[f]);
  }
  for (int f = 0; f < 2 && !rc; ++f) {
    PassArgs<T> q = a;
    q.mode = PC_GREEN;
    q.fam[3] = f;
    rc = best_of([&] { return launch_pass_c<T>(q, st); }, &tC[f]);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  int def[4];
  default_families(g.shape.P, d == 1, def);
  auto pick = [](const float* t, int n, int dflt) {
    int best = dflt;
    for (int f = 0; f < n; ++f)
      if (t[f] < 0.97f * t[dflt] && t[f] < t[best]) best = f;
    return best;
  };
  fam[0] = pick(tA, 2, def[0]);
  const int fb = pick(tB, 4, def[1] * 2 + def[2]);
  fam[1] = fb / 2;
  fam[2] = fb % 2;
  fam[3] = pick(tC, 2, def[3]);
  for (int k = 0; k < 4; ++k) grid->fam[d][k] = fam[k];
  grid->tuned[d] = true;
  const int* M = g.shape.M;
  plan->tune_known[{M[0], M[1], M[2], g.shape.P, d}] = {fam[0], fam[1], fam[2], fam[3]};
  if (!plan->tune_cache.empty()) {
    if (FILE* f = std::fopen(plan->tune_cache.c_str(), "a")) {
      std::fprintf(f, "%s P=%d M=%d,%d,%d %s S=%d fam=%d,%d,%d,%d us=%.1f,%.1f,%.1f\n", plan->arch.c_str(),
                   g.shape.P, M[0], M[1], M[2], d ? "c128" : "c64", S, fam[0], fam[1], fam[2], fam[3],
                   1e3 * tA[fam[0]], 1e3 * tB[fb], 1e3 * tC[fam[3]]);
      std::fclose(f);
    }
  }
  return GSM_OK;
}

// Entries of a tuning cache file for this architecture.
void read_tune_cache(gsm_plan_s* plan) {
  FILE* f = std::fopen(plan->tune_cache.c_str(), "r");
  if (!f) return;
  char line[512], arch[128], prec[8];
  while (std::fgets(line, sizeof line, f)) {
    int P, M0, M1, M2, S, a, b, c, e;
    if (std::sscanf(line, "%127s P=%d M=%d,%d,%d %7s S=%d fam=%d,%d,%d,%d", arch, &P, &M0, &M1, &M2, prec, &S, &a,
                    &b, &c, &e) != 11)
      continue;
    if (plan->arch != arch) continue;
    const int d = std::strcmp(prec, "c128") == 0 ? 1 : 0;
    plan->tune_known[{M0, M1, M2, P, d}] = {a & 1, b & 1, c & 1, e & 1};
  }
  std::fclose(f);
}

#ifndef GSM_LEAD
#define GSM_LEAD 2
#endif
constexpr int kLead = GSM_LEAD;  // Arnoldi steps the host may run ahead of the device
#ifndef GSM_CHUNK
#define GSM_CHUNK 4
#endif
constexpr int kChunk = GSM_CHUNK;  // Arnoldi steps per launch graph
constexpr int kChunkLead = 2;      // graphs the host may run ahead of the device
constexpr int kMaxLagSlots = 4;    // GMRES slots a cycle may add for systems running behind

__global__ void k_export(const SysState* st, const double2* x64, GroupShape g, SysExport* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.S) return;
  SysExport e{};
  e.status = st[s].status;
  e.iters = st[s].iters;
  e.refinements = st[s].refinements;
  e.reorth = st[s].nreorth;
  e.rel = st[s].rel;
  const long long i0 = ((long long)g.M[2] * g.N1[1] + g.M[1]) * g.N1[0] + g.M[0];
  const long long cs = (long long)g.npencil * g.N1[2];
  for (int c = 0; c < 3; ++c) {
    e.e0[c] = x64[(long long)s * g.n + c * cs + i0];
    e.w0[c] = st[s].w0[c];
  }
  out[s] = e;
}

// The solve of one group as a state machine the scheduler advances without
// blocking: FP64 residual check -> Krylov cycle (Arnoldi steps or BiCGStab
// iterations issued at most kLead ahead of the device, or GMRES steps as
// launch graphs of kChunk steps at most kChunkLead graphs ahead; the host
// stops when the kernels' pinned per-system flags say every cycle has ended)
// -> residual check ... -> export of the results.  Everything runs on the
// slot's stream.  Steps issued after a system's cycle ended return at once
// for that system (the kernels test its flags), so a graph may run past the
// end of a cycle.
template <typename T>
struct GroupRun {
  enum Phase { START, RESID_WAIT, CYCLE, EXPORT_WAIT, DONE };
  gsm_plan_s* plan = nullptr;
  Group* g = nullptr;
  RunSlot* sl = nullptr;
  const gsm_solver_opts* so = nullptr;
  const std::vector<SysDesc>* sys = nullptr;
  const double* rhs = nullptr;  // adjoint right-hand sides (flat layout) or null
  double* E_out = nullptr;
  bool out_host = false;
  std::vector<SysExport>* exp = nullptr;
  int tag = 0;
  hipStream_t st = nullptr;

  KrylovArgs<double> k64{};
  KrylovArgs<T> kt{};
  PassArgs<double> r{};
  PassArgs<T> p{}, pbi{};
  int r_pa = 0, S = 0, m = 0, cap_outer = 0, it_cap = 0;
  long long n = 0;
  bool adjoint = false, bicg = false;
  static constexpr bool fp64 = sizeof(T) == 8;
  static constexpr size_t vb = sizeof(cplx<T>);
  double vecb = 0;
  cplx<T>* V = nullptr;
  std::vector<SysParam> par_host;
  std::vector<long long> off_host;

  Phase phase = START;
  int outer = 0, j = 0, n_outer = 0;
  bool graph = false;              // GMRES steps issued as cached launch graphs
  std::vector<unsigned char> fp;   // bytes of the step launches' fixed arguments

  void setup(const Grid* grid) {
    S = g->shape.S;
    n = g->shape.n;
    m = so->restart;
    adjoint = rhs != nullptr;
    bicg = so->method == GSM_BICGSTAB;
    vecb = (double)n * vb;
    st = sl->stream;
    k64 = krylov_args<double>(*g, m);
    kt = krylov_args<T>(*g, m);
    kt.host_inner = sl->h_inner;
    kt.reorth_all = (so->flags & GSM_SOLVE_REORTH) ? 1 : 0;
    r = pass_args<double>(*g, grid);
    r.g.nblk_c = nblk_c_for(g->shape, true);
    k64.g.nblk_c = r.g.nblk_c;
    r.x = g->x64;
    r.xs = n;
    r.y = g->r64;
    r.ys = n;
    // forward: A = I - B with B = G V; adjoint: A^H = I - B^H with B^H = V G
    // (G real symmetric, V Hermitian for real eps), i.e. the Green tensor is
    // applied by pass A before the convolution
    r.mode = adjoint ? PC_ADJ_RESID : PC_RESID;
    r.rhs = g->rhs64;
    r.rs = n;
    r.gate = GATE_OUTER;
    r_pa = adjoint ? PA_GREEN_PRE : 0;
    p = pass_args<T>(*g, grid);
    p.g.nblk_c = nblk_c_for(g->shape, fp64);
    p.xs = (long long)(m + 1) * n;
    p.ys = p.xs;
    p.mode = adjoint ? PC_CONV : PC_GREEN;  // the Arnoldi process runs on B (or B^H)
    p.gate = GATE_INNER;
    pbi = p;                                // BiCGStab applies A (or A^H) itself
    pbi.mode = adjoint ? PC_ADJ : PC_FWD;
    p.x = (cplx<T>*)g->V;                   // V_j -> V_j+1 at each system's step j
    p.y = (cplx<T>*)g->V + n;
    p.xstep = 1;
    V = (cplx<T>*)g->V;
    cap_outer = so->max_refine + 2;
    it_cap = std::max(1, so->max_iter / 2 + 1);
    for (int si : g->sys) {
      par_host.push_back((*sys)[si].par);
      off_host.push_back((*sys)[si].out_off);
    }
    // Launch graphs need every kernel argument of a step to follow from
    // these bytes and the step index; timed launches carry events and are
    // not captured.
    graph = !bicg && (so->flags & GSM_SOLVE_GRAPH) && !g_prof.on && !plan->graph_off;
    if (graph) {
      auto add = [&](const void* q, size_t b) {
        fp.insert(fp.end(), (const unsigned char*)q, (const unsigned char*)q + b);
      };
      const int ints[4] = {r_pa, m, (int)sizeof(T), adjoint ? 1 : 0};
      add(ints, sizeof ints);
      add(&kt, sizeof kt);
      add(&p, sizeof p);
      add(&st, sizeof st);
    }
  }

  int issue_residual() {
    if (outer == 0 && !so->x0) {
      // x = 0: the residual is the right-hand side, no operator application
      HIP_TRY(launch_zero_start(r.g, g->par, g->r64, adjoint ? g->rhs64 : nullptr, g->partc, st));
    } else {
      const int rc = apply_passes<double>(r, r_pa, st, n_outer);
      if (rc) return rc;
    }
    ++outer;
    HIP_TRY(timed(K_FINAL, true, 0.0, -1, 0.0, st, [&] { return launch_resid_finalize(k64, fp64 ? 1 : 0, g->flags, st); }));
    HIP_TRY(hipMemcpyAsync(sl->h_flags, g->flags, 2 * S * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(sl->phase_ev, st));
    phase = RESID_WAIT;
    return GSM_OK;
  }

  int issue_export() {
    if (out_host) {
      for (int k = 0; k < S; ++k) {
        const SysDesc& d = (*sys)[g->sys[k]];
        HIP_TRY(hipMemcpyAsync(E_out + 2 * d.out_off, g->x64 + (long long)k * n, d.n * sizeof(double2),
                               hipMemcpyDeviceToHost, st));
      }
    } else {
      HIP_TRY(move_fields(*g, g->x64, E_out, true, st));
    }
    hipLaunchKernelGGL(k_export, dim3((S + 63) / 64), dim3(64), 0, st, g->st, g->x64, g->shape, (SysExport*)g->exp);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(sl->h_exp, g->exp, S * sizeof(SysExport), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(sl->phase_ev, st));
    phase = EXPORT_WAIT;
    return GSM_OK;
  }

  // The launches of one Arnoldi (or BiCGStab) step; the step counter
  // advances, no event is recorded.
  int step_kernels() {
    if (bicg) {
      const int it = j;
      pbi.x = V + BI_P * n;
      pbi.y = V + BI_V * n;
      int rc = apply_passes<T>(pbi, r_pa, st, 0, it);
      if (rc) return rc;
      HIP_TRY(timed(K_BICG_DOT, fp64, 0.0, it, 2 * vecb, st, [&] { return launch_bicg<T>(kt, BICG_DOT_RV, it, it_cap, st); }));
      HIP_TRY(timed(K_BICG_UPD, fp64, 0.0, it, 3 * vecb, st, [&] { return launch_bicg<T>(kt, BICG_S, it, it_cap, st); }));
      pbi.x = V + BI_S * n;
      pbi.y = V + BI_T * n;
      rc = apply_passes<T>(pbi, r_pa, st, 0, it);
      if (rc) return rc;
      HIP_TRY(timed(K_BICG_DOT, fp64, 0.0, it, 2 * vecb, st, [&] { return launch_bicg<T>(kt, BICG_DOT_TS, it, it_cap, st); }));
      HIP_TRY(timed(K_BICG_UPD, fp64, 0.0, it, 5 * vecb + 2.0 * n * sizeof(double2), st,
                    [&] { return launch_bicg<T>(kt, BICG_XR, it, it_cap, st); }));
      HIP_TRY(timed(K_BICG_UPD, fp64, 0.0, it, 4 * vecb, st, [&] { return launch_bicg<T>(kt, BICG_P, it, it_cap, st); }));
    } else {
      // the passes read V_j and write V_j+1 at each system's own step index
      // (one behind the group's after a second Gram-Schmidt pass, which
      // takes a step's slot; the passes skip a system in that slot)
      const int rc = apply_passes<T>(p, r_pa, st, 0, j);
      if (rc) return rc;
      HIP_TRY(timed(K_CGS_DOT, fp64, 0.0, j, (j + 2) * vecb, st, [&] { return launch_cgs_dot<T>(kt, st); }));
      HIP_TRY(timed(K_CGS_UPD, fp64, 0.0, j, (j + 3) * vecb, st, [&] { return launch_cgs_update<T>(kt, st); }));
      // finish: Givens step, unless the first pass removed nearly all of w:
      // then the system's next slot makes the second pass
      HIP_TRY(timed(K_CGS_FIN, fp64, 0.0, j, 0.0, st, [&] { return launch_cgs_finish<T>(kt, st); }));
    }
    ++j;
    return GSM_OK;
  }

  int issue_step() {
    const int rc = step_kernels();
    if (rc) return rc;
    HIP_TRY(hipEventRecord(sl->step_ev[(j - 1) % kRing], st));
    return GSM_OK;
  }

  // Steps j .. j + cnt - 1 as one launch graph: the slot's cached graph of
  // exactly these launches if there is one, else captured from the stream
  // now.  Records the chunk's event (chunk index j / kChunk).
  int issue_chunk(int cnt) {
    const int c = j / kChunk;
    std::vector<unsigned char> key = fp;
    const int tail[2] = {j, cnt};
    key.insert(key.end(), (const unsigned char*)tail, (const unsigned char*)tail + sizeof tail);
    RunSlot::GraphEntry* hit = nullptr;
    for (auto& e : sl->graphs)
      if (e.key == key) hit = &e;
    if (hit) {
      j += cnt;
    } else {
      const int j0 = j;
      HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      t_capturing = true;
      int rc = GSM_OK;
      for (int q = 0; q < cnt && !rc; ++q) rc = step_kernels();
      t_capturing = false;
      hipGraph_t gr = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &gr);
      hipGraphExec_t ex = nullptr;
      const hipError_t ei = (rc || ec != hipSuccess) ? hipErrorUnknown : hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      if (gr) (void)hipGraphDestroy(gr);
      if (rc || ec != hipSuccess || ei != hipSuccess) {
        // not capturable here: separate launches for the rest of the plan's life
        (void)hipGetLastError();
        plan->graph_off = true;
        graph = false;
        j = j0;
        for (int q = 0; q < cnt; ++q)
          if ((rc = step_kernels())) return rc;
        HIP_TRY(hipEventRecord(sl->step_ev[c % kRing], st));
        return GSM_OK;
      }
      if (sl->graphs.size() >= kGraphsPerSlot) {
        auto old = std::min_element(sl->graphs.begin(), sl->graphs.end(),
                                    [](const RunSlot::GraphEntry& a, const RunSlot::GraphEntry& b) { return a.used < b.used; });
        (void)hipGraphExecDestroy(old->exec);
        sl->graphs.erase(old);
      }
      sl->graphs.push_back(RunSlot::GraphEntry{std::move(key), ex, 0});
      hit = &sl->graphs.back();
      ++plan->graph_captures;
    }
    hit->used = ++plan->graph_clock;
    HIP_TRY(hipGraphLaunch(hit->exec, st));
    ++plan->graph_launches;
    HIP_TRY(hipEventRecord(sl->step_ev[c % kRing], st));
    return GSM_OK;
  }

  int end_cycle() {
    if (bicg)
      HIP_TRY(launch_bicg<T>(kt, BICG_END, 0, it_cap, st));
    else
      HIP_TRY(timed(K_LSQ, fp64, 0.0, -2, 0.0, st, [&] { return launch_lsq_update<T>(kt, st); }));
    return issue_residual();
  }

  // Issue everything that needs no wait; *moved says whether anything was.
  int advance(bool* moved) {
    *moved = false;
    t_group_tag = tag;
    int rc = GSM_OK;
    switch (phase) {
      case START:
        HIP_TRY(hipMemcpyAsync(g->par, par_host.data(), S * sizeof(SysParam), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(g->off, off_host.data(), S * sizeof(long long), hipMemcpyHostToDevice, st));
        if (adjoint) {
          HIP_TRY(move_fields(*g, g->rhs64, rhs, false, st));
          HIP_TRY(launch_rhs_norm(g->shape, g->rhs64, g->par, st));
        }
        HIP_TRY(launch_state_init(g->shape, g->st, g->x64, nullptr, st));
        if (so->x0) HIP_TRY(move_fields(*g, g->x64, so->x0, false, st));
        n_outer = S;
        *moved = true;
        return issue_residual();
      case RESID_WAIT: {
        const hipError_t q = hipEventQuery(sl->phase_ev);
        if (q == hipErrorNotReady) return GSM_OK;
        HIP_TRY(q);
        *moved = true;
        prof_resolve(sl->h_flags + S, S, n, vb);
        n_outer = 0;
        for (int s = 0; s < S; ++s) n_outer += sl->h_flags[s] != 0;
        if (!n_outer || outer >= cap_outer) return issue_export();
        j = 0;
        phase = CYCLE;
        if (bicg) {
          HIP_TRY(timed(K_BICG_INIT, fp64, n_outer * (n * sizeof(double2) + 3 * vecb), -1, 0.0, st,
                        [&] { return launch_bicg<T>(kt, BICG_INIT, 0, it_cap, st); }));
        } else {
          HIP_TRY(timed(K_CAST, fp64, n_outer * (n * sizeof(double2) + vecb), -1, 0.0, st,
                        [&] { return launch_cast_v0<T>(kt, st); }));
        }
        return GSM_OK;
      }
      case CYCLE:
        for (;;) {
          const int limit = bicg ? it_cap : m;
          if (j >= limit) {
            // GMRES: slots past m for the systems seen to run behind after
            // second Gram-Schmidt passes (pinned flag 1 + lag while running),
            // so that they too complete m steps (with separate launches; a
            // cycle issued as launch graphs ends at m)
            if (!bicg && !graph && j < m + kMaxLagSlots) {
              int lag = 0;
              for (int s = 0; s < S; ++s) lag = std::max(lag, sl->h_inner[s] - 1);
              if (j < m + lag) {
                if ((rc = issue_step())) return rc;
                *moved = true;
                continue;
              }
            }
            *moved = true;
            return end_cycle();
          }
          if (graph) {
            // chunks of kChunk steps; the host runs kChunkLead chunks ahead
            const int c = j / kChunk;
            if (c >= kChunkLead) {
              const hipError_t q = hipEventQuery(sl->step_ev[(c - kChunkLead) % kRing]);
              if (q == hipErrorNotReady) return GSM_OK;
              HIP_TRY(q);
              bool running = false;
              for (int s = 0; s < S && !running; ++s) running = sl->h_inner[s] != 0;
              if (!running) {
                *moved = true;
                return end_cycle();
              }
            }
            if ((rc = issue_chunk(std::min(kChunk, limit - j)))) return rc;
            *moved = true;
            continue;
          }
          if (j >= kLead) {
            const hipError_t q = hipEventQuery(sl->step_ev[(j - kLead) % kRing]);
            if (q == hipErrorNotReady) return GSM_OK;
            HIP_TRY(q);
            bool running = false;
            for (int s = 0; s < S && !running; ++s) running = sl->h_inner[s] != 0;
            if (!running) {
              *moved = true;
              return end_cycle();
            }
          }
          if ((rc = issue_step())) return rc;
          *moved = true;
        }
      case EXPORT_WAIT: {
        const hipError_t q = hipEventQuery(sl->phase_ev);
        if (q == hipErrorNotReady) return GSM_OK;
        HIP_TRY(q);
        const SysExport* e = (const SysExport*)sl->h_exp;
        for (int k = 0; k < S; ++k) (*exp)[g->sys[k]] = e[k];
        phase = DONE;
        *moved = true;
        return GSM_OK;
      }
      case DONE:
        return GSM_OK;
    }
    return GSM_OK;
  }

  // the event a blocked run waits on
  hipEvent_t blocker() const {
    if (phase == CYCLE && graph) return sl->step_ev[(j / kChunk - kChunkLead + kRing) % kRing];
    if (phase == CYCLE) return sl->step_ev[(j - kLead + kRing) % kRing];
    return sl->phase_ev;
  }
};

// Run every group of a call: the largest groups first, up to kSlots at once,
// each on a stream of its own, their steps interleaved by the host (a work
// queue: a slot takes the next group as soon as its group is done).  The
// slots' streams start after the work queued on the caller's stream and the
// caller's stream waits for them at the end.
template <typename T>
int run_groups(gsm_plan_s* plan, std::vector<SysDesc>& sys, std::vector<Group>& groups,
               std::vector<const Grid*>& grids, const gsm_solver_opts* so, double* E_out, bool out_host,
               std::vector<SysExport>& exp, hipStream_t st, const double* rhs) {
  std::vector<int> order(groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (double)groups[a].shape.S * groups[a].shape.tsize > (double)groups[b].shape.S * groups[b].shape.tsize;
  });
  int max_s = 0;
  for (auto& g : groups) max_s = std::max(max_s, g.shape.S);
  const int nslot = std::min<int>(kSlots, (int)groups.size());
  hipEvent_t start = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  int rc = GSM_OK;
  auto finish = [&](int code) {
    for (int k = 0; k < nslot; ++k) {
      RunSlot& sl = plan->slots[k];
      if (!sl.stream) continue;
      if (code) hipStreamSynchronize(sl.stream);
      if (hipEventRecord(sl.phase_ev, sl.stream) == hipSuccess) (void)hipStreamWaitEvent(st, sl.phase_ev, 0);
    }
    (void)hipEventDestroy(start);
    return code;
  };
  HIP_TRY(hipEventRecord(start, st));
  for (int k = 0; k < nslot; ++k) {
    if ((rc = ensure_slot(plan, k, max_s, sizeof(SysExport)))) return finish(rc);
    if (hipStreamWaitEvent(plan->slots[k].stream, start, 0) != hipSuccess)
      return finish(fail(GSM_E_DEVICE, "stream wait failed"));
  }
  std::vector<GroupRun<T>> runs(groups.size());
  std::vector<int> active(nslot, -1);
  size_t next = 0;
  int done = 0;
  while (done < (int)groups.size()) {
    for (int k = 0; k < nslot; ++k) {
      if (active[k] >= 0 || next >= order.size()) continue;
      const int gi = order[next++];
      GroupRun<T>& R = runs[gi];
      R.plan = plan;
      R.g = &groups[gi];
      R.sl = &plan->slots[k];
      R.so = so;
      R.sys = &sys;
      R.rhs = rhs;
      R.E_out = E_out;
      R.out_host = out_host;
      R.exp = &exp;
      R.tag = ++g_prof.tag_counter;
      R.setup(grids[gi]);
      active[k] = gi;
    }
    bool any = false;
    for (int k = 0; k < nslot; ++k) {
      if (active[k] < 0) continue;
      GroupRun<T>& R = runs[active[k]];
      bool moved = false;
      if ((rc = R.advance(&moved))) return finish(rc);
      any = any || moved;
      if (R.phase == GroupRun<T>::DONE) {
        active[k] = -1;
        ++done;
        any = true;
      }
    }
    if (!any) {
      // nothing can be issued: sleep on what the first active group waits for
      for (int k = 0; k < nslot; ++k)
        if (active[k] >= 0) {
          const hipError_t e = hipEventSynchronize(runs[active[k]].blocker());
          if (e != hipSuccess) return finish(fail(GSM_E_DEVICE, "%s", hipGetErrorString(e)));
          break;
        }
    }
  }
  return finish(GSM_OK);
}

int solve_all(gsm_plan_s* plan, std::vector<SysDesc>& sys, std::vector<Group>& groups, const gsm_solver_opts* so,
              void* ws, size_t ws_bytes, double* E_out, bool out_host, std::vector<SysExport>& exp,
              hipStream_t st, const double* rhs = nullptr) {
  const bool fp64 = so->precision == GSM_FP64;
  int rc = carve(groups, ws, ws_bytes, so->restart, fp64);
  if (rc) return rc;
  exp.assign(sys.size(), SysExport{});
  std::vector<const Grid*> grids(groups.size());
  for (size_t i = 0; i < groups.size(); ++i) {
    Grid* grid = nullptr;
    if ((rc = ensure_grid(plan, groups[i].shape.M, groups[i].shape.P, st, &grid, groups[i].shape.form))) return rc;
    rc = fp64 ? tune_families<double>(plan, groups[i], grid, so->restart, st)
              : tune_families<float>(plan, groups[i], grid, so->restart, st);
    if (rc) return rc;
    grids[i] = grid;
  }
  rc = fp64 ? run_groups<double>(plan, sys, groups, grids, so, E_out, out_host, exp, st, rhs)
            : run_groups<float>(plan, sys, groups, grids, so, E_out, out_host, exp, st, rhs);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(st));
  return GSM_OK;
}

void fill_info(const std::vector<SysDesc>& sys, const std::vector<SysExport>& exp, gsm_solve_info* info,
               int* worst) {
  for (size_t i = 0; i < sys.size(); ++i) {
    gsm_solve_info& f = info[i];
    f.status = exp[i].status == 0 ? GSM_OK : GSM_W_NOT_CONVERGED;
    f.iterations = exp[i].iters;
    f.refinements = exp[i].refinements;
    f.fft_size = sys[i].P;
    f.reorth = exp[i].reorth;
    f.reserved = 0;
    f.rel_residual = exp[i].rel;
    f.eps_b = sys[i].par.eps_b;
    if (f.status == GSM_W_NOT_CONVERGED) *worst = GSM_W_NOT_CONVERGED;
  }
}

int set_device(const gsm_plan_s* plan) {
  HIP_TRY(hipSetDevice(plan->device));
  return GSM_OK;
}

// ------------------------------------------------------------ pole search --

int check_pole_query(const gsm_pole_query& q, const int* mmax, int i) {
  if (!std::isfinite(q.wavelength) || !(q.wavelength > 0)) return fail(GSM_E_ARG, "query %d: wavelength", i);
  double kk = 0;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(q.k_hat[a])) return fail(GSM_E_NONFINITE, "query %d: k_hat not finite", i);
    kk += q.k_hat[a] * q.k_hat[a];
    if (q.M[a] < 0 || q.M[a] > mmax[a]) return fail(GSM_E_ARG, "query %d: M[%d]=%d outside the plan", i, a, q.M[a]);
  }
  if (!(kk > 0)) return fail(GSM_E_ARG, "query %d: k_hat is zero", i);
  if (q.n_poles < 1 || q.n_poles > GSM_POLE_MAX_NP)
    return fail(GSM_E_ARG, "query %d: n_poles=%d outside [1, %d]", i, q.n_poles, GSM_POLE_MAX_NP);
  if (q.n_div <= q.n_poles || q.n_div > GSM_POLE_MAX_ND)
    return fail(GSM_E_ARG, "query %d: n_div=%d must exceed n_poles and be <= %d", i, q.n_div, GSM_POLE_MAX_ND);
  if (q.component < 0 || q.component > 2) return fail(GSM_E_ARG, "query %d: component %d", i, q.component);
  double nn = 0;
  for (int c = 0; c < 6; ++c) {
    if (!std::isfinite(q.pol[c])) return fail(GSM_E_NONFINITE, "query %d: pol not finite", i);
    nn += q.pol[c] * q.pol[c];
  }
  if (nn == 0) return fail(GSM_E_ARG, "query %d: drive is zero", i);
  if (!(std::isfinite(q.kappa_min) && std::isfinite(q.kappa_max) && q.kappa_min > 0 && q.kappa_max > q.kappa_min))
    return fail(GSM_E_ARG, "query %d: need 0 < kappa_min < kappa_max", i);
  if (!std::isfinite(q.eps_b)) return fail(GSM_E_NONFINITE, "query %d: eps_b not finite", i);
  return GSM_OK;
}

// The N_d + N_p instances of a query's mesh (eps_b left to the caller).
void pole_mesh(const gsm_pole_query& q, std::vector<gsm_instance>& out, std::vector<double>& kappa) {
  const int npts = q.n_div + q.n_poles;
  const double nk = std::sqrt(q.k_hat[0] * q.k_hat[0] + q.k_hat[1] * q.k_hat[1] + q.k_hat[2] * q.k_hat[2]);
  for (int i = 0; i < npts; ++i) {
    const double kap = q.kappa_min + (q.kappa_max - q.kappa_min) * i / (npts - 1);
    gsm_instance in{};
    in.wavelength = q.wavelength;
    for (int a = 0; a < 3; ++a) {
      in.k_inc[a] = kap * q.k_hat[a] / nk;
      in.M[a] = q.M[a];
    }
    in.n_drive = 1;
    for (int c = 0; c < 6; ++c) in.pol[0][c] = q.pol[c];
    in.eps_b = 0;
    out.push_back(in);
    kappa.push_back(kap);
  }
}

// One basis permittivity for a whole mesh (xi must be a single function of
// kappa): see gsm_pole_query.
int resolve_eps_b_mesh(const gsm_plan_s* plan, const gsm_instance* mesh, int n, double req, int qi, double* out) {
  if (req > 0) {
    for (int i = 0; i < n; ++i)
      if (margin_scan(mesh[i], plan->period, req) < kSingularRel * req)
        return fail(GSM_E_SINGULAR, "query %d: |k_m|^2 = k_b^2 within 1e-3 at mesh point %d for eps_b=%g", qi, i, req);
    *out = req;
    return GSM_OK;
  }
  bool ok = true;
  for (int i = 0; i < n && ok; ++i) ok = margin_scan(mesh[i], plan->period, plan->eps_mean) >= kSingularRel * plan->eps_mean;
  if (ok) {
    *out = plan->eps_mean;
    return GSM_OK;
  }
  std::vector<std::vector<double>> sh(n);
  for (int i = 0; i < n; ++i) sh[i] = shell_values(mesh[i], plan->period);
  const double lo = 0.5 * plan->eps_min, hi = 2.0 * plan->eps_max;
  double best = -1, best_eb = plan->eps_mean;
  const int ns = 4001;
  for (int k = 0; k < ns; ++k) {
    const double eb = lo + (hi - lo) * k / (ns - 1);
    double r = INFINITY;
    for (int i = 0; i < n; ++i) r = std::min(r, margin_of(sh[i], eb) / eb);
    if (r > best) {
      best = r;
      best_eb = eb;
    }
  }
  if (best < kSingularRel) return fail(GSM_E_SINGULAR, "query %d: no admissible eps_b for the whole mesh", qi);
  *out = best_eb;
  return GSM_OK;
}

// Buffers of a pole search after the groups' solve buffers: the mesh fields
// and the fit's inputs and outputs (base == nullptr: size only).
struct PoleBufs {
  double2* E = nullptr;
  long long* idx = nullptr;
  double* kappa = nullptr;
  double* xi = nullptr;
  double* eta = nullptr;
  double* zeta = nullptr;
  int* status = nullptr;
};
size_t pole_layout(const std::vector<SysDesc>& sys, long long n_eta, int n_q, char* base, PoleBufs* out) {
  long long total = 0;
  for (auto& s : sys) total += s.n;
  const long long ns = (long long)sys.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += align256(std::max<size_t>(bytes, 1));
    return (void*)q;
  };
  PoleBufs b;
  b.E = (double2*)take(total * sizeof(double2));
  b.idx = (long long*)take(ns * sizeof(long long));
  b.kappa = (double*)take(ns * sizeof(double));
  b.xi = (double*)take(2 * ns * sizeof(double));
  b.eta = (double*)take(2 * n_eta * sizeof(double));
  b.zeta = (double*)take(2 * n_eta * sizeof(double));
  b.status = (int*)take(std::max(n_q, 1) * sizeof(int));
  if (out) *out = b;
  return off;
}

// Mesh instances of every query (basis permittivity resolved per query),
// the systems and groups of one batched solve.
int pole_systems(gsm_plan_s* p, int n_q, const gsm_pole_query* q, const gsm_solver_opts* so,
                 std::vector<gsm_instance>& mesh, std::vector<double>& kappa, std::vector<double>& eb_q,
                 std::vector<SysDesc>& sys, std::vector<Group>& groups) {
  int rc;
  for (int i = 0; i < n_q; ++i)
    if ((rc = check_pole_query(q[i], p->mmax, i))) return rc;
  eb_q.assign(n_q, 0.0);
  for (int i = 0; i < n_q; ++i) {
    const size_t first = mesh.size();
    pole_mesh(q[i], mesh, kappa);
    if ((rc = resolve_eps_b_mesh(p, mesh.data() + first, (int)(mesh.size() - first), q[i].eps_b, i, &eb_q[i])))
      return rc;
    for (size_t k = first; k < mesh.size(); ++k) mesh[k].eps_b = eb_q[i];
  }
  if ((rc = build_systems(p, (int)mesh.size(), mesh.data(), so, false, sys))) return rc;
  build_groups(sys, groups, so->group_max);
  return GSM_OK;
}

// Common start of every plan (voxel, shape or coefficient body): device,
// options, tuning cache, periods and order ranges.  The caller fills the
// coefficients and the permittivity statistics.
int plan_begin(const gsm_plan_opts* opts, const double period[3], gsm_plan_s** out) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(GSM_E_DEVICE, "no HIP device");
  if (opts->device < 0 || opts->device >= ndev) return fail(GSM_E_ARG, "device %d not present", opts->device);
  auto* p = new gsm_plan_s();
  p->device = opts->device;
  p->autotune = (opts->flags & GSM_PLAN_AUTOTUNE) != 0;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, opts->device) == hipSuccess) {
      p->arch = prop.gcnArchName;
      const size_t colon = p->arch.find(':');
      if (colon != std::string::npos) p->arch.resize(colon);
    }
    if (p->arch.empty()) p->arch = "unknown";
  }
  if (opts->tune_cache) {
    p->tune_cache = opts->tune_cache;
    read_tune_cache(p);
  }
  for (int a = 0; a < 3; ++a) {
    p->period[a] = period[a];
    p->mmax[a] = opts->m_max[a];
    p->nc[a] = 4 * opts->m_max[a] + 1;
  }
  int rc;
  if ((rc = set_device(p))) {
    delete p;
    return rc;
  }
  *out = p;
  return GSM_OK;
}

// One operator application for the systems of one group: gather their
// vectors from the caller's flat layout into the group's staging vector,
// passes A, B and C, scatter the results back.  Synchronises the stream.
int apply_group(Group& g, const std::vector<SysDesc>& sys, const Grid* grid, bool dbl, int mode, const void* x,
                void* y, hipStream_t st) {
  int rc;
  const size_t eb = dbl ? sizeof(double2) : sizeof(float2);
  std::vector<SysParam> par;
  for (int si : g.sys) par.push_back(sys[si].par);
  HIP_TRY(hipMemcpyAsync(g.par, par.data(), par.size() * sizeof(SysParam), hipMemcpyHostToDevice, st));
  for (int k = 0; k < g.shape.S; ++k) {
    const SysDesc& s = sys[g.sys[k]];
    HIP_TRY(hipMemcpyAsync((char*)g.x64 + k * g.shape.n * eb, (const char*)x + s.out_off * eb, s.n * eb,
                           hipMemcpyDeviceToDevice, st));
  }
  const int pa_mode = mode == GSM_APPLY_ADJOINT ? PA_GREEN_PRE : 0;
  const int pc_mode = mode == GSM_APPLY_ADJOINT ? PC_ADJ : PC_FWD;
  if (dbl) {
    PassArgs<double> a = pass_args<double>(g, grid);
    a.g.nblk_c = nblk_c_for(g.shape, true);
    a.x = g.x64;
    a.y = g.r64;
    a.xs = a.ys = g.shape.n;
    a.mode = pc_mode;
    a.gate = GATE_NONE;
    if ((rc = apply_passes<double>(a, pa_mode, st, g.shape.S))) return rc;
  } else {
    PassArgs<float> a = pass_args<float>(g, grid);
    a.g.nblk_c = nblk_c_for(g.shape, false);
    a.x = (float2*)g.x64;
    a.y = (float2*)g.r64;
    a.xs = a.ys = g.shape.n;
    a.mode = pc_mode;
    a.gate = GATE_NONE;
    if ((rc = apply_passes<float>(a, pa_mode, st, g.shape.S))) return rc;
  }
  for (int k = 0; k < g.shape.S; ++k) {
    const SysDesc& s = sys[g.sys[k]];
    HIP_TRY(hipMemcpyAsync((char*)y + s.out_off * eb, (const char*)g.r64 + k * g.shape.n * eb, s.n * eb,
                           hipMemcpyDeviceToDevice, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  return GSM_OK;
}

// ---------------------------------------------- allocation-free apply ----
// gsm_apply_static takes its buffers from this array instead of a caller
// workspace.  On the host the array's name only stands in for the device
// symbol: no kernel argument, copy or fill ever names it.  Each device's
// address of its copy is looked up once, with that device current, and kept
// in g_scratch_ptr.  Only the forward and adjoint applications use it, and
// they read nothing of it before writing it, so it is never cleared.
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kScratchDevices] = {};

int static_scratch(int device, char** out) {
  if (device < 0 || device >= kScratchDevices)
    return fail(GSM_E_UNSUPPORTED, "gsm_apply_static: device ordinal %d beyond %d", device, kScratchDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;  // the caller has made `device` current
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(GSM_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = (char*)ptr;
  }
  *out = g_scratch_ptr[device];
  return GSM_OK;
}

// Buffers of one group's operator application carved from base (nullptr:
// size only): parameters, the staged input and output vectors, the pass
// intermediate.
size_t layout_apply(Group& g, char* base, size_t eb) {
  const long long S = g.shape.S, n = g.shape.n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += align256(bytes);
    return (void*)q;
  };
  g.par = (SysParam*)take(S * sizeof(SysParam));
  g.x64 = (double2*)take(S * n * eb);
  g.r64 = (double2*)take(S * n * eb);
  g.T = (double2*)take(S * g.shape.tsize * eb);
  g.U = (double2*)take(S * plane_split_size(g.shape) * eb);
  g.st = nullptr;  // not read without gating or basis scaling
  g.partc = nullptr;  // written only in the residual modes
  return off;
}

}  // namespace

// ===================================================================== ABI ==

extern "C" {

int gsm_version(void) { return GSM_VERSION; }

const char* gsm_strerror(int s) {
  switch (s) {
    case GSM_OK: return "ok";
    case GSM_W_NOT_CONVERGED: return "not converged within the iteration caps";
    case GSM_E_ARG: return "invalid argument";
    case GSM_E_NONFINITE: return "non-finite input";
    case GSM_E_NOMEM: return "out of device memory";
    case GSM_E_DEVICE: return "HIP runtime error";
    case GSM_E_SINGULAR: return "singular Green factor or effective-tensor system";
    case GSM_E_WORKSPACE: return "workspace missing or too small";
    case GSM_E_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

const char* gsm_last_error(void) { return g_err.c_str(); }

void gsm_solver_opts_default(gsm_solver_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-9;
  o->inner_tol = 1e-5;
  o->restart = 30;
  o->max_iter = 5000;
  o->max_refine = 200;
  o->precision = GSM_MIXED;
  o->method = GSM_GMRES;
  o->flags = 0;
  o->x0 = nullptr;
  o->group_max = 32;
  o->formulation = GSM_FORM_E;
}

int gsm_fft_size(const int32_t M[3]) {
  if (!M) return fail(GSM_E_ARG, "M is NULL");
  for (int a = 0; a < 3; ++a)
    if (M[a] < 0 || M[a] > kMaxOrder) return fail(GSM_E_UNSUPPORTED, "M[%d]=%d outside [0, %d]", a, M[a], kMaxOrder);
  return fft_size_for(M);
}

int gsm_plan_validate(const gsm_geometry* geo, const gsm_plan_opts* opts, int32_t n_inst,
                      const gsm_instance* inst) {
  int rc;
  if (geo && (rc = check_geometry(geo))) return rc;
  if (opts && (rc = check_plan_opts(opts))) return rc;
  if (n_inst < 0) return fail(GSM_E_ARG, "n_inst < 0");
  if (n_inst > 0) {
    if (!inst) return fail(GSM_E_ARG, "instances are NULL");
    double mean = 1, mn = 1, mx = 1;
    if (geo) {
      const long long nv = (long long)geo->nvox[0] * geo->nvox[1] * geo->nvox[2];
      double s = 0;
      mn = INFINITY;
      mx = 0;
      for (long long i = 0; i < nv; ++i) {
        s += geo->eps[i];
        mn = std::min(mn, geo->eps[i]);
        mx = std::max(mx, geo->eps[i]);
      }
      mean = s / nv;
    }
    const double per[3] = {geo ? geo->period[0] : 1.0, geo ? geo->period[1] : 1.0, geo ? geo->period[2] : 1.0};
    for (int i = 0; i < n_inst; ++i) {
      if ((rc = check_instance(inst[i], opts ? opts->m_max : nullptr, i, true))) return rc;
      if (inst[i].eps_b > 0 || geo) {
        double eb;
        if ((rc = resolve_eps_b(per, mean, mn, mx, inst[i], i, &eb))) return rc;
      }
    }
  }
  return GSM_OK;
}

int gsm_plan(const gsm_geometry* geo, const gsm_plan_opts* opts, gsm_plan_t* out) {
  int rc;
  if (!out) return fail(GSM_E_ARG, "out is NULL");
  if ((rc = check_geometry(geo)) || (rc = check_plan_opts(opts))) return rc;
  gsm_plan_s* p = nullptr;
  if ((rc = plan_begin(opts, geo->period, &p))) return rc;
  for (int a = 0; a < 3; ++a) p->vox[a] = geo->nvox[a];
  p->voxel_body = true;
  const long long nv = (long long)p->vox[0] * p->vox[1] * p->vox[2];
  double s = 0, mn = INFINITY, mx = 0;
  for (long long i = 0; i < nv; ++i) {
    s += geo->eps[i];
    mn = std::min(mn, geo->eps[i]);
    mx = std::max(mx, geo->eps[i]);
  }
  p->eps_mean = s / nv;
  p->eps_min = mn;
  p->eps_max = mx;
  auto cleanup = [&](int code) {
    gsm_plan_destroy(p);
    return code;
  };
  double* d_eps = nullptr;
  double2 *a = nullptr, *b = nullptr;
  const long long ncx = p->nc[0], ncy = p->nc[1], ncz = p->nc[2];
  const long long na = std::max(nv, (long long)p->vox[2] * ncy * ncx);
  const long long nb = (long long)p->vox[2] * p->vox[1] * ncx;
  hipError_t e = dev_malloc(&d_eps, nv * sizeof(double));
  if (e == hipSuccess) e = dev_malloc(&a, na * sizeof(double2));
  if (e == hipSuccess) e = dev_malloc(&b, nb * sizeof(double2));
  if (e == hipSuccess) e = dev_malloc(&p->d_coef, ncx * ncy * ncz * sizeof(double2));
  if (e == hipSuccess) e = dev_malloc(&p->d_coef_inv, ncx * ncy * ncz * sizeof(double2));
  if (e != hipSuccess) {
    hipFree(d_eps);
    hipFree(a);
    hipFree(b);
    return cleanup(fail(GSM_E_NOMEM, "plan allocation: %s", hipGetErrorString(e)));
  }
  hipStream_t st = nullptr;
  // the exact image of a piecewise-constant voxel body: of eps (Eq.(4)) and
  // of 1/eps (Eq.(5))
  std::vector<double> inv(nv);
  for (long long i = 0; i < nv; ++i) inv[i] = 1.0 / geo->eps[i];
  auto image = [&](const double* host, double2* coef) -> int {
    HIP_TRY(hipMemcpy(d_eps, host, nv * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(launch_real_to_complex(d_eps, a, nv, st));
    // voxel DFT along x: a[vz][vy][vx] -> b[vz][vy][ncx], n = j - 2 m_max
    HIP_TRY(launch_dft_axis(a, b, p->vox[2] * p->vox[1], p->vox[0], (int)ncx, 1, 0, -2 * p->mmax[0], p->vox[0], -1, st));
    // along y: b[vz][vy][ncx] -> a[vz][ncy][ncx]
    HIP_TRY(launch_dft_axis(b, a, p->vox[2], p->vox[1], (int)ncy, (int)ncx, 0, -2 * p->mmax[1], p->vox[1], -1, st));
    // along z: a[vz][ncy*ncx] -> coef[ncz][ncy*ncx]
    HIP_TRY(launch_dft_axis(a, coef, 1, p->vox[2], (int)ncz, (int)(ncy * ncx), 0, -2 * p->mmax[2], p->vox[2], -1, st));
    HIP_TRY(launch_box_factor(coef, p->nc, p->vox, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GSM_OK;
  };
  rc = image(geo->eps, p->d_coef);
  if (!rc) rc = image(inv.data(), p->d_coef_inv);
  hipFree(d_eps);
  hipFree(a);
  hipFree(b);
  if (rc) return cleanup(rc);
  *out = p;
  return GSM_OK;
}

int gsm_plan_shapes(const gsm_shape_body* body, const gsm_plan_opts* opts, gsm_plan_t* out) {
  int rc;
  if (!out) return fail(GSM_E_ARG, "out is NULL");
  if ((rc = check_shape_body(body)) || (rc = check_plan_opts(opts))) return rc;
  gsm_plan_s* p = nullptr;
  if ((rc = plan_begin(opts, body->period, &p))) return rc;
  auto cleanup = [&](int code) {
    gsm_plan_destroy(p);
    return code;
  };
  // permittivity statistics: the mean is c_0 (host plus each inclusion's
  // contrast times its volume fraction), the range spans host and inclusions
  const double cell = body->period[0] * body->period[1] * body->period[2];
  double mean = body->eps_host, mn = body->eps_host, mx = body->eps_host;
  std::vector<ShapeDesc> sd(body->n_shapes);
  for (int k = 0; k < body->n_shapes; ++k) {
    const gsm_shape& sh = body->shapes[k];
    ShapeDesc& d = sd[k];
    d.kind = sh.kind == GSM_SHAPE_BOX ? SHAPE_BOX : (sh.kind == GSM_SHAPE_SPHERE ? SHAPE_SPHERE : SHAPE_ELLIPSOID);
    d.pad = 0;
    for (int a = 0; a < 3; ++a) {
      d.centre[a] = sh.centre[a];
      d.size[a] = sh.kind == GSM_SHAPE_SPHERE ? sh.size[0] : sh.size[a];
    }
    d.weight = sh.eps - body->eps_host;
    const double vol = d.kind == SHAPE_BOX ? 8.0 * d.size[0] * d.size[1] * d.size[2]
                                           : 4.0 * M_PI / 3.0 * d.size[0] * d.size[1] * d.size[2];
    mean += d.weight * vol / cell;
    mn = std::min(mn, sh.eps);
    mx = std::max(mx, sh.eps);
  }
  p->eps_mean = mean;
  p->eps_min = mn;
  p->eps_max = mx;
  const long long ncn = (long long)p->nc[0] * p->nc[1] * p->nc[2];
  ShapeDesc* d_sh = nullptr;
  hipError_t e = dev_malloc(&p->d_coef, ncn * sizeof(double2));
  if (e == hipSuccess) e = dev_malloc(&p->d_coef_inv, ncn * sizeof(double2));
  if (e == hipSuccess) e = dev_malloc(&d_sh, 2 * std::max<size_t>(sd.size(), 1) * sizeof(ShapeDesc));
  if (e != hipSuccess) {
    hipFree(d_sh);
    return cleanup(fail(GSM_E_NOMEM, "plan allocation: %s", hipGetErrorString(e)));
  }
  // the same shapes weighted by 1/eps_i - 1/eps_h give the image of 1/eps
  std::vector<ShapeDesc> all = sd;
  for (int k = 0; k < body->n_shapes; ++k) {
    ShapeDesc d = sd[k];
    d.weight = 1.0 / body->shapes[k].eps - 1.0 / body->eps_host;
    all.push_back(d);
  }
  const int nsh = (int)sd.size();
  auto run = [&]() -> int {
    if (!all.empty()) HIP_TRY(hipMemcpy(d_sh, all.data(), all.size() * sizeof(ShapeDesc), hipMemcpyHostToDevice));
    HIP_TRY(launch_shape_image(p->d_coef, p->nc, p->period, body->eps_host, d_sh, nsh, nullptr));
    HIP_TRY(launch_shape_image(p->d_coef_inv, p->nc, p->period, 1.0 / body->eps_host, d_sh + nsh, nsh, nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    return GSM_OK;
  };
  rc = run();
  hipFree(d_sh);
  if (rc) return cleanup(rc);
  *out = p;
  return GSM_OK;
}

int gsm_plan_from_coeffs(const gsm_coeff_body* body, const gsm_plan_opts* opts, gsm_plan_t* out) {
  int rc;
  if (!out) return fail(GSM_E_ARG, "out is NULL");
  if ((rc = check_plan_opts(opts)) || (rc = check_coeff_body(body, opts))) return rc;
  gsm_plan_s* p = nullptr;
  if ((rc = plan_begin(opts, body->period, &p))) return rc;
  auto cleanup = [&](int code) {
    gsm_plan_destroy(p);
    return code;
  };
  const int sx = 2 * body->n_max[0] + 1, sy = 2 * body->n_max[1] + 1;
  p->eps_mean = body->coef[2 * (((long long)body->n_max[2] * sy + body->n_max[1]) * sx + body->n_max[0])];
  p->eps_min = body->eps_min;
  p->eps_max = body->eps_max;
  // the |n_a| <= 2 m_max block of the caller's arrays, gathered on the host
  const long long ncn = (long long)p->nc[0] * p->nc[1] * p->nc[2];
  auto take = [&](const double* from, double2** to) -> int {
    std::vector<double> blk(2 * ncn);
    for (int z = 0; z < p->nc[2]; ++z)
      for (int y = 0; y < p->nc[1]; ++y)
        for (int x = 0; x < p->nc[0]; ++x) {
          const long long src = ((long long)(z - 2 * p->mmax[2] + body->n_max[2]) * sy +
                                 (y - 2 * p->mmax[1] + body->n_max[1])) * sx +
                                (x - 2 * p->mmax[0] + body->n_max[0]);
          const long long dst = ((long long)z * p->nc[1] + y) * p->nc[0] + x;
          blk[2 * dst] = from[2 * src];
          blk[2 * dst + 1] = from[2 * src + 1];
        }
    if (dev_malloc(to, ncn * sizeof(double2)) != hipSuccess) return fail(GSM_E_NOMEM, "plan allocation failed");
    if (hipMemcpy(*to, blk.data(), ncn * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess)
      return fail(GSM_E_DEVICE, "copy of the coefficients failed");
    return GSM_OK;
  };
  if ((rc = take(body->coef, &p->d_coef))) return cleanup(rc);
  if (body->coef_inv && (rc = take(body->coef_inv, &p->d_coef_inv))) return cleanup(rc);
  *out = p;
  return GSM_OK;
}

int gsm_plan_destroy(gsm_plan_t p) {
  if (!p) return GSM_OK;
  hipSetDevice(p->device);
  for (auto& kv : p->grids) {
    hipFree(kv.second.g64);
    hipFree(kv.second.g32);
  }
  hipFree(p->d_coef);
  hipFree(p->d_coef_inv);
  for (auto& sl : p->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    if (sl.h_flags) hipHostFree(sl.h_flags);
    if (sl.h_inner) hipHostFree(sl.h_inner);
    if (sl.h_exp) hipHostFree(sl.h_exp);
    for (auto& ge : sl.graphs) hipGraphExecDestroy(ge.exec);
    for (auto& e : sl.step_ev)
      if (e) hipEventDestroy(e);
    if (sl.phase_ev) hipEventDestroy(sl.phase_ev);
    if (sl.stream) hipStreamDestroy(sl.stream);
  }
  delete p;
  return GSM_OK;
}

int gsm_plan_graph_stats(gsm_plan_t p, int64_t* captured, int64_t* launched) {
  if (!p) return fail(GSM_E_ARG, "NULL plan");
  if (captured) *captured = p->graph_captures;
  if (launched) *launched = p->graph_launches;
  return GSM_OK;
}

int gsm_allocation_stats(int64_t* count, int64_t* bytes) {
  if (count) *count = g_alloc_count.load();
  if (bytes) *bytes = g_alloc_bytes.load();
  return GSM_OK;
}

int gsm_plan_tuning(gsm_plan_t p, const int32_t M[3], int32_t precision, int32_t fam[4], int32_t* tuned) {
  if (!p || !M || !fam) return fail(GSM_E_ARG, "NULL argument");
  if (precision != GSM_MIXED && precision != GSM_FP64) return fail(GSM_E_ARG, "unknown precision %d", precision);
  const int P = fft_size_for(M);
  if (P < 0) return fail(GSM_E_UNSUPPORTED, "no FFT size for these orders");
  const int d = precision == GSM_FP64 ? 1 : 0;
  int f[4];
  int t = 0;
  auto g = p->grids.find({M[0], M[1], M[2], P, FORM_E});
  if (g != p->grids.end()) {
    for (int k = 0; k < 4; ++k) f[k] = g->second.fam[d][k];
    t = g->second.tuned[d];
  } else {
    default_families(P, d == 1, f);
    auto tk = p->tune_known.find({M[0], M[1], M[2], P, d});
    if (tk != p->tune_known.end()) {
      for (int k = 0; k < 4; ++k) f[k] = tk->second[k];
      t = 1;
    }
  }
  for (int k = 0; k < 4; ++k) fam[k] = f[k];
  if (tuned) *tuned = t;
  return GSM_OK;
}

int gsm_plan_coefficients(gsm_plan_t p, double* c_out) {
  if (!p || !c_out) return fail(GSM_E_ARG, "NULL argument");
  int rc;
  if ((rc = set_device(p))) return rc;
  const long long n = (long long)p->nc[0] * p->nc[1] * p->nc[2];
  HIP_TRY(hipMemcpy(c_out, p->d_coef, n * sizeof(double2), hipMemcpyDeviceToHost));
  return GSM_OK;
}

int gsm_plan_inverse_coefficients(gsm_plan_t p, double* c_out) {
  if (!p || !c_out) return fail(GSM_E_ARG, "NULL argument");
  if (!p->d_coef_inv) return fail(GSM_E_ARG, "the plan holds no inverse-permittivity coefficients");
  int rc;
  if ((rc = set_device(p))) return rc;
  const long long n = (long long)p->nc[0] * p->nc[1] * p->nc[2];
  HIP_TRY(hipMemcpy(c_out, p->d_coef_inv, n * sizeof(double2), hipMemcpyDeviceToHost));
  return GSM_OK;
}

int gsm_plan_contrast_grid(gsm_plan_t p, const int32_t M[3], int32_t P, double* g_out) {
  if (!p || !M || !g_out) return fail(GSM_E_ARG, "NULL argument");
  for (int a = 0; a < 3; ++a)
    if (M[a] < 0 || M[a] > p->mmax[a]) return fail(GSM_E_ARG, "M[%d]=%d outside the plan", a, M[a]);
  bool ok = false;
  for (int q : kSupportedP) ok |= q == P;
  if (!ok) return fail(GSM_E_UNSUPPORTED, "P=%d is not a supported FFT size", P);
  for (int a = 0; a < 3; ++a)
    if (P < 4 * M[a] + 1) return fail(GSM_E_ARG, "P=%d < 4 M + 1", P);
  int rc;
  if ((rc = set_device(p))) return rc;
  Grid* g = nullptr;
  int Mi[3] = {M[0], M[1], M[2]};
  if ((rc = ensure_grid(p, Mi, P, nullptr, &g))) return rc;
  HIP_TRY(hipMemcpy(g_out, g->g64, (size_t)P * P * P * sizeof(double), hipMemcpyDeviceToHost));
  return GSM_OK;
}

int gsm_basis_eps(gsm_plan_t p, const gsm_instance* inst, double* eps_b) {
  if (!p || !inst || !eps_b) return fail(GSM_E_ARG, "NULL argument");
  int rc = check_instance(*inst, p->mmax, 0, false);
  if (rc) return rc;
  return resolve_eps_b(p->period, p->eps_mean, p->eps_min, p->eps_max, *inst, 0, eps_b);
}

int gsm_workspace_size(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, const gsm_solver_opts* so,
                       size_t* bytes) {
  if (!p || !bytes) return fail(GSM_E_ARG, "NULL argument");
  if (n_inst < 0 || (n_inst > 0 && !inst)) return fail(GSM_E_ARG, "bad instance list");
  gsm_solver_opts d;
  if (!so) {
    gsm_solver_opts_default(&d);
    so = &d;
  }
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  std::vector<SysDesc> sys;
  // size for three drives per instance when that is larger (gsm_eff_tensor)
  std::vector<SysDesc> sys3;
  if ((rc = build_systems(p, n_inst, inst, so, true, sys3))) return rc;
  std::vector<Group> groups;
  build_groups(sys3, groups, so->group_max);
  // plus the effective-tensor region (fields and correlation buffers), so
  // that no call on the workspace allocates device memory of its own
  *bytes = workspace_for(groups, so->restart, so->precision == GSM_FP64) + aux_layout(p, sys3, nullptr, nullptr);
  return GSM_OK;
}

int gsm_solve(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, const gsm_solver_opts* so, void* ws,
              size_t ws_bytes, double* E_out, gsm_solve_info* info, void* stream) {
  if (!p || !inst || n_inst < 1 || !E_out || !info) return fail(GSM_E_ARG, "NULL argument or n_inst < 1");
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  if ((rc = set_device(p))) return rc;
  std::vector<SysDesc> sys;
  if ((rc = build_systems(p, n_inst, inst, so, false, sys))) return rc;
  std::vector<Group> groups;
  build_groups(sys, groups, so->group_max);
  hipStream_t st = (hipStream_t)stream;
  std::vector<SysExport> exp;
  rc = solve_all(p, sys, groups, so, ws, ws_bytes, E_out, (so->flags & GSM_OUT_HOST) != 0, exp, st);
  if (rc) return rc;
  int worst = GSM_OK;
  fill_info(sys, exp, info, &worst);
  return worst;
}

int gsm_apply(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, int32_t precision, int32_t mode,
              const void* x, void* y, void* ws, size_t ws_bytes, void* stream) {
  if (!p || !inst || n_inst < 1 || !x || !y) return fail(GSM_E_ARG, "NULL argument or n_inst < 1");
  if (precision != GSM_FP64 && precision != GSM_MIXED) return fail(GSM_E_ARG, "unknown precision");
  if (mode != GSM_APPLY_FORWARD && mode != GSM_APPLY_ADJOINT && mode != GSM_APPLY_FORWARD_H)
    return fail(GSM_E_ARG, "unknown mode");
  int rc;
  if ((rc = set_device(p))) return rc;
  gsm_solver_opts so;
  gsm_solver_opts_default(&so);
  so.precision = precision;
  so.formulation = mode == GSM_APPLY_FORWARD_H ? GSM_FORM_H : GSM_FORM_E;
  std::vector<SysDesc> sys;
  if ((rc = build_systems(p, n_inst, inst, &so, false, sys))) return rc;
  std::vector<Group> groups;
  build_groups(sys, groups, 0);  // one pass: nothing to overlap, and never more groups than the workspace query
  if ((rc = carve(groups, ws, ws_bytes, so.restart, precision == GSM_FP64))) return rc;
  hipStream_t st = (hipStream_t)stream;
  for (auto& g : groups) {
    Grid* grid = nullptr;
    if ((rc = ensure_grid(p, g.shape.M, g.shape.P, st, &grid, g.shape.form))) return rc;
    if ((rc = apply_group(g, sys, grid, precision == GSM_FP64, mode, x, y, st))) return rc;
  }
  return GSM_OK;
}

int gsm_apply_static(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, int32_t precision, int32_t mode,
                     const void* x, void* y, void* stream) {
  if (!p || !inst || n_inst < 1 || !x || !y) return fail(GSM_E_ARG, "NULL argument or n_inst < 1");
  if (precision != GSM_FP64 && precision != GSM_MIXED) return fail(GSM_E_ARG, "unknown precision");
  if (mode != GSM_APPLY_FORWARD && mode != GSM_APPLY_ADJOINT && mode != GSM_APPLY_FORWARD_H)
    return fail(GSM_E_ARG, "unknown mode");
  int rc;
  if ((rc = set_device(p))) return rc;
  char* base = nullptr;
  if ((rc = static_scratch(p->device, &base))) return rc;
  gsm_solver_opts so;
  gsm_solver_opts_default(&so);
  so.precision = precision;
  so.formulation = mode == GSM_APPLY_FORWARD_H ? GSM_FORM_H : GSM_FORM_E;
  std::vector<SysDesc> sys;
  if ((rc = build_systems(p, n_inst, inst, &so, false, sys))) return rc;
  std::vector<Group> groups;
  build_groups(sys, groups, 0);
  const bool dbl = precision == GSM_FP64;
  const size_t eb = dbl ? sizeof(double2) : sizeof(float2);
  // every group must fit on its own (groups run one after the other and each
  // starts at the base of the array) and its contrast grid must exist already
  std::vector<Grid*> grids;
  for (auto& g : groups) {
    const size_t need = layout_apply(g, nullptr, eb);
    if (need > kScratchBytes)
      return fail(GSM_E_WORKSPACE,
                  "gsm_apply_static: %d systems at M = (%d, %d, %d) need %zu bytes of scratch, the static array "
                  "holds %zu (split the call)",
                  g.shape.S, g.shape.M[0], g.shape.M[1], g.shape.M[2], need, kScratchBytes);
    auto it = p->grids.find({g.shape.M[0], g.shape.M[1], g.shape.M[2], g.shape.P, g.shape.form});
    if (it == p->grids.end())
      return fail(GSM_E_ARG,
                  "gsm_apply_static: the plan has no contrast grid for M = (%d, %d, %d), P = %d yet (one call of "
                  "gsm_apply, gsm_solve or gsm_plan_contrast_grid with these orders makes it)",
                  g.shape.M[0], g.shape.M[1], g.shape.M[2], g.shape.P);
    grids.push_back(&it->second);
  }
  hipStream_t st = (hipStream_t)stream;
  for (size_t k = 0; k < groups.size(); ++k) {
    layout_apply(groups[k], base, eb);
    if ((rc = apply_group(groups[k], sys, grids[k], dbl, mode, x, y, st))) return rc;
  }
  return GSM_OK;
}

int gsm_eff_tensor(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, const gsm_solver_opts* so,
                   double* eps_eff, double* E_save, void* ws, size_t ws_bytes, gsm_solve_info* info,
                   void* stream) {
  if (!p || !inst || n_inst < 1 || !eps_eff || !info) return fail(GSM_E_ARG, "NULL argument or n_inst < 1");
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  if (so->formulation != GSM_FORM_E)
    return fail(GSM_E_ARG, "the effective tensor D0 E0^-1 is defined on the E-field system (formulation E)");
  if ((rc = set_device(p))) return rc;
  std::vector<SysDesc> sys;
  if ((rc = build_systems(p, n_inst, inst, so, true, sys))) return rc;
  std::vector<Group> groups;
  build_groups(sys, groups, so->group_max);
  hipStream_t st = (hipStream_t)stream;
  Aux ax;
  if ((rc = carve_aux(p, groups, sys, ws, ws_bytes, so->restart, so->precision == GSM_FP64, &ax))) return rc;
  // the fields go to the caller's E_save, else to the workspace
  double* E = E_save ? E_save : (double*)ax.f[0];
  std::vector<SysExport> exp;
  gsm_solver_opts so2 = *so;
  so2.flags &= ~GSM_OUT_HOST;
  rc = solve_all(p, sys, groups, &so2, ws, ws_bytes, E, false, exp, st);
  if (rc) return rc;
  int worst = GSM_OK;
  fill_info(sys, exp, info, &worst);
  using cd = std::complex<double>;
  for (int i = 0; i < n_inst; ++i) {
    cd E0[3][3], D0[3][3];
    for (int d = 0; d < 3; ++d) {
      const SysExport& e = exp[3 * i + d];
      const double eb = sys[3 * i + d].par.eps_b;
      for (int c = 0; c < 3; ++c) {
        E0[c][d] = cd(e.e0[c].x, e.e0[c].y);
        D0[c][d] = eb * (cd(e.e0[c].x, e.e0[c].y) + cd(e.w0[c].x, e.w0[c].y));
      }
    }
    // inverse of E0 by cofactors
    const cd det = E0[0][0] * (E0[1][1] * E0[2][2] - E0[1][2] * E0[2][1]) -
                   E0[0][1] * (E0[1][0] * E0[2][2] - E0[1][2] * E0[2][0]) +
                   E0[0][2] * (E0[1][0] * E0[2][1] - E0[1][1] * E0[2][0]);
    double scale = 0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) scale = std::max(scale, std::abs(E0[r][c]));
    if (!(std::abs(det) > 1e-14 * scale * scale * scale))
      return fail(GSM_E_SINGULAR, "instance %d: zeroth-order field matrix E0 is singular", i);
    cd inv[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        inv[r][c] = (E0[r1][c1] * E0[r2][c2] - E0[r1][c2] * E0[r2][c1]) / det;
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        cd v = 0;
        for (int k = 0; k < 3; ++k) v += D0[r][k] * inv[k][c];
        eps_eff[(9 * i + 3 * r + c) * 2] = v.real();
        eps_eff[(9 * i + 3 * r + c) * 2 + 1] = v.imag();
      }
  }
  return worst;
}

int gsm_pole_workspace_size(gsm_plan_t p, int32_t n_q, const gsm_pole_query* q, const gsm_solver_opts* so,
                            size_t* bytes) {
  if (!p || !q || n_q < 1 || !bytes) return fail(GSM_E_ARG, "NULL argument or n_q < 1");
  gsm_solver_opts d;
  if (!so) {
    gsm_solver_opts_default(&d);
    so = &d;
  }
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  std::vector<gsm_instance> mesh;
  std::vector<double> kappa, eb;
  std::vector<SysDesc> sys;
  std::vector<Group> groups;
  if ((rc = pole_systems(p, n_q, q, so, mesh, kappa, eb, sys, groups))) return rc;
  long long n_eta = 0;
  for (int i = 0; i < n_q; ++i) n_eta += q[i].n_poles;
  *bytes = workspace_for(groups, so->restart, so->precision == GSM_FP64) + pole_layout(sys, n_eta, n_q, nullptr, nullptr);
  return GSM_OK;
}

int gsm_pole_search(gsm_plan_t p, int32_t n_q, const gsm_pole_query* q, const gsm_solver_opts* so, void* ws,
                    size_t ws_bytes, gsm_pole_result* out, void* stream) {
  if (!p || !q || n_q < 1 || !out) return fail(GSM_E_ARG, "NULL argument or n_q < 1");
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  if ((rc = set_device(p))) return rc;
  std::vector<gsm_instance> mesh;
  std::vector<double> kappa, eb;
  std::vector<SysDesc> sys;
  std::vector<Group> groups;
  if ((rc = pole_systems(p, n_q, q, so, mesh, kappa, eb, sys, groups))) return rc;
  long long n_eta = 0;
  for (int i = 0; i < n_q; ++i) n_eta += q[i].n_poles;
  const size_t gbytes = workspace_for(groups, so->restart, so->precision == GSM_FP64);
  const size_t need = gbytes + pole_layout(sys, n_eta, n_q, nullptr, nullptr);
  if (!ws) return fail(GSM_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(GSM_E_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  // the groups' buffers come first (gbytes includes 256 bytes of alignment slack)
  char* base = (char*)(((uintptr_t)ws + 255) & ~uintptr_t(255)) + (gbytes - 256);
  PoleBufs b;
  pole_layout(sys, n_eta, n_q, base, &b);
  hipStream_t st = (hipStream_t)stream;
  std::vector<SysExport> exp;
  gsm_solver_opts so2 = *so;
  so2.flags &= ~GSM_OUT_HOST;
  so2.x0 = nullptr;
  if ((rc = solve_all(p, sys, groups, &so2, ws, ws_bytes, (double*)b.E, false, exp, st))) return rc;
  // xi_i: the chosen component of each mesh field's zeroth harmonic
  std::vector<long long> idx(sys.size());
  size_t si = 0;
  for (int i = 0; i < n_q; ++i) {
    const int npts = q[i].n_div + q[i].n_poles;
    for (int k = 0; k < npts; ++k, ++si) {
      const SysDesc& s = sys[si];
      const long long n1x = 2 * s.M[0] + 1, n1y = 2 * s.M[1] + 1, n1z = 2 * s.M[2] + 1;
      const long long i0 = ((long long)s.M[2] * n1y + s.M[1]) * n1x + s.M[0];
      idx[si] = s.out_off + (long long)q[i].component * n1x * n1y * n1z + i0;
    }
  }
  HIP_TRY(hipMemcpyAsync(b.idx, idx.data(), idx.size() * sizeof(long long), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(b.kappa, kappa.data(), kappa.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_gather_zero_order(b.E, b.idx, b.xi, (int)sys.size(), st));
  // one fit launch per run of consecutive queries with equal (N_p, N_d)
  long long pt = 0, et = 0;
  for (int i = 0; i < n_q;) {
    int j = i;
    while (j < n_q && q[j].n_poles == q[i].n_poles && q[j].n_div == q[i].n_div) ++j;
    PoleFitArgs fa{};
    fa.n = j - i;
    fa.n_poles = q[i].n_poles;
    fa.n_div = q[i].n_div;
    fa.kappa = b.kappa + pt;
    fa.xi = b.xi + 2 * pt;
    fa.eta = b.eta + 2 * et;
    fa.zeta = b.zeta + 2 * et;
    fa.status = b.status + i;
    HIP_TRY(launch_pole_fit(fa, st));
    pt += (long long)(j - i) * (q[i].n_div + q[i].n_poles);
    et += (long long)(j - i) * q[i].n_poles;
    i = j;
  }
  std::vector<double> eta(2 * n_eta), zeta(2 * n_eta);
  std::vector<int> fst(n_q);
  HIP_TRY(hipMemcpyAsync(eta.data(), b.eta, eta.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(zeta.data(), b.zeta, zeta.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(fst.data(), b.status, n_q * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int worst = GSM_OK;
  si = 0;
  et = 0;
  for (int i = 0; i < n_q; ++i) {
    gsm_pole_result r{};
    const int npts = q[i].n_div + q[i].n_poles, Np = q[i].n_poles;
    r.status = GSM_OK;
    r.n_poles = Np;
    r.eps_b = eb[i];
    for (int k = 0; k < npts; ++k, ++si) {
      if (exp[si].status != 0) r.status = GSM_W_NOT_CONVERGED;
      r.iterations += exp[si].iters;
      r.max_rel_residual = std::max(r.max_rel_residual, exp[si].rel);
    }
    if (fst[i] != GSM_OK) r.status = fst[i];
    const double k0 = 2.0 * M_PI / q[i].wavelength;
    r.best = -1;
    double bz = -1;
    for (int k = 0; k < Np; ++k) {
      for (int c = 0; c < 2; ++c) {
        r.eta[k][c] = eta[2 * (et + k) + c];
        r.zeta[k][c] = zeta[2 * (et + k) + c];
      }
      const double az = std::hypot(r.zeta[k][0], r.zeta[k][1]);
      // a mode of the window: real part inside it, within half its width of
      // the real axis (poles far off it model the regular part of xi)
      const bool near = r.eta[k][0] >= q[i].kappa_min && r.eta[k][0] <= q[i].kappa_max &&
                        std::fabs(r.eta[k][1]) <= 0.5 * (q[i].kappa_max - q[i].kappa_min);
      if (fst[i] == GSM_OK && near && az > bz) {
        bz = az;
        r.best = k;
      }
    }
    r.n_eff = r.best >= 0 ? r.eta[r.best][0] / k0 : 0.0;
    et += Np;
    out[i] = r;
    if (r.status < 0 && (worst >= 0 || r.status < worst)) worst = r.status;
    if (r.status > 0 && worst == GSM_OK) worst = r.status;
  }
  return worst;
}

int gsm_pole_fit(int32_t n, int32_t n_poles, int32_t n_div, const double* kappa, const double* xi, double* eta,
                 double* zeta, int32_t* status, void* stream) {
  if (n < 0) return fail(GSM_E_ARG, "n < 0");
  if (n_poles < 1 || n_poles > GSM_POLE_MAX_NP) return fail(GSM_E_ARG, "n_poles=%d outside [1, %d]", n_poles, GSM_POLE_MAX_NP);
  if (n_div <= n_poles || n_div > GSM_POLE_MAX_ND)
    return fail(GSM_E_ARG, "n_div=%d must exceed n_poles and be <= %d", n_div, GSM_POLE_MAX_ND);
  if (n == 0) return GSM_OK;
  if (!kappa || !xi || !eta || !zeta || !status) return fail(GSM_E_ARG, "NULL argument");
  PoleFitArgs fa{};
  fa.n = n;
  fa.n_poles = n_poles;
  fa.n_div = n_div;
  fa.kappa = kappa;
  fa.xi = xi;
  fa.eta = eta;
  fa.zeta = zeta;
  fa.status = status;
  HIP_TRY(launch_pole_fit(fa, (hipStream_t)stream));
  return GSM_OK;
}

namespace {

// ---- Fresnel normal surface (host): 3x3 row-major helpers

double det3(const double* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

// adjugate: adj(a) a = det(a) I; d det(a) / d a_ij = adj(a)_ji
void adj3(const double* a, double* c) {
  c[0] = a[4] * a[8] - a[5] * a[7];
  c[1] = a[2] * a[7] - a[1] * a[8];
  c[2] = a[1] * a[5] - a[2] * a[4];
  c[3] = a[5] * a[6] - a[3] * a[8];
  c[4] = a[0] * a[8] - a[2] * a[6];
  c[5] = a[2] * a[3] - a[0] * a[5];
  c[6] = a[3] * a[7] - a[4] * a[6];
  c[7] = a[1] * a[6] - a[0] * a[7];
  c[8] = a[0] * a[4] - a[1] * a[3];
}

bool unit3(const double* k, double* u) {
  const double nn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  if (!(nn > 0.0)) return false;
  for (int i = 0; i < 3; ++i) u[i] = k[i] / nn;
  return true;
}

// roots t = n^2, ascending, of (u.e.u) t^2 - (tr C - u.C.u) t + det e = 0
int fresnel_roots(const double* e, const double* u, double* t) {
  double c[9];
  adj3(e, c);
  double qa = 0.0, qc = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      qa += u[i] * e[3 * i + j] * u[j];
      qc += u[i] * c[3 * i + j] * u[j];
    }
  const double b = c[0] + c[4] + c[8] - qc, d = det3(e);
  if (!(qa > 0.0) || !(d > 0.0)) return GSM_E_SINGULAR;
  double disc = b * b - 4.0 * qa * d;
  if (disc < 0.0) {
    if (disc < -1e-12 * b * b) return GSM_E_SINGULAR;
    disc = 0.0;  // a double root (isotropic, or an optic axis) rounded below zero
  }
  const double q = 0.5 * (b + std::sqrt(disc));
  if (!(q > 0.0)) return GSM_E_SINGULAR;
  const double t1 = d / q, t2 = q / qa;  // smaller, larger (product d / qa)
  t[0] = std::min(t1, t2);
  t[1] = std::max(t1, t2);
  return GSM_OK;
}

// symmetric tensor of the fit parameters: xx, yy, zz (diagonal), then xy, xz, yz
void fresnel_tensor(const double* p, bool diag, double* e) {
  e[0] = p[0];
  e[4] = p[1];
  e[8] = p[2];
  e[1] = e[3] = diag ? 0.0 : p[3];
  e[2] = e[6] = diag ? 0.0 : p[4];
  e[5] = e[7] = diag ? 0.0 : p[5];
}

// Solve the np x np symmetric positive system A x = b in place (Cholesky);
// false when a pivot falls below rel_tol times the largest diagonal.
bool spd_solve(double* A, double* b, int np, double rel_tol) {
  double dmax = 0.0;
  for (int i = 0; i < np; ++i) dmax = std::max(dmax, A[i * np + i]);
  if (!(dmax > 0.0)) return false;
  for (int j = 0; j < np; ++j) {
    double s = A[j * np + j];
    for (int k = 0; k < j; ++k) s -= A[j * np + k] * A[j * np + k];
    if (!(s > rel_tol * dmax)) return false;
    const double l = std::sqrt(s);
    A[j * np + j] = l;
    for (int i = j + 1; i < np; ++i) {
      double v = A[i * np + j];
      for (int k = 0; k < j; ++k) v -= A[i * np + k] * A[j * np + k];
      A[i * np + j] = v / l;
    }
  }
  for (int i = 0; i < np; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= A[i * np + k] * b[k];
    b[i] = v / A[i * np + i];
  }
  for (int i = np - 1; i >= 0; --i) {
    double v = b[i];
    for (int k = i + 1; k < np; ++k) v -= A[k * np + i] * b[k];
    b[i] = v / A[i * np + i];
  }
  return true;
}

}  // namespace

int gsm_fresnel_indices(const double* eps, const double* k_hat, double* n_out) {
  if (!eps || !k_hat || !n_out) return fail(GSM_E_ARG, "NULL argument");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(eps[i])) return fail(GSM_E_NONFINITE, "eps not finite");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(k_hat[i])) return fail(GSM_E_NONFINITE, "k_hat not finite");
  double u[3], e[9], t[2];
  if (!unit3(k_hat, u)) return fail(GSM_E_ARG, "zero direction");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) e[3 * i + j] = eps[3 * std::min(i, j) + std::max(i, j)];
  if (fresnel_roots(e, u, t) != GSM_OK)
    return fail(GSM_E_SINGULAR, "the normal equation has no two positive roots along this direction");
  n_out[0] = std::sqrt(t[0]);
  n_out[1] = std::sqrt(t[1]);
  return GSM_OK;
}

int gsm_fresnel_fit(int32_t n_dir, const double* k_hat, const double* n_pair, int32_t diagonal, double* eps_out,
                    double* rms_out) {
  if (!k_hat || !n_pair || !eps_out) return fail(GSM_E_ARG, "NULL argument");
  const bool diag = diagonal != 0;
  const int np = diag ? 3 : 6;
  if (n_dir < np) return fail(GSM_E_ARG, "%d directions cannot determine %d components", n_dir, np);
  std::vector<double> U(3 * (size_t)n_dir), T(2 * (size_t)n_dir);
  for (int d = 0; d < n_dir; ++d) {
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(k_hat[3 * d + i])) return fail(GSM_E_NONFINITE, "direction %d not finite", d);
    if (!unit3(k_hat + 3 * d, &U[3 * d])) return fail(GSM_E_ARG, "direction %d is zero", d);
    for (int r = 0; r < 2; ++r) {
      const double n = n_pair[2 * d + r];
      if (!std::isfinite(n)) return fail(GSM_E_NONFINITE, "index %d of direction %d not finite", r, d);
      if (!(n > 0.0)) return fail(GSM_E_ARG, "index %d of direction %d is not positive", r, d);
      T[2 * d + r] = n * n;
    }
  }
  // linear estimate: u.E.u = 1 / (t1 t2) with E = eps / det(eps)
  double N[36] = {}, g[6] = {};
  for (int d = 0; d < n_dir; ++d) {
    const double* u = &U[3 * d];
    const double row[6] = {u[0] * u[0], u[1] * u[1], u[2] * u[2], 2 * u[0] * u[1], 2 * u[0] * u[2], 2 * u[1] * u[2]};
    const double b = 1.0 / (T[2 * d] * T[2 * d + 1]);
    for (int i = 0; i < np; ++i) {
      g[i] += row[i] * b;
      for (int j = 0; j < np; ++j) N[i * np + j] += row[i] * row[j];
    }
  }
  if (!spd_solve(N, g, np, 1e-12)) return fail(GSM_E_SINGULAR, "the directions do not determine the tensor");
  double e[9], p[6];
  fresnel_tensor(g, diag, e);
  const double dE = det3(e);
  if (!(dE > 0.0)) return fail(GSM_E_SINGULAR, "the linear estimate is not positive definite");
  const double scale = 1.0 / std::sqrt(dE);
  for (int i = 0; i < np; ++i) p[i] = g[i] * scale;
  // Levenberg-Marquardt on r = det(eps - t P) / t^3
  const int m = 2 * n_dir;
  std::vector<double> r(m), rt(m), J((size_t)m * np);
  // residuals of parameters pp into rr (and the Jacobian into J when asked)
  auto eval = [&](const double* pp, double* rr, bool jac) {
    double ee[9], A[9], C[9], ss = 0.0;
    fresnel_tensor(pp, diag, ee);
    for (int o = 0; o < m; ++o) {
      const double* u = &U[3 * (o / 2)];
      const double t = T[o], it3 = 1.0 / (t * t * t);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[3 * i + j] = ee[3 * i + j] - t * ((i == j ? 1.0 : 0.0) - u[i] * u[j]);
      rr[o] = det3(A) * it3;
      ss += rr[o] * rr[o];
      if (jac) {
        adj3(A, C);
        double* Jo = &J[(size_t)o * np];
        Jo[0] = C[0] * it3;
        Jo[1] = C[4] * it3;
        Jo[2] = C[8] * it3;
        if (!diag) {
          Jo[3] = (C[1] + C[3]) * it3;
          Jo[4] = (C[2] + C[6]) * it3;
          Jo[5] = (C[5] + C[7]) * it3;
        }
      }
    }
    return ss;
  };
  double ss = eval(p, r.data(), true), mu = 1e-3;
  for (int it = 0; it < 200 && ss > 0.0; ++it) {
    double JtJ[36] = {}, Jtr[6] = {};
    for (int o = 0; o < m; ++o)
      for (int i = 0; i < np; ++i) {
        Jtr[i] -= J[(size_t)o * np + i] * r[o];
        for (int j = 0; j < np; ++j) JtJ[i * np + j] += J[(size_t)o * np + i] * J[(size_t)o * np + j];
      }
    double A[36], step[6], trial[6];
    for (int i = 0; i < np * np; ++i) A[i] = JtJ[i];
    for (int i = 0; i < np; ++i) {
      A[i * np + i] *= 1.0 + mu;
      step[i] = Jtr[i];
    }
    if (!spd_solve(A, step, np, 1e-300)) break;
    double sn = 0.0, pn = 0.0;
    for (int i = 0; i < np; ++i) {
      trial[i] = p[i] + step[i];
      sn += step[i] * step[i];
      pn += p[i] * p[i];
    }
    const double ss_new = eval(trial, rt.data(), false);
    if (ss_new < ss) {
      for (int i = 0; i < np; ++i) p[i] = trial[i];
      ss = eval(p, r.data(), true);
      mu = std::max(mu / 3.0, 1e-12);
    } else {
      mu *= 4.0;
      if (mu > 1e12) break;
    }
    if (sn <= 1e-30 * (1.0 + pn)) break;
  }
  fresnel_tensor(p, diag, eps_out);
  if (rms_out) *rms_out = std::sqrt(eval(p, rt.data(), false) / m);
  return GSM_OK;
}

int gsm_profile_begin(void) { return gsm_profile_begin_sampled(nullptr, 1); }

int gsm_profile_begin_only(const char* cls) { return gsm_profile_begin_sampled(cls, 1); }

int gsm_profile_begin_sampled(const char* cls, int32_t every) {
  if (every < 1) return fail(GSM_E_ARG, "sampling period %d must be >= 1", every);
  int only = -1;
  if (cls) {
    for (int c = 0; c < K_NBASE; ++c)
      if (std::strcmp(cls, kClassNames[c]) == 0) only = c;
    if (only < 0) return fail(GSM_E_ARG, "unknown kernel class '%s'", cls);
  }
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.only = only;
  g_prof.every = every;
  for (auto& q : g_prof.seq) q = 0;
  g_prof.recs.clear();
  g_prof.used = 0;
  g_prof.on = true;
  return GSM_OK;
}

int gsm_profile_end(gsm_kernel_stat* out, int32_t max, int32_t* n_out) {
  if (!g_prof.on) return fail(GSM_E_ARG, "profiling was not started");
  g_prof.on = false;
  HIP_TRY(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_prof.mu);
  std::vector<gsm_kernel_stat> st(2 * K_NBASE);
  for (int c = 0; c < 2 * K_NBASE; ++c) {
    std::memset(&st[c], 0, sizeof st[c]);
    snprintf(st[c].name, sizeof st[c].name, "%s_%s", kClassNames[c / 2], (c & 1) ? "c128" : "c64");
  }
  for (auto& r : g_prof.recs) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    st[r.cls].launches += 1;
    st[r.cls].ms += ms;
    st[r.cls].bytes += r.step == -1 ? r.bytes : 0.0;
    st[r.cls].bytes_min += r.step == -1 ? r.bytes * r.pmin_ratio : 0.0;
    st[r.cls].flops += r.step == -1 ? r.flops : 0.0;
  }
  g_prof.recs.clear();
  g_prof.used = 0;
  int k = 0;
  for (int c = 0; c < 2 * K_NBASE; ++c)
    if (st[c].launches > 0) {
      if (out && k < max) out[k] = st[c];
      ++k;
    }
  if (n_out) *n_out = k;
  return GSM_OK;
}

int gsm_solve_adjoint(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, const gsm_solver_opts* so,
                      const double* rhs, double* lambda_out, void* ws, size_t ws_bytes, gsm_solve_info* info,
                      void* stream) {
  if (!p || !inst || n_inst < 1 || !rhs || !lambda_out || !info)
    return fail(GSM_E_ARG, "NULL argument or n_inst < 1");
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  if (so->formulation != GSM_FORM_E) return fail(GSM_E_ARG, "the adjoint solve is built for the E-field system");
  if ((rc = set_device(p))) return rc;
  std::vector<SysDesc> sys;
  if ((rc = build_systems(p, n_inst, inst, so, false, sys))) return rc;
  std::vector<Group> groups;
  build_groups(sys, groups, so->group_max);
  std::vector<SysExport> exp;
  rc = solve_all(p, sys, groups, so, ws, ws_bytes, lambda_out, (so->flags & GSM_OUT_HOST) != 0, exp,
                 (hipStream_t)stream, rhs);
  if (rc) return rc;
  int worst = GSM_OK;
  fill_info(sys, exp, info, &worst);
  return worst;
}

namespace {

// Zero-padded inverse DFT of one component block [N1z][N1y][N1x] onto P^3.
int expand3(const double2* in, const int M[3], int P, double2* t1, double2* t2, double2* out, hipStream_t st) {
  const int N1[3] = {2 * M[0] + 1, 2 * M[1] + 1, 2 * M[2] + 1};
  HIP_TRY(launch_dft_axis(in, t1, N1[2] * N1[1], N1[0], P, 1, -M[0], 0, P, +1, st));
  HIP_TRY(launch_dft_axis(t1, t2, N1[2], N1[1], P, P, -M[1], 0, P, +1, st));
  HIP_TRY(launch_dft_axis(t2, out, 1, N1[2], P, P * P, -M[2], 0, P, +1, st));
  return GSM_OK;
}

using cplxd = std::complex<double>;

void inv3(const cplxd a[3][3], cplxd inv[3][3], cplxd* det_out) {
  const cplxd det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                    a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      inv[r][c] = (a[r1][c1] * a[r2][c2] - a[r1][c2] * a[r2][c1]) / det;
    }
  *det_out = det;
}

}  // namespace

int gsm_eff_tensor_vjp(gsm_plan_t p, int32_t n_inst, const gsm_instance* inst, const gsm_solver_opts* so,
                       const double* E_save, const double* eps_eff, const double* gbar, double* grad_vox, void* ws,
                       size_t ws_bytes, gsm_solve_info* info, void* stream) {
  if (!p || !inst || n_inst < 1 || !E_save || !eps_eff || !gbar || !grad_vox || !info)
    return fail(GSM_E_ARG, "NULL argument or n_inst < 1");
  if (!p->voxel_body)
    return fail(GSM_E_ARG, "the plan was made from shapes or coefficients: it has no voxels to differentiate by");
  int rc;
  if ((rc = check_solver_opts(so))) return rc;
  if (so->formulation != GSM_FORM_E) return fail(GSM_E_ARG, "the gradient is built for the E-field system");
  if ((rc = set_device(p))) return rc;
  hipStream_t st = (hipStream_t)stream;
  std::vector<SysDesc> sys;
  if ((rc = build_systems(p, n_inst, inst, so, true, sys))) return rc;
  std::vector<Group> groups;
  build_groups(sys, groups, so->group_max);
  // right-hand sides, adjoint solutions and correlation buffers: workspace
  Aux ax;
  if ((rc = carve_aux(p, groups, sys, ws, ws_bytes, so->restart, so->precision == GSM_FP64, &ax))) return rc;
  double2* rhs = ax.f[0];
  double2* lam = ax.f[1];
  std::vector<AdjInst> ais(n_inst);
  const double2* E = (const double2*)E_save;
  for (int i = 0; i < n_inst; ++i) {
    const SysDesc& s0 = sys[3 * i];
    const long long N = s0.n / 3;
    const long long i0 = ((long long)s0.M[2] * (2 * s0.M[1] + 1) + s0.M[1]) * (2 * s0.M[0] + 1) + s0.M[0];
    cplxd E0[3][3], E0inv[3][3], det, ee[3][3], gb[3][3];
    for (int d = 0; d < 3; ++d)
      for (int a = 0; a < 3; ++a) {
        double2 v;
        if (hipMemcpy(&v, E + sys[3 * i + d].out_off + a * N + i0, sizeof v, hipMemcpyDeviceToHost) != hipSuccess)
          return fail(GSM_E_DEVICE, "reading the saved fields failed");
        E0[a][d] = cplxd(v.x, v.y);
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        ee[r][c] = cplxd(eps_eff[(9 * i + 3 * r + c) * 2], eps_eff[(9 * i + 3 * r + c) * 2 + 1]);
        gb[r][c] = cplxd(gbar[(9 * i + 3 * r + c) * 2], gbar[(9 * i + 3 * r + c) * 2 + 1]);
      }
    inv3(E0, E0inv, &det);
    if (!(std::abs(det) > 0)) return fail(GSM_E_SINGULAR, "instance %d: E0 is singular", i);
    AdjInst& ai = ais[i];
    std::memset(&ai, 0, sizeof ai);
    for (int a = 0; a < 3; ++a) {
      ai.M[a] = s0.M[a];
      ai.N1[a] = 2 * s0.M[a] + 1;
      ai.mmax[a] = p->mmax[a];
      ai.q0[a] = s0.par.q0[a];
      ai.b[a] = s0.par.b[a];
    }
    ai.n = s0.n;
    ai.eps_b = s0.par.eps_b;
    // W = Gbar E0^-H: column p is w_p; u_p = eps_eff^H w_p
    for (int pp = 0; pp < 3; ++pp) {
      cplxd w[3];
      for (int a = 0; a < 3; ++a) {
        w[a] = 0;
        for (int k = 0; k < 3; ++k) w[a] += gb[a][k] * std::conj(E0inv[pp][k]);
        ai.w[pp][a] = make_double2(w[a].real(), w[a].imag());
      }
      for (int a = 0; a < 3; ++a) {
        cplxd u = 0;
        for (int k = 0; k < 3; ++k) u += std::conj(ee[k][a]) * w[k];
        ai.u[pp][a] = make_double2(u.real(), u.imag());
      }
    }
    if (hipSuccess != launch_adjoint_rhs(p->d_coef, ai, rhs + s0.out_off, st))
      return fail(GSM_E_DEVICE, "adjoint right-hand side launch failed");
  }
  std::vector<SysExport> exp;
  rc = solve_all(p, sys, groups, so, ws, ws_bytes, (double*)lam, false, exp, st, (const double*)rhs);
  if (rc) return rc;
  const long long nvox = (long long)p->vox[0] * p->vox[1] * p->vox[2];
  for (int i = 0; i < n_inst; ++i) {
    const SysDesc& s0 = sys[3 * i];
    const AdjInst& ai = ais[i];
    const int P = s0.P;
    const long long P3 = (long long)P * P * P;
    const long long N = s0.n / 3;
    const int nc[3] = {4 * ai.M[0] + 1, 4 * ai.M[1] + 1, 4 * ai.M[2] + 1};
    double2 *t1 = ax.tmp[AUX_T1], *t2 = ax.tmp[AUX_T2], *ah = ax.tmp[AUX_AH], *eh = ax.tmp[AUX_EH];
    double2 *Y = ax.tmp[AUX_Y], *X = ax.tmp[AUX_X], *gv = ax.tmp[AUX_GV];
    auto run = [&]() -> int {
      HIP_TRY(hipMemsetAsync(Y, 0, P3 * sizeof(double2), st));
      HIP_TRY(launch_adjoint_weight(ai, lam + s0.out_off, st));
      for (int pp = 0; pp < 3; ++pp)
        for (int a = 0; a < 3; ++a) {
          int r2;
          if ((r2 = expand3(lam + s0.out_off + pp * s0.n + a * N, ai.M, P, t1, t2, ah, st))) return r2;
          if ((r2 = expand3(E + s0.out_off + pp * s0.n + a * N, ai.M, P, t1, t2, eh, st))) return r2;
          HIP_TRY(launch_conj_mul_acc(ah, eh, Y, P3, st));
        }
      // X_n = (1/P^3) sum_r Y(r) e^{+2 pi i n.r / P}, |n_a| <= 2 M_a (the 1/P^3 is applied at the end)
      HIP_TRY(launch_dft_axis(Y, t1, P * P, P, nc[0], 1, 0, -2 * ai.M[0], P, +1, st));
      HIP_TRY(launch_dft_axis(t1, t2, P, P, nc[1], nc[0], 0, -2 * ai.M[1], P, +1, st));
      HIP_TRY(launch_dft_axis(t2, X, 1, P, nc[2], nc[1] * nc[0], 0, -2 * ai.M[2], P, +1, st));
      // times the exact image of one voxel box, then sum_n e^{-2 pi i n.v / V}
      HIP_TRY(launch_box_factor(X, nc, p->vox, st));
      HIP_TRY(launch_dft_axis(X, t1, nc[2] * nc[1], nc[0], p->vox[0], 1, -2 * ai.M[0], 0, p->vox[0], -1, st));
      HIP_TRY(launch_dft_axis(t1, t2, nc[2], nc[1], p->vox[1], p->vox[0], -2 * ai.M[1], 0, p->vox[1], -1, st));
      HIP_TRY(launch_dft_axis(t2, gv, 1, nc[2], p->vox[2], p->vox[1] * p->vox[0], -2 * ai.M[2], 0, p->vox[2], -1, st));
      HIP_TRY(launch_acc_real(gv, grad_vox, nvox, 2.0 / (double)P3, st));
      HIP_TRY(hipStreamSynchronize(st));
      return GSM_OK;
    };
    rc = run();
    if (rc) return rc;
  }
  int worst = GSM_OK;
  fill_info(sys, exp, info, &worst);
  return worst;
}

}  // extern "C"
