// Host side of the msv C-ABI: validation, geometry, near-panel support nodes,
// pair classification, workspace, and the per-mode factor/solve drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "msv_internal.h"

// Workspace of msv_solve_noalloc: one array per device, held by the process
// for its whole life.  In host code `scratch` names a host-side stand-in, not
// the device memory: host code uses only the per-device address that
// hipGetSymbolAddress returns for it (g_scratch below).
constexpr size_t kScratchBytes = (size_t)192 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

using msv::kOrder;
using cplx = std::complex<double>;

struct msv_plan {
  int N = 0, S = 0, NS = 0, npan = 0, closed = 0, n_self = 0, n_adj = 0;
  int M = 0, L = 0, Mq = 0, Nf = 0, fwd_n = 0;
  double a_min = 0, fwd_lim = 3.0, miller_extra = 20.0, tau = 36.0;
  double k0 = 0, omega = 0;
  cplx k1, eps0, mu0, eps1, mu1;
  int precision = 0;
  int formulation = 0;  // 0: eq. mullerrep, 1: eq. dualmullrep
  double ir_tol = 1e-13;
  int ir_max_iter = 10;
  int last_ir_iters = 0;
  int ir_pred = 0;  // refinement steps of the last converged solve
  std::vector<double> h_r, h_w, h_z, h_dru, h_dzu;  // nodes, weights, dr/du, dz/du
  // sub-panel geometry of msv_fields with upsample = up_U > 1: [5][N U]
  // (r, z, r', z', arclength weight) then the [16 U][16] interpolation matrix
  int up_U = 0;
  double* d_up = nullptr;
  size_t up_bytes = 0;
  // device
  double *d_r = nullptr, *d_z = nullptr, *d_tr = nullptr, *d_tz = nullptr, *d_w = nullptr, *d_sqw = nullptr;
  double *d_sup = nullptr, *d_lag_self = nullptr, *d_lag_adj = nullptr;
  int *d_left = nullptr, *d_right = nullptr;
  uint8_t* d_cls = nullptr;
  int2* d_near = nullptr;
  int n_near = 0;
  double2* d_spec = nullptr;  // Legendre-Q spectra of up to spec_cap near pairs
  int spec_cap = 0;
  double* d_tabs = nullptr;   // azimuth tables of the transforms
  std::vector<int> near_start;  // [N+1]: near pairs of target t are near[near_start[t] ..]
  // factors
  int fac_lo = -1, fac_hi = -1;
  msv_c128* fac_A = nullptr;   // caller's matrices (FP64 factors or FP64 originals)
  float2* d_fac32 = nullptr;   // complex64 factors (precision 1)
  size_t fac32_elems = 0;
  int32_t* d_ipiv = nullptr;
  int32_t* d_info = nullptr;
  int32_t* d_perm = nullptr;   // row permutation of each factor
  void* d_inv = nullptr;       // inverses of the 64 x 64 diagonal blocks of L and U
  size_t inv_bytes = 0;
  void* d_luw = nullptr;       // LU workspace (block inverses, complex64 update planes)
  size_t luw_bytes = 0;
  // extra streams and events of the staggered factorization (created at the
  // first factorization of two or more modes)
  hipStream_t stag_st[msv::kStaggerMax - 1] = {};
  hipEvent_t stag_ev[msv::kStaggerEvents] = {};
  bool stag_ready = false;
  size_t ipiv_elems = 0;
  bool info_checked = false;
  // solve workspace (SolveWork, carved from one allocation)
  void* d_work = nullptr;
  size_t work_bytes = 0;
  // batches that hold raw pointers to this plan's factor storage: while any
  // does, that storage is never reallocated, and a destroy is deferred until
  // the last such batch is destroyed
  size_t geom_bytes = 0;  // device bytes of the geometry uploaded at creation
  int batch_refs = 0;
  bool destroy_pending = false;
  // device address of `scratch` on the plan's device (null if it could not be
  // resolved; scratch_err says why)
  void* scratch = nullptr;
  std::string scratch_err;
  std::string err;
};

static thread_local std::string g_create_err;

// Device memory of the library's own buffers: hipMalloc / hipFree, or the
// caller's pool when one is set (msv_set_allocator).  The hook may change
// only while no plan or batch exists, so every buffer goes back to the
// allocator that gave it.
namespace {
std::mutex g_alloc_mu;
msv_alloc_fn g_alloc = nullptr;
msv_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;
int g_live = 0;  // plans and batches alive (under g_alloc_mu)

hipError_t dev_alloc(void** ptr, size_t bytes) {
  msv_alloc_fn a;
  void* ctx;
  {
    std::lock_guard<std::mutex> l(g_alloc_mu);
    a = g_alloc;
    ctx = g_alloc_ctx;
  }
  if (!a) return hipMalloc(ptr, bytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  *ptr = a(bytes, dev, ctx);
  return *ptr ? hipSuccess : hipErrorOutOfMemory;
}

// hipFree waits for the device.  A buffer given back to a pool inside a
// stream-ordered call (storage regrown for more modes) may still be touched
// by queued work, so the same wait comes first there (wait = true).  A plan
// being destroyed has no work left in flight: with a pool the caller has
// waited for its last call (see msv_set_allocator), and no device-wide wait
// holds up the other streams.
void dev_free(void* ptr, bool wait = true) {
  msv_free_fn f;
  void* ctx;
  {
    std::lock_guard<std::mutex> l(g_alloc_mu);
    f = g_free;
    ctx = g_alloc_ctx;
  }
  if (!f) {
    (void)hipFree(ptr);
    return;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (wait) (void)hipDeviceSynchronize();
  f(ptr, dev, ctx);
}

void live_add(int d) {
  std::lock_guard<std::mutex> l(g_alloc_mu);
  g_live += d;
}
}  // namespace

// Per-device address of `scratch`, resolved once per device with that device
// current.
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

void* scratch_address(std::string& err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}
}  // namespace

namespace {

msv_status fail(msv_plan* p, msv_status st, const std::string& msg) {
  if (p) p->err = msg;
  else g_create_err = msg;
  return st;
}

// Gauss-Legendre nodes (ascending, rounded to double from a long double Newton
// iteration, so that differences of nearby points and nodes are exact) and
// weights.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  auto legendre = [n](long double z, long double& pn, long double& dpn) {
    long double p0 = 1.0L, p1 = z;
    for (int k = 2; k <= n; ++k) {
      long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pn = p1;
    dpn = n * (z * p1 - p0) / (z * z - 1.0L);
  };
  for (int i = 0; i < n; ++i) {
    long double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    long double pn, dpn;
    for (int it = 0; it < 12; ++it) {  // quadratic convergence: far more than enough
      legendre(z, pn, dpn);
      z -= pn / dpn;
    }
    legendre(z, pn, dpn);
    x[n - 1 - i] = (double)z;
    w[n - 1 - i] = (double)(2.0L / ((1.0L - z * z) * dpn * dpn));
  }
}

// Lagrange basis values l_k(y) on nodes xn (barycentric form).
void lagrange_row(const std::vector<double>& xn, const std::vector<double>& bw, double y, double* out) {
  const int n = (int)xn.size();
  for (int k = 0; k < n; ++k)
    if (y == xn[k]) {
      for (int j = 0; j < n; ++j) out[j] = (j == k) ? 1.0 : 0.0;
      return;
    }
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    out[k] = bw[k] / (y - xn[k]);
    s += out[k];
  }
  for (int k = 0; k < n; ++k) out[k] /= s;
}

template <typename T>
msv_status upload(msv_plan* p, T** dst, const T* src, size_t count) {
  if (count == 0) return MSV_OK;
  if (dev_alloc((void**)dst, sizeof(T) * count) != hipSuccess) return fail(p, MSV_ENOMEM, "hipMalloc failed");
  p->geom_bytes += sizeof(T) * count;
  if (hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice) != hipSuccess)
    return fail(p, MSV_EHIP, "hipMemcpy failed");
  return MSV_OK;
}

#define MSV_CHECK(x)                    \
  do {                                  \
    msv_status st_ = (x);               \
    if (st_ != MSV_OK) return st_;      \
  } while (0)

#define MSV_HIP(p, x)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return fail(p, MSV_EHIP, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

// Azimuthal bandwidth of the analytic factors: smallest j with
// (x/2)^(2j) / (2j)! <= 1e-16, x = 2 max|k| r_max (bound on J_{2j}(x)).
int bandwidth(double kmax, double rmax) {
  double x = 2.0 * kmax * rmax;
  for (int j = 1;; ++j) {
    double nu = 2.0 * j;
    double lb = nu * std::log(std::max(x, 1e-300) / 2.0) - std::lgamma(nu + 1.0);
    if (lb <= std::log(1e-16)) return j;
  }
}

}  // namespace

extern "C" {

msv_status msv_set_allocator(msv_alloc_fn alloc, msv_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) return fail(nullptr, MSV_EINVAL, "give both hooks or neither");
  std::lock_guard<std::mutex> l(g_alloc_mu);
  if (g_live > 0) return fail(nullptr, MSV_EINVAL, "plans or batches exist: destroy them first");
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_ctx = alloc ? ctx : nullptr;
  return MSV_OK;
}

const char* msv_last_error(const msv_plan* p) { return p ? p->err.c_str() : g_create_err.c_str(); }
int32_t msv_num_nodes(const msv_plan* p) { return p ? p->N : 0; }
int32_t msv_num_support(const msv_plan* p) { return p ? p->S : 0; }
int32_t msv_matrix_order(const msv_plan* p) { return p ? 4 * p->N : 0; }
int32_t msv_last_ir_iterations(const msv_plan* p) { return p ? p->last_ir_iters : 0; }
size_t msv_table_entries(const msv_plan* p) {
  return p ? (size_t)(p->M + 2) * msv::kTypes * p->N * p->NS : 0;
}

static void plan_free(msv_plan* p) {
  void* bufs[] = {p->d_r, p->d_z, p->d_tr, p->d_tz, p->d_w, p->d_sqw, p->d_sup, p->d_lag_self,
                  p->d_lag_adj, p->d_left, p->d_right, p->d_cls, p->d_near, p->d_fac32, p->d_ipiv,
                  p->d_info, p->d_perm, p->d_inv, p->d_luw, p->d_work, p->d_spec, p->d_tabs, p->d_up};
  for (void* b : bufs)
    if (b) dev_free(b, false);
  for (hipEvent_t e : p->stag_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipStream_t q : p->stag_st)
    if (q) (void)hipStreamDestroy(q);
  delete p;
  live_add(-1);
}

// Device bytes of the factor storage for nb modes of order n.
static size_t factor_bytes(int n, int nb, int precision) {
  const size_t nn = (size_t)n * n;
  return (size_t)nb * n * 2 * sizeof(int32_t) + (size_t)nb * sizeof(int32_t) +
         msv::lu_work_bytes(n, nb, precision == 0) + (precision == 1 ? (size_t)nb * nn * sizeof(float2) : 0) +
         (size_t)nb * ((n + 63) / 64) * 2 * 64 * 64 * (precision == 0 ? 16 : 8);
}
// Device bytes of the solve workspace for `vectors` vectors of order n in nvb
// batches, laid out as SolveWork, each part 256-byte aligned.
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }
static size_t solve_work_bytes(size_t n, size_t vectors, size_t nvb, int precision) {
  const size_t elems = vectors * n;
  return 3 * align256(sizeof(double2) * elems) + (precision == 1 ? 2 * align256(sizeof(float2) * elems) : 0) +
         align256(sizeof(double) * (vectors + 1)) + align256(sizeof(msv::VecBatch) * nvb);
}

size_t msv_workspace_bytes(int32_t n_nodes, int32_t n_support, int32_t fft_len, int32_t n_modes,
                           int32_t n_solve_vectors, int32_t precision) {
  if (n_nodes < 1 || n_support < 0 || fft_len < 8 || fft_len > 1024 || n_modes < 1 || n_solve_vectors < 0 ||
      (precision != 0 && precision != 1))
    return 0;
  const size_t N = n_nodes, S = n_support, NS = N + S, n = 4 * N;
  // geometry: 6 node arrays, support records, Lagrange rows (bounded by the
  // slot count), neighbour lists, pair classes, near-pair list and the
  // near pairs' spectra scratch (at most every pair near)
  const int near_max = (int)std::min<size_t>(N * NS, (size_t)1 << 30);
  size_t b = 6 * N * sizeof(double) + N * S * msv::kSupFields * sizeof(double) +
             (size_t)kOrder * kOrder * S * sizeof(double) + kOrder * S * sizeof(double) +
             2 * (N / kOrder) * sizeof(int) + N * NS + N * NS * sizeof(int2) + msv::spec_bytes(fft_len, near_max) +
             msv::tab_doubles(fft_len) * sizeof(double);
  b += factor_bytes((int)n, n_modes, precision);
  if (n_solve_vectors > 0)
    b += solve_work_bytes(n, n_solve_vectors, (size_t)n_modes + (n_solve_vectors + msv::kVB - 1) / msv::kVB,
                          precision);
  return b;
}

size_t msv_plan_device_bytes(const msv_plan* p) {
  if (!p) return 0;
  const size_t n = 4 * (size_t)p->N;
  size_t b = p->geom_bytes;
  const size_t nbf = p->ipiv_elems / n;  // modes of the pivot storage
  b += p->ipiv_elems * 2 * sizeof(int32_t) + nbf * sizeof(int32_t) + p->luw_bytes + p->fac32_elems * sizeof(float2) +
       p->inv_bytes;
  b += p->work_bytes + p->up_bytes;
  return b;
}

void msv_plan_destroy(msv_plan* p) {
  if (!p) return;
  if (p->batch_refs > 0) {
    p->destroy_pending = true;  // freed by the last msv_batch_destroy that holds it
    return;
  }
  plan_free(p);
}

msv_status msv_plan_create(msv_plan** out, const msv_curve* c, const msv_rules* ru, const msv_desc* d,
                           void* stream) {
  g_create_err.clear();
  if (!out || !c || !ru || !d) return fail(nullptr, MSV_EINVAL, "null argument");
  *out = nullptr;
  if (c->order != kOrder) return fail(nullptr, MSV_EINVAL, "order must be 16");
  if (c->n_panels < 1 || (c->closed && c->n_panels < 3))
    return fail(nullptr, MSV_EINVAL, "need >= 1 panel (>= 3 for a closed curve)");
  if (!c->h_r || !c->h_z || !c->h_nr || !c->h_nz || !c->h_dsdu)
    return fail(nullptr, MSV_EINVAL, "curve arrays missing");
  if (ru->n_self < 1 || ru->n_adj < 1 || !ru->h_self_u || !ru->h_self_w || !ru->h_adj_u || !ru->h_adj_w)
    return fail(nullptr, MSV_EINVAL, "rules missing");
  if (!(d->k0 > 0.0)) return fail(nullptr, MSV_EINVAL, "k0 must be > 0");
  if (!(d->eps0.re > 0 && d->eps0.im == 0 && d->mu0.re > 0 && d->mu0.im == 0))
    return fail(nullptr, MSV_EINVAL, "eps0, mu0 must be real and positive");
  if (!(d->eps1.re > 0 && d->eps1.im >= 0 && d->mu1.re > 0 && d->mu1.im >= 0))
    return fail(nullptr, MSV_EINVAL, "need Re eps1, Re mu1 > 0 and Im eps1, Im mu1 >= 0");
  if (d->m_max < 0) return fail(nullptr, MSV_EINVAL, "m_max must be >= 0");
  if (d->fft_len < 8 || d->fft_len > 1024 || (d->fft_len & (d->fft_len - 1)))
    return fail(nullptr, MSV_EINVAL, "fft_len must be a power of two in [8, 1024]");
  if (d->precision != 0 && d->precision != 1) return fail(nullptr, MSV_EINVAL, "precision must be 0 or 1");
  if (d->formulation != 0 && d->formulation != 1) return fail(nullptr, MSV_EINVAL, "formulation must be 0 or 1");
  const int N = c->n_panels * kOrder;
  if (4 * N > 12288) return fail(nullptr, MSV_EINVAL, "4N > 12288 exceeds the LU panel kernel");
  for (int i = 0; i < N; ++i) {
    if (!(c->h_r[i] > 0.0)) return fail(nullptr, MSV_EINVAL, "r must be > 0 at every node");
    if (!(c->h_dsdu[i] > 0.0)) return fail(nullptr, MSV_EINVAL, "ds/du must be > 0");
    double nn = std::hypot(c->h_nr[i], c->h_nz[i]);
    if (std::fabs(nn - 1.0) > 1e-12) return fail(nullptr, MSV_EINVAL, "normals must have unit length");
  }

  msv_plan* p = new msv_plan();
  live_add(1);
  p->N = N;
  p->npan = c->n_panels;
  p->closed = c->closed ? 1 : 0;
  p->n_self = ru->n_self;
  p->n_adj = ru->n_adj;
  p->S = ru->n_self + 2 * ru->n_adj;
  p->NS = N + p->S;
  p->M = d->m_max;
  p->L = d->fft_len;
  p->Mq = p->L / 2 - 1;
  p->k0 = d->k0;
  p->eps0 = cplx(d->eps0.re, d->eps0.im);
  p->mu0 = cplx(d->mu0.re, d->mu0.im);
  p->eps1 = cplx(d->eps1.re, d->eps1.im);
  p->mu1 = cplx(d->mu1.re, d->mu1.im);
  p->omega = d->k0 / std::sqrt(d->eps0.re * d->mu0.re);
  p->k1 = p->omega * std::sqrt(p->eps1 * p->mu1);
  if (p->k1.imag() < 0) p->k1 = -p->k1;
  p->precision = d->precision;
  p->formulation = d->formulation;
  p->ir_tol = d->ir_tol > 0 ? d->ir_tol : 1e-13;
  p->ir_max_iter = d->ir_max_iter > 0 ? d->ir_max_iter : 10;

  // geometry: arclength weights, tangents, panel lengths, neighbours
  std::vector<double> ug, wg;
  gauss_legendre(kOrder, ug, wg);
  std::vector<double> bw(kOrder, 1.0);
  for (int j = 0; j < kOrder; ++j)
    for (int k = 0; k < kOrder; ++k)
      if (k != j) bw[j] /= (ug[j] - ug[k]);
  std::vector<double> w(N), sqw(N), tr(N), tz(N), plen(p->npan, 0.0);
  double rmax = 0.0;
  for (int i = 0; i < N; ++i) {
    w[i] = wg[i % kOrder] * c->h_dsdu[i];
    sqw[i] = std::sqrt(w[i]);
    tr[i] = -c->h_nz[i];
    tz[i] = c->h_nr[i];
    plen[i / kOrder] += w[i];
    rmax = std::max(rmax, c->h_r[i]);
  }
  std::vector<int> left(p->npan), right(p->npan);
  for (int q = 0; q < p->npan; ++q) {
    left[q] = q - 1;
    right[q] = q + 1;
  }
  if (p->closed) {
    left[0] = p->npan - 1;
    right[p->npan - 1] = 0;
  } else {
    left[0] = -1;
    right[p->npan - 1] = -1;
  }
  for (int q = 0; q < p->npan; ++q)
    for (int nb : {left[q], right[q]})
      if (nb >= 0) {
        double ratio = plen[nb] / plen[q];
        if (ratio > 2.2 || ratio < 1.0 / 2.2) {
          msv_plan_destroy(p);
          return fail(nullptr, MSV_EINVAL, "adjacent panels differ in length by more than 2.2x");
        }
      }
  // kernel parameters (classification and recurrences)
  p->Nf = bandwidth(std::max(p->k0, std::abs(p->k1)), rmax);
  const int m_hi = p->M + 1;
  if (m_hi + p->Nf > p->Mq) {
    char buf[200];
    snprintf(buf, sizeof buf, "fft_len %d too short: need M+1+N_f = %d <= L/2-1 = %d", p->L, m_hi + p->Nf, p->Mq);
    msv_plan_destroy(p);
    return fail(nullptr, MSV_EINVAL, buf);
  }
  p->a_min = p->tau / (double)(p->L - m_hi - p->Nf);
  p->fwd_n = m_hi + p->Nf;

  // support slots: offsets from the target (interpolated nodal differences),
  // source geometry and weights
  const int S = p->S, NSf = msv::kSupFields;
  std::vector<double> sup((size_t)N * S * NSf, 0.0);
  std::vector<double> lag_self((size_t)kOrder * p->n_self * kOrder), lag_adj((size_t)p->n_adj * kOrder);
  for (int k = 0; k < kOrder; ++k)
    for (int q = 0; q < p->n_self; ++q)
      lagrange_row(ug, bw, ru->h_self_u[k * p->n_self + q], &lag_self[((size_t)k * p->n_self + q) * kOrder]);
  for (int q = 0; q < p->n_adj; ++q) lagrange_row(ug, bw, ru->h_adj_u[q], &lag_adj[(size_t)q * kOrder]);
  // Offsets r_s - r_t, z_s - z_t in long double: near the axis the z offset
  // can be far smaller than the distance, and in double it would keep only
  // about 12 digits.  Own panel: (y - u_t) Q(y) with Q interpolating the
  // divided differences (x_k - x_t)/(u_k - u_t) on the other 15 nodes, so
  // nothing cancels as y -> u_t (y - u_t itself is exact).
  typedef long double ld;
  std::vector<ld> bw16(kOrder, 1.0L), bw15((size_t)kOrder * kOrder, 0.0L);
  for (int j = 0; j < kOrder; ++j)
    for (int k = 0; k < kOrder; ++k)
      if (k != j) bw16[j] /= ((ld)ug[j] - (ld)ug[k]);
  for (int kt = 0; kt < kOrder; ++kt)
    for (int j = 0; j < kOrder; ++j) {
      if (j == kt) continue;
      ld b = 1.0L;
      for (int k = 0; k < kOrder; ++k)
        if (k != j && k != kt) b /= ((ld)ug[j] - (ld)ug[k]);
      bw15[kt * kOrder + j] = b;
    }
  // sum_k c_k l_k(y) in barycentric (second) form over nodes k != skip
  auto interp = [&](const ld* bw, int skip, double y, const ld* cr, const ld* cz, ld& outr, ld& outz) {
    ld nr = 0, nz = 0, den = 0;
    for (int k = 0; k < kOrder; ++k) {
      if (k == skip) continue;
      if (y == ug[k]) {
        outr = cr[k];
        outz = cz[k];
        return;
      }
      ld b = bw[k] / ((ld)y - (ld)ug[k]);
      nr += b * cr[k];
      nz += b * cz[k];
      den += b;
    }
    outr = nr / den;
    outz = nz / den;
  };
  auto fill = [&](int t, int slot0, int pan, int nq, const double* lagrows, const double* wts,
                  const double* u) {
    const double* rp = c->h_r + pan * kOrder;
    const double* zp = c->h_z + pan * kOrder;
    const bool own = pan == t / kOrder;
    const int kt = t % kOrder;
    ld cr[kOrder], cz[kOrder];
    for (int k = 0; k < kOrder; ++k) {
      cr[k] = (ld)rp[k] - (ld)c->h_r[t];
      cz[k] = (ld)zp[k] - (ld)c->h_z[t];
      if (own && k != kt) {
        ld du = (ld)ug[k] - (ld)ug[kt];
        cr[k] /= du;
        cz[k] /= du;
      }
    }
    for (int q = 0; q < nq; ++q) {
      const double* l = lagrows + (size_t)q * kOrder;
      double r = 0, drdu = 0, dzdu = 0;
      for (int k = 0; k < kOrder; ++k) {
        int j = pan * kOrder + k;
        r += l[k] * rp[k];
        drdu += l[k] * (-c->h_nz[j] * c->h_dsdu[j]);
        dzdu += l[k] * (c->h_nr[j] * c->h_dsdu[j]);
      }
      ld dr, dz;
      if (own) {
        interp(&bw15[kt * kOrder], kt, u[q], cr, cz, dr, dz);
        ld yu = (ld)u[q] - (ld)ug[kt];
        dr *= yu;
        dz *= yu;
      } else {
        interp(bw16.data(), -1, u[q], cr, cz, dr, dz);
      }
      double sp = std::hypot(drdu, dzdu);
      double* o = &sup[((size_t)t * S + slot0 + q) * NSf];
      o[msv::kSupDr] = (double)dr;
      o[msv::kSupDz] = (double)dz;
      o[msv::kSupR] = r;
      o[msv::kSupTr] = drdu / sp;
      o[msv::kSupTz] = dzdu / sp;
      o[msv::kSupW] = wts[q] * sp;
    }
  };
  for (int t = 0; t < N; ++t) {
    int pan = t / kOrder, k = t % kOrder;
    fill(t, 0, pan, p->n_self, &lag_self[(size_t)k * p->n_self * kOrder], ru->h_self_w + k * p->n_self,
         ru->h_self_u + k * p->n_self);
    if (left[pan] >= 0)
      fill(t, p->n_self, left[pan], p->n_adj, lag_adj.data(), ru->h_adj_w, ru->h_adj_u);
    if (right[pan] >= 0)
      fill(t, p->n_self + p->n_adj, right[pan], p->n_adj, lag_adj.data(), ru->h_adj_w, ru->h_adj_u);
  }
  // pair classes: near iff acosh(chi) < a_min (split + convolution), else the
  // plain L-point trapezoid; coincident pairs and unused slots are zero
  std::vector<uint8_t> cls((size_t)N * p->NS);
  std::vector<int2> nearv;
  for (int t = 0; t < N; ++t) {
    const double rt = c->h_r[t];
    for (int col = 0; col < p->NS; ++col) {
      double dr, dz;
      uint8_t cl;
      if (col < N) {
        dr = c->h_r[col] - rt;
        dz = c->h_z[col] - c->h_z[t];
        if (col == t) {
          cls[(size_t)t * p->NS + col] = msv::kZero;
          continue;
        }
      } else {
        const double* o = &sup[((size_t)t * S + (col - N)) * NSf];
        if (o[msv::kSupW] == 0.0) {
          cls[(size_t)t * p->NS + col] = msv::kZero;
          continue;
        }
        dr = o[msv::kSupDr];
        dz = o[msv::kSupDz];
      }
      double rs = rt + dr;
      double eta = (dr * dr + dz * dz) / (2.0 * rt * rs);
      double ach = std::log1p(eta + std::sqrt(eta * (2.0 + eta)));
      cl = ach < p->a_min ? msv::kNear : msv::kFar;
      if (eta == 0.0) cl = msv::kZero;
      cls[(size_t)t * p->NS + col] = cl;
      if (cl == msv::kNear) nearv.push_back(make_int2(t, col));
    }
  }
  p->n_near = (int)nearv.size();
  p->near_start.assign(N + 1, 0);
  for (const int2& pr : nearv) p->near_start[pr.x + 1]++;
  for (int t = 0; t < N; ++t) p->near_start[t + 1] += p->near_start[t];
  p->h_r.assign(c->h_r, c->h_r + N);
  p->h_w = w;
  p->h_z.assign(c->h_z, c->h_z + N);
  p->h_dru.resize(N);
  p->h_dzu.resize(N);
  for (int i = 0; i < N; ++i) {
    p->h_dru[i] = tr[i] * c->h_dsdu[i];
    p->h_dzu[i] = tz[i] * c->h_dsdu[i];
  }

  msv_status st;
#define UP(dst, vec) \
  if ((st = upload(p, &dst, vec.data(), vec.size())) != MSV_OK) { msv_plan_destroy(p); return st; }
  std::vector<double> vr(c->h_r, c->h_r + N), vz(c->h_z, c->h_z + N);
  UP(p->d_r, vr);
  UP(p->d_z, vz);
  UP(p->d_tr, tr);
  UP(p->d_tz, tz);
  UP(p->d_w, w);
  UP(p->d_sqw, sqw);
  UP(p->d_sup, sup);
  UP(p->d_lag_self, lag_self);
  UP(p->d_lag_adj, lag_adj);
  UP(p->d_left, left);
  UP(p->d_right, right);
  UP(p->d_cls, cls);
  UP(p->d_near, nearv);
#undef UP
  {
    // azimuth tables (long double, rounded once): e^{-2 pi i k / L},
    // (cos, sin)(2 pi j / L), sin^2(pi j / L)
    const int Nh = p->L / 2;
    std::vector<double> tabs(msv::tab_doubles(p->L), 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < Nh; ++k) {
      tabs[2 * k] = (double)std::cos(pi * k / Nh);
      tabs[2 * k + 1] = (double)-std::sin(pi * k / Nh);
    }
    double* cs = tabs.data() + 2 * Nh;
    for (int j = 0; j <= Nh / 2; ++j) {
      cs[2 * j] = (double)std::cos(pi * j / Nh);
      cs[2 * j + 1] = (double)std::sin(pi * j / Nh);
    }
    double* s2 = cs + 2 * (Nh / 2 + 1);
    for (int j = 0; j <= Nh; ++j) {
      const long double sn = std::sin(pi * j / (2 * Nh));
      s2[j] = (double)(sn * sn);
    }
    msv_status st2 = upload(p, &p->d_tabs, tabs.data(), tabs.size());
    if (st2 != MSV_OK) {
      msv_plan_destroy(p);
      return st2;
    }
  }
  p->spec_cap = std::min(p->n_near, msv::kSpecCap);
  if (p->spec_cap > 0) {
    const size_t sb = msv::spec_bytes(p->L, p->n_near);
    if (dev_alloc((void**)&p->d_spec, sb) != hipSuccess) {
      msv_plan_destroy(p);
      return fail(nullptr, MSV_ENOMEM, "spectra scratch allocation failed");
    }
    p->geom_bytes += sb;
  }
  // set-up of the allocation-free solve's workspace on this device
  p->scratch = scratch_address(p->scratch_err);
  (void)stream;
  *out = p;
  return MSV_OK;
}

msv_status msv_tabulate_rows(msv_plan* p, int32_t t0, int32_t nt, msv_c128* d_kern, size_t kern_elems,
                             void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  if (!d_kern) return fail(p, MSV_EINVAL, "null table");
  if (t0 < 0 || nt < 1 || t0 + nt > p->N) return fail(p, MSV_EINVAL, "need 0 <= t0, 1 <= nt, t0 + nt <= N");
  if (kern_elems != (size_t)(p->M + 2) * msv::kTypes * nt * p->NS)
    return fail(p, MSV_EINVAL, "table size mismatch");
  msv::TabParams T{};
  T.N = p->N;
  T.S = p->S;
  T.NS = p->NS;
  T.M2 = p->M + 2;
  T.L = p->L;
  T.Mq = p->Mq;
  T.fwd_n = p->fwd_n;
  T.fwd_lim = p->fwd_lim;
  T.miller_extra = p->miller_extra;
  T.k0 = p->k0;
  T.k1r = p->k1.real();
  T.k1i = p->k1.imag();
  T.r = p->d_r;
  T.z = p->d_z;
  T.sup = p->d_sup;
  T.cls = p->d_cls;
  T.near = p->d_near;
  T.n_near = p->n_near;
  T.t0 = t0;
  T.nt = nt;
  T.near_lo = p->near_start[t0];
  T.near_hi = p->near_start[t0 + nt];
  T.spec = p->d_spec;
  T.spec_cap = p->spec_cap;
  T.tabs = reinterpret_cast<const double2*>(p->d_tabs);
  T.out = reinterpret_cast<double2*>(d_kern);
  MSV_HIP(p, msv::launch_tabulate(T, (hipStream_t)stream));
  return MSV_OK;
}

msv_status msv_tabulate(msv_plan* p, msv_c128* d_kern, size_t kern_elems, void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  return msv_tabulate_rows(p, 0, p->N, d_kern, kern_elems, stream);
}

msv_status msv_assemble_rows(msv_plan* p, const msv_c128* d_kern, int32_t t0, int32_t nt, int32_t m_lo,
                             int32_t m_hi, msv_c128* d_A, void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  if (!d_kern || !d_A) return fail(p, MSV_EINVAL, "null buffer");
  if (m_lo < 0 || m_hi < m_lo || m_hi > p->M) return fail(p, MSV_EINVAL, "need 0 <= m_lo <= m_hi <= M");
  if (t0 < 0 || nt < 1 || t0 + nt > p->N) return fail(p, MSV_EINVAL, "need 0 <= t0, 1 <= nt, t0 + nt <= N");
  msv::AsmParams A{};
  A.t0 = t0;
  A.nt = nt;
  A.N = p->N;
  A.S = p->S;
  A.NS = p->NS;
  A.M2 = p->M + 2;
  A.npan = p->npan;
  A.n_self = p->n_self;
  A.n_adj = p->n_adj;
  A.m_lo = m_lo;
  A.m_hi = m_hi;
  A.k0 = p->k0;
  A.k1r = p->k1.real();
  A.k1i = p->k1.imag();
  A.omega = p->omega;
  A.eps0r = p->eps0.real();
  A.eps0i = p->eps0.imag();
  A.mu0r = p->mu0.real();
  A.mu0i = p->mu0.imag();
  A.eps1r = p->eps1.real();
  A.eps1i = p->eps1.imag();
  A.mu1r = p->mu1.real();
  A.mu1i = p->mu1.imag();
  A.formulation = p->formulation;
  A.r = p->d_r;
  A.tr = p->d_tr;
  A.tz = p->d_tz;
  A.w = p->d_w;
  A.sqw = p->d_sqw;
  A.sup = p->d_sup;
  A.left = p->d_left;
  A.right = p->d_right;
  A.lag_self = p->d_lag_self;
  A.lag_adj = p->d_lag_adj;
  A.kern = reinterpret_cast<const double2*>(d_kern);
  A.A = reinterpret_cast<double2*>(d_A);
  MSV_HIP(p, msv::launch_assemble(A, (hipStream_t)stream));
  return MSV_OK;
}

msv_status msv_assemble(msv_plan* p, const msv_c128* d_kern, int32_t m_lo, int32_t m_hi, msv_c128* d_A,
                        void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  return msv_assemble_rows(p, d_kern, 0, p->N, m_lo, m_hi, d_A, stream);
}

// Factor nb matrices (complex128 at A64 or complex64 at A32) on s.
// The extra streams and events of the staggered factorization, created once
// per plan on the current device.
static hipError_t stagger_init(msv_plan* p) {
  if (p->stag_ready) return hipSuccess;
  hipError_t e = hipSuccess;
  for (int i = 0; i + 1 < msv::kLuGroups && e == hipSuccess; ++i)
    if (!p->stag_st[i]) e = hipStreamCreateWithFlags(&p->stag_st[i], hipStreamNonBlocking);
  for (int i = 0; i < msv::kStaggerEvents && e == hipSuccess; ++i)
    if (!p->stag_ev[i]) e = hipEventCreateWithFlags(&p->stag_ev[i], hipEventDisableTiming);
  p->stag_ready = e == hipSuccess;
  return e;
}

// Every mode's matrix is factored by the same launches; two or more modes of
// an order of at least kStaggerMinOrder are cut into kLuGroups groups on as
// many streams, staggered by panel phases.
static hipError_t factor_groups(msv_plan* p, msv_c128* A64, float2* A32, int n, int nb, hipStream_t s) {
  msv::LuBatch b{n, nb, n, (long long)n * n};
  if (nb >= 2 && msv::kLuGroups >= 2 && n >= msv::kStaggerMinOrder) {
    hipError_t e = stagger_init(p);
    if (e != hipSuccess) return e;
    hipStream_t st[msv::kStaggerMax] = {s};
    for (int i = 0; i + 1 < msv::kLuGroups; ++i) st[i + 1] = p->stag_st[i];
    return A64 ? msv::lu_factor_staggered_z(reinterpret_cast<double2*>(A64), p->d_ipiv, p->d_info, b, p->d_luw,
                                            msv::kLuGroups, st, p->stag_ev)
               : msv::lu_factor_staggered_c(A32, p->d_ipiv, p->d_info, b, p->d_luw, msv::kLuGroups, st, p->stag_ev);
  }
  return A64 ? msv::lu_factor_z(reinterpret_cast<double2*>(A64), p->d_ipiv, p->d_info, b, p->d_luw, s)
             : msv::lu_factor_c(A32, p->d_ipiv, p->d_info, b, p->d_luw, s);
}

// Factor storage of modes m_lo .. m_lo + nb - 1: pivots, permutations, info
// flags, LU workspace, complex64 factors (precision 1), block inverses.
static msv_status factor_buffers(msv_plan* p, int n, int nb) {
  const size_t nn = (size_t)n * n;
  if (p->batch_refs > 0) {
    // a batch's captured launches and matrix list point into this storage
    const size_t inv_need = (size_t)nb * ((n + 63) / 64) * 2 * 64 * 64 * (p->precision == 0 ? 16 : 8);
    if ((size_t)nb * n > p->ipiv_elems || msv::lu_work_bytes(n, nb, p->precision == 0) > p->luw_bytes ||
        (p->precision == 1 && (size_t)nb * nn > p->fac32_elems) || inv_need > p->inv_bytes)
      return fail(p, MSV_EINVAL, "the plan is held by a batch: factor at most the batch's mode count");
    return MSV_OK;
  }
  if ((size_t)nb * n > p->ipiv_elems) {
    if (p->d_ipiv) dev_free(p->d_ipiv);
    if (p->d_info) dev_free(p->d_info);
    if (p->d_perm) dev_free(p->d_perm);
    p->d_ipiv = nullptr;
    p->d_info = nullptr;
    p->d_perm = nullptr;
    p->ipiv_elems = 0;
    if (dev_alloc((void**)&p->d_ipiv, sizeof(int32_t) * (size_t)nb * n) != hipSuccess ||
        dev_alloc((void**)&p->d_perm, sizeof(int32_t) * (size_t)nb * n) != hipSuccess ||
        dev_alloc((void**)&p->d_info, sizeof(int32_t) * nb) != hipSuccess)
      return fail(p, MSV_ENOMEM, "pivot allocation failed");
    p->ipiv_elems = (size_t)nb * n;
  }
  const size_t luw_bytes = msv::lu_work_bytes(n, nb, p->precision == 0);
  if (luw_bytes > p->luw_bytes) {
    if (p->d_luw) dev_free(p->d_luw);
    p->d_luw = nullptr;
    p->luw_bytes = 0;
    if (dev_alloc((void**)&p->d_luw, luw_bytes) != hipSuccess) return fail(p, MSV_ENOMEM, "LU workspace allocation failed");
    p->luw_bytes = luw_bytes;
  }
  if (p->precision == 1 && (size_t)nb * nn > p->fac32_elems) {
    if (p->d_fac32) dev_free(p->d_fac32);
    p->d_fac32 = nullptr;
    p->fac32_elems = 0;
    if (dev_alloc((void**)&p->d_fac32, sizeof(float2) * (size_t)nb * nn) != hipSuccess)
      return fail(p, MSV_ENOMEM, "complex64 factor allocation failed");
    p->fac32_elems = (size_t)nb * nn;
  }
  const size_t inv_bytes = (size_t)nb * ((n + 63) / 64) * 2 * 64 * 64 * (p->precision == 0 ? 16 : 8);
  if (inv_bytes > p->inv_bytes) {
    if (p->d_inv) dev_free(p->d_inv);
    p->d_inv = nullptr;
    p->inv_bytes = 0;
    if (dev_alloc((void**)&p->d_inv, inv_bytes) != hipSuccess) return fail(p, MSV_ENOMEM, "block inverse allocation failed");
    p->inv_bytes = inv_bytes;
  }
  return MSV_OK;
}

// After the LU: row permutations, diagonal-block inverses, bookkeeping.
static msv_status factor_finish(msv_plan* p, msv_c128* d_A, int m_lo, int m_hi, hipStream_t s) {
  const int n = 4 * p->N, nb = m_hi - m_lo + 1;
  const long long nn = (long long)n * n;
  MSV_HIP(p, msv::lu_perm(p->d_ipiv, p->d_perm, n, nb, s));
  if (p->precision == 0)
    MSV_HIP(p, msv::lu_inv_diag_z(reinterpret_cast<const double2*>(d_A), nn, n, nb, static_cast<double2*>(p->d_inv), s));
  else
    MSV_HIP(p, msv::lu_inv_diag_c(p->d_fac32, nn, n, nb, static_cast<float2*>(p->d_inv), s));
  p->fac_lo = m_lo;
  p->fac_hi = m_hi;
  p->fac_A = d_A;
  p->info_checked = false;
  return MSV_OK;
}

msv_status msv_factor(msv_plan* p, msv_c128* d_A, int32_t m_lo, int32_t m_hi, void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  if (!d_A) return fail(p, MSV_EINVAL, "null matrix buffer");
  if (m_lo < 0 || m_hi < m_lo || m_hi > p->M) return fail(p, MSV_EINVAL, "need 0 <= m_lo <= m_hi <= M");
  hipStream_t s = (hipStream_t)stream;
  const int n = 4 * p->N, nb = m_hi - m_lo + 1;
  const size_t nn = (size_t)n * n;
  msv_status st = factor_buffers(p, n, nb);
  if (st != MSV_OK) return st;
  if (p->precision == 0) {
    MSV_HIP(p, factor_groups(p, d_A, nullptr, n, nb, s));
  } else {
    MSV_HIP(p, msv::conv_c64(reinterpret_cast<const double2*>(d_A), p->d_fac32, (size_t)nb * nn, s));
    MSV_HIP(p, factor_groups(p, nullptr, p->d_fac32, n, nb, s));
  }
  return factor_finish(p, d_A, m_lo, m_hi, s);
}

// ---------------------------------------------------------------------------
// Batching form: the modes of several bodies factored by the same launches
// (a listed batch of matrices of different orders), the launch sequence
// captured once in a HIP graph and replayed; the outer panel width is picked
// at creation by timing both candidates on the batch itself.
// ---------------------------------------------------------------------------
struct msv_batch {
  std::vector<msv_plan*> plans;
  std::vector<msv_c128*> A;
  int m_lo = 0, m_hi = 0;
  int nb = 0, nmax = 0;
  msv::LuMat* d_list = nullptr;
  void* d_work = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool pinned = false;  // holds a reference on every plan
  int panel = 128;
  int plane_min = 256;
  float tuned_ms[4] = {-1.f, -1.f, -1.f, -1.f};   // panel 64, 128, 256, 512 (plane_min 256)
  float tuned_plane_ms[3] = {-1.f, -1.f, -1.f};   // plane_min 256, 512, 1024 (the chosen panel)
  bool from_table = false;
  std::string err;
};

// Tuned (panel, plane_min) per size class: device, largest order and matrix
// count rounded up to powers of two, and which panel widths the orders allow.
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tune;
int ceil_log2(long long v) {
  int l = 0;
  while ((1LL << l) < v) ++l;
  return l;
}
}  // namespace

static thread_local std::string g_batch_err;

static msv_status batch_fail(msv_batch* b, msv_status st, const std::string& msg) {
  if (b) b->err = msg;
  else g_batch_err = msg;
  return st;
}

// The launch sequence of one batched factorization, on stream s.
static hipError_t batch_sequence(msv_batch* b, int panel, int plane_min, hipStream_t s) {
  hipError_t e;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    msv_plan* p = b->plans[i];
    const size_t n = 4 * (size_t)p->N, cnt = (size_t)(b->m_hi - b->m_lo + 1) * n * n;
    if ((e = msv::conv_c64(reinterpret_cast<const double2*>(b->A[i]), p->d_fac32, cnt, s)) != hipSuccess) return e;
  }
  if ((e = msv::lu_factor_list_c(b->d_list, b->nb, b->nmax, panel, plane_min, b->d_work, s)) != hipSuccess) return e;
  const int nbp = b->m_hi - b->m_lo + 1;
  for (msv_plan* p : b->plans) {
    const int n = 4 * p->N;
    if ((e = msv::lu_perm(p->d_ipiv, p->d_perm, n, nbp, s)) != hipSuccess) return e;
    if ((e = msv::lu_inv_diag_c(p->d_fac32, (long long)n * n, n, nbp, static_cast<float2*>(p->d_inv), s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

static hipError_t batch_capture(msv_batch* b, int panel, int plane_min, hipGraph_t* g, hipGraphExec_t* x) {
  hipError_t e = hipStreamBeginCapture(b->st, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  hipError_t e2 = batch_sequence(b, panel, plane_min, b->st);
  e = hipStreamEndCapture(b->st, g);
  if (e2 != hipSuccess) return e2;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(x, *g, nullptr, nullptr, 0);
}

void msv_batch_destroy(msv_batch* b) {
  if (!b) return;
  if (b->pinned) {
    (void)hipStreamSynchronize(b->st);  // a replay may still read the plans' storage
    for (msv_plan* p : b->plans)
      if (--p->batch_refs == 0 && p->destroy_pending) plan_free(p);
  }
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_list) dev_free(b->d_list);
  if (b->d_work) dev_free(b->d_work);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
  live_add(-1);
}

const char* msv_batch_last_error(const msv_batch* b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

int32_t msv_batch_panel(const msv_batch* b) { return b ? b->panel : 0; }

msv_status msv_batch_create(msv_batch** out, msv_plan* const* plans, msv_c128* const* d_A, int32_t n_plans,
                            int32_t m_lo, int32_t m_hi, void* stream) {
  g_batch_err.clear();
  if (!out || !plans || !d_A || n_plans < 1) return batch_fail(nullptr, MSV_EINVAL, "need plans and matrices");
  *out = nullptr;
  int nmax = 0;
  for (int i = 0; i < n_plans; ++i) {
    const msv_plan* p = plans[i];
    if (!p || !d_A[i]) return batch_fail(nullptr, MSV_EINVAL, "null plan or matrix buffer");
    if (p->precision != 1) return batch_fail(nullptr, MSV_EINVAL, "batched factorization needs precision 1 plans");
    if (m_lo < 0 || m_hi < m_lo || m_hi > p->M) return batch_fail(nullptr, MSV_EINVAL, "need 0 <= m_lo <= m_hi <= M");
    for (int j = 0; j < i; ++j)
      if (plans[j] == p) return batch_fail(nullptr, MSV_EINVAL, "a plan appears twice");
    nmax = std::max(nmax, 4 * p->N);
  }
  // a panel width is a candidate when every order below the largest is a
  // multiple of it (a panel then never straddles the end of a smaller matrix)
  bool ok128 = true, ok256 = true, ok512 = true;
  for (int i = 0; i < n_plans; ++i) {
    const int n = 4 * plans[i]->N;
    if (n != nmax && n % 128 != 0) ok128 = false;
    if (n != nmax && n % 256 != 0) ok256 = false;
    if (n != nmax && n % 512 != 0) ok512 = false;
  }
  msv_batch* b = new msv_batch();
  live_add(1);
  b->plans.assign(plans, plans + n_plans);
  b->A.assign(d_A, d_A + n_plans);
  b->m_lo = m_lo;
  b->m_hi = m_hi;
  b->nmax = nmax;
  const int nbp = m_hi - m_lo + 1;
  b->nb = n_plans * nbp;
  std::vector<msv::LuMat> list;
  for (int i = 0; i < n_plans; ++i) {
    msv_plan* p = plans[i];
    const int n = 4 * p->N;
    msv_status st = factor_buffers(p, n, nbp);
    if (st != MSV_OK) {
      std::string m = p->err;
      msv_batch_destroy(b);
      return batch_fail(nullptr, st, m);
    }
    for (int k = 0; k < nbp; ++k)
      list.push_back(msv::LuMat{p->d_fac32 + (size_t)k * n * n, p->d_ipiv + (size_t)k * n, p->d_info + k, n, 0});
  }
  if (dev_alloc((void**)&b->d_list, sizeof(msv::LuMat) * list.size()) != hipSuccess ||
      dev_alloc((void**)&b->d_work, msv::lu_work_bytes(nmax, b->nb, false)) != hipSuccess ||
      hipMemcpy(b->d_list, list.data(), sizeof(msv::LuMat) * list.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&b->ev_in) != hipSuccess || hipEventCreate(&b->ev_out) != hipSuccess) {
    msv_batch_destroy(b);
    return batch_fail(nullptr, MSV_ENOMEM, "batch allocation failed");
  }
  // Autotune the tiling: the outer panel width (64, 128, 256, 512) with the
  // planes kernel from 256, then at that width the smallest update that goes
  // to the planes kernel (256, 512, 1024).  Each candidate is captured, run
  // once to warm up and timed once; the fastest graph is kept.  A size class
  // tuned before in this process takes its choice from the table untimed.
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  int dev = 0;
  (void)hipGetDevice(&dev);
  const auto key = std::make_tuple(dev, ceil_log2(b->nmax), ceil_log2(b->nb),
                                   (ok128 ? 1 : 0) | (ok256 ? 2 : 0) | (ok512 ? 4 : 0));
  std::pair<int, int> known{0, 0};
  {
    std::lock_guard<std::mutex> l(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) known = it->second;
  }
  float best_ms = -1.f;
  auto try_one = [&](int panel, int plane_min, float* slot) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    float ms = -1.f;
    e = batch_capture(b, panel, plane_min, &g, &x);
    if (e == hipSuccess) e = hipGraphLaunch(x, b->st);
    if (e == hipSuccess) e = hipEventRecord(b->ev_in, b->st);
    if (e == hipSuccess) e = hipGraphLaunch(x, b->st);
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->st);
    if (e == hipSuccess) e = hipEventSynchronize(b->ev_out);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev_in, b->ev_out);
    if (slot) *slot = ms;
    if (e == hipSuccess && (best_ms < 0.f || ms < best_ms)) {
      best_ms = ms;
      if (b->exec) (void)hipGraphExecDestroy(b->exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->exec = x;
      b->graph = g;
      b->panel = panel;
      b->plane_min = plane_min;
    } else {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  };
  const int cands[4] = {64, 128, 256, 512}, planes[3] = {256, 512, 1024};
  if (known.first) {
    b->from_table = true;
    try_one(known.first, known.second, nullptr);
    for (int c = 0; c < 4; ++c)
      if (cands[c] == b->panel) b->tuned_ms[c] = best_ms;
    for (int q = 0; q < 3; ++q)
      if (planes[q] == b->plane_min) b->tuned_plane_ms[q] = best_ms;
  } else {
    for (int c = 0; c < 4 && e == hipSuccess; ++c) {
      if ((cands[c] == 128 && !ok128) || (cands[c] == 256 && !ok256) || (cands[c] == 512 && !ok512)) continue;
      try_one(cands[c], planes[0], &b->tuned_ms[c]);
    }
    const int panel = b->panel;
    for (int c = 0; c < 4; ++c)
      if (cands[c] == panel) b->tuned_plane_ms[0] = b->tuned_ms[c];
    for (int q = 1; q < 3 && e == hipSuccess; ++q) try_one(panel, planes[q], &b->tuned_plane_ms[q]);
    if (e == hipSuccess && b->exec) {
      std::lock_guard<std::mutex> l(g_tune_mu);
      g_tune[key] = std::make_pair(b->panel, b->plane_min);
    }
  }
  // leave the plans factored by the chosen configuration
  if (e == hipSuccess && b->exec) e = hipGraphLaunch(b->exec, b->st);
  if (e == hipSuccess) e = hipStreamSynchronize(b->st);
  if (e != hipSuccess || !b->exec) {
    std::string m = std::string("HIP: ") + hipGetErrorString(e);
    msv_batch_destroy(b);
    return batch_fail(nullptr, MSV_EHIP, m);
  }
  for (int i = 0; i < n_plans; ++i) {
    plans[i]->fac_lo = m_lo;
    plans[i]->fac_hi = m_hi;
    plans[i]->fac_A = d_A[i];
    plans[i]->info_checked = false;
    plans[i]->batch_refs++;
  }
  b->pinned = true;
  *out = b;
  return MSV_OK;
}

int32_t msv_batch_plane_min(const msv_batch* b) { return b ? b->plane_min : 0; }

float msv_batch_tuned_plane_ms(const msv_batch* b, int32_t plane_min) {
  if (!b) return -1.f;
  return plane_min == 256 ? b->tuned_plane_ms[0] : plane_min == 512 ? b->tuned_plane_ms[1]
         : plane_min == 1024 ? b->tuned_plane_ms[2] : -1.f;
}

int32_t msv_batch_tuned_from_table(const msv_batch* b) { return b && b->from_table ? 1 : 0; }

float msv_batch_tuned_ms(const msv_batch* b, int32_t panel) {
  if (!b) return -1.f;
  return panel == 64 ? b->tuned_ms[0] : panel == 128 ? b->tuned_ms[1] : panel == 256 ? b->tuned_ms[2]
         : panel == 512 ? b->tuned_ms[3] : -1.f;
}

msv_status msv_batch_factor(msv_batch* b, void* stream) {
  if (!b) return batch_fail(nullptr, MSV_EINVAL, "null batch");
  hipStream_t s = (hipStream_t)stream;
  if (hipEventRecord(b->ev_in, s) != hipSuccess || hipStreamWaitEvent(b->st, b->ev_in, 0) != hipSuccess ||
      hipGraphLaunch(b->exec, b->st) != hipSuccess || hipEventRecord(b->ev_out, b->st) != hipSuccess ||
      hipStreamWaitEvent(s, b->ev_out, 0) != hipSuccess)
    return batch_fail(b, MSV_EHIP, "graph launch failed");
  for (size_t i = 0; i < b->plans.size(); ++i) {
    b->plans[i]->fac_lo = b->m_lo;
    b->plans[i]->fac_hi = b->m_hi;
    b->plans[i]->fac_A = b->A[i];
    b->plans[i]->info_checked = false;
  }
  return MSV_OK;
}

// Device workspace of one solve: weighted right-hand sides, solution and
// residual (complex128), complex64 correction and sweep scratch (precision 1),
// per-vector residual ratios and their maximum, the vector-batch table.
struct SolveWork {
  double2 *bw, *xw, *rw;
  float2 *r32, *y32;
  double* nrm;
  msv::VecBatch* vb;
};

// Checks shared by both solve entry points; on success sets nvb.
static msv_status solve_check(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_rhs, const msv_c128* d_rhs,
                              msv_c128* d_x, int* nvb) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  if (!d_rhs || !d_x || d_rhs == d_x) return fail(p, MSV_EINVAL, "need distinct rhs and x buffers");
  if (n_rhs < 1 || m_hi < m_lo) return fail(p, MSV_EINVAL, "empty solve");
  if (p->fac_lo < 0) return fail(p, MSV_EINVAL, "no factors: call msv_factor first");
  for (int m = m_lo; m <= m_hi; ++m) {
    int a = m < 0 ? -m : m;
    if (a < p->fac_lo || a > p->fac_hi) return fail(p, MSV_EINVAL, "mode outside the factored range");
  }
  *nvb = msv::count_vec_batches(m_lo, m_hi - m_lo + 1, n_rhs, p->fac_lo, p->fac_hi - p->fac_lo + 1);
  return MSV_OK;
}

static SolveWork carve_solve_work(char* base, size_t n, size_t vectors, size_t nvb, int precision) {
  const size_t elems = vectors * n;
  SolveWork w{};
  w.bw = reinterpret_cast<double2*>(base);
  base += align256(sizeof(double2) * elems);
  w.xw = reinterpret_cast<double2*>(base);
  base += align256(sizeof(double2) * elems);
  w.rw = reinterpret_cast<double2*>(base);
  base += align256(sizeof(double2) * elems);
  if (precision == 1) {
    w.r32 = reinterpret_cast<float2*>(base);
    base += align256(sizeof(float2) * elems);
    w.y32 = reinterpret_cast<float2*>(base);
    base += align256(sizeof(float2) * elems);
  }
  w.nrm = reinterpret_cast<double*>(base);
  base += align256(sizeof(double) * (vectors + 1));
  w.vb = reinterpret_cast<msv::VecBatch*>(base);
  return w;
}

// The solve itself, on a workspace the caller provides; allocates nothing.
static msv_status solve_run(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_rhs, const msv_c128* d_rhs,
                            msv_c128* d_x, int nvb, const SolveWork& w, hipStream_t s) {
  const int n = 4 * p->N, nm = m_hi - m_lo + 1;
  const int nfac = p->fac_hi - p->fac_lo + 1;
  if (!p->info_checked) {
    // zero-pivot flags of the factorization, read in chunks into a fixed buffer
    int32_t info[64];
    for (int f0 = 0; f0 < nfac; f0 += 64) {
      const int cnt = std::min(64, nfac - f0);
      MSV_HIP(p, hipMemcpyAsync(info, p->d_info + f0, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s));
      MSV_HIP(p, hipStreamSynchronize(s));
      for (int i = 0; i < cnt; ++i)
        if (info[i] != 0) {
          char buf[120];
          snprintf(buf, sizeof buf, "zero pivot in mode %d at column %d", p->fac_lo + f0 + i, info[i] - 1);
          return fail(p, MSV_ESINGULAR, buf);
        }
    }
    p->info_checked = true;
  }
  const size_t elems = (size_t)nm * n_rhs * n;
  // the batch table is written on the device, in stream order behind any
  // earlier solve that still reads the same workspace
  MSV_HIP(p, msv::build_vec_batches(w.vb, nvb, m_lo, nm, n_rhs, p->fac_lo, nfac, s));
  const long long nn = (long long)n * n;
  const double2* rhs = reinterpret_cast<const double2*>(d_rhs);
  double2* x = reinterpret_cast<double2*>(d_x);
  MSV_HIP(p, msv::solve_prep(rhs, w.bw, p->d_sqw, n, n_rhs, nm, m_lo, s));
  if (p->precision == 0) {
    MSV_HIP(p, msv::gather_z(w.bw, w.xw, p->d_perm, w.vb, nvb, n, s));
    MSV_HIP(p, msv::trsv_z(reinterpret_cast<const double2*>(p->fac_A), static_cast<const double2*>(p->d_inv), nn, n,
                           w.vb, nvb, w.xw, w.rw, s));
    p->last_ir_iters = 0;
    MSV_HIP(p, msv::solve_finish(w.xw, x, p->d_sqw, n, n_rhs, nm, m_lo, s));
    return MSV_OK;
  }
  const double2* Aref = reinterpret_cast<const double2*>(p->fac_A);
  MSV_HIP(p, msv::zero_c128(w.xw, elems, s));
  MSV_HIP(p, hipMemcpyAsync(w.rw, w.bw, sizeof(double2) * elems, hipMemcpyDeviceToDevice, s));
  const int nvec = nm * n_rhs;
  bool conv = false;
  int it = 0;
  // The steps that the plan's previous converged solve needed are queued
  // without waiting; the largest residual ratio is read on the host only from
  // the last of them on, so a repeated solve waits on the device once.
  const int unchecked = std::min(p->ir_max_iter, std::max(p->ir_pred, 1)) - 1;
  for (it = 1; it <= p->ir_max_iter; ++it) {
    MSV_HIP(p, msv::gather_c(w.rw, w.r32, p->d_perm, w.vb, nvb, n, s));
    MSV_HIP(p, msv::trsv_c(p->d_fac32, static_cast<const float2*>(p->d_inv), nn, n, w.vb, nvb, w.r32, w.y32, s));
    MSV_HIP(p, msv::accum_c64(w.xw, w.r32, elems, s));
    MSV_HIP(p, msv::residual_batches(Aref, nn, n, w.vb, nvb, w.bw, w.xw, w.rw, s));
    if (it <= unchecked) continue;
    MSV_HIP(p, msv::ratios(w.rw, w.bw, w.nrm, n, nvec, s));
    double mx = 0.0;
    MSV_HIP(p, hipMemcpyAsync(&mx, w.nrm + nvec, sizeof(double), hipMemcpyDeviceToHost, s));
    MSV_HIP(p, hipStreamSynchronize(s));
    if (mx <= p->ir_tol) {
      conv = true;
      break;
    }
  }
  p->last_ir_iters = conv ? it : p->ir_max_iter;
  p->ir_pred = conv ? it : 0;
  MSV_HIP(p, msv::solve_finish(w.xw, x, p->d_sqw, n, n_rhs, nm, m_lo, s));
  if (!conv) return fail(p, MSV_ENOCONV, "iterative refinement did not reach ir_tol");
  return MSV_OK;
}

msv_status msv_solve(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_rhs, const msv_c128* d_rhs,
                     msv_c128* d_x, void* stream) {
  int nvb = 0;
  MSV_CHECK(solve_check(p, m_lo, m_hi, n_rhs, d_rhs, d_x, &nvb));
  const size_t n = 4 * (size_t)p->N, vectors = (size_t)(m_hi - m_lo + 1) * n_rhs;
  const size_t need = solve_work_bytes(n, vectors, (size_t)nvb, p->precision);
  if (need > p->work_bytes) {
    if (p->d_work) dev_free(p->d_work);
    p->d_work = nullptr;
    p->work_bytes = 0;
    if (dev_alloc((void**)&p->d_work, need) != hipSuccess) return fail(p, MSV_ENOMEM, "solve workspace allocation failed");
    p->work_bytes = need;
  }
  const SolveWork w = carve_solve_work(static_cast<char*>(p->d_work), n, vectors, (size_t)nvb, p->precision);
  return solve_run(p, m_lo, m_hi, n_rhs, d_rhs, d_x, nvb, w, (hipStream_t)stream);
}

msv_status msv_solve_noalloc(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_rhs, const msv_c128* d_rhs,
                             msv_c128* d_x, void* stream) {
  int nvb = 0;
  MSV_CHECK(solve_check(p, m_lo, m_hi, n_rhs, d_rhs, d_x, &nvb));
  if (!p->scratch) return fail(p, MSV_EHIP, "no device address for the static workspace: " + p->scratch_err);
  const size_t n = 4 * (size_t)p->N, vectors = (size_t)(m_hi - m_lo + 1) * n_rhs;
  const size_t need = solve_work_bytes(n, vectors, (size_t)nvb, p->precision);
  if (need > kScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf, "solve needs %zu bytes of workspace; msv_solve_noalloc has %zu: solve fewer modes "
             "or right-hand sides per call", need, kScratchBytes);
    return fail(p, MSV_EINVAL, buf);
  }
  const SolveWork w = carve_solve_work(static_cast<char*>(p->scratch), n, vectors, (size_t)nvb, p->precision);
  return solve_run(p, m_lo, m_hi, n_rhs, d_rhs, d_x, nvb, w, (hipStream_t)stream);
}

size_t msv_solve_noalloc_max_bytes(void) { return kScratchBytes; }

// ---------------------------------------------------------------------------
// fields off the surface and far field
// ---------------------------------------------------------------------------
namespace {

msv_status field_common(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_vec, const msv_c128* d_x,
                        int32_t n_pts, const void* d_pts, double kabs, double tmul, double tadd, int U,
                        size_t extra_elems, msv::FieldParams& F, void** buf, hipStream_t s) {
  if (!d_x || !d_pts) return fail(p, MSV_EINVAL, "null buffer");
  if (m_lo < -p->M || m_hi < m_lo || m_hi > p->M) return fail(p, MSV_EINVAL, "need -M <= m_lo <= m_hi <= M");
  if (n_vec < 1 || n_pts < 1) return fail(p, MSV_EINVAL, "need n_vec >= 1 and at least one point");
  const int mmax = std::max(std::abs(m_lo), std::abs(m_hi));
  double rmax = 0.0;
  for (double r : p->h_r) rmax = std::max(rmax, r);
  const int T = (int)(tmul * (mmax + kabs * rmax) + tadd);
  const size_t grid_elems = (size_t)n_vec * p->N * U * T * 4;
  if ((long long)n_vec * p->N * U >= (1LL << 23) || (long long)n_vec * n_pts >= (1LL << 23))
    return fail(p, MSV_EINVAL, "too many vectors x nodes or vectors x points for one launch");
  const size_t bytes = (grid_elems + T + extra_elems) * sizeof(double2);
  if (hipMallocAsync(buf, bytes, s) != hipSuccess) {
    (void)hipGetLastError();  // clear the sticky error of the failed allocation
    return fail(p, MSV_ENOMEM, "surface-grid workspace allocation failed");
  }
  F.N = p->N * U;
  F.T = T;
  F.nm = m_hi - m_lo + 1;
  F.m_lo = m_lo;
  F.nvec = n_vec;
  F.r = p->d_r;
  F.z = p->d_z;
  F.tr = p->d_tr;
  F.tz = p->d_tz;
  F.w = p->d_w;
  F.x = reinterpret_cast<const double2*>(d_x);
  F.grid = static_cast<double2*>(*buf);
  F.tw = F.grid + grid_elems;
  F.npts = n_pts;
  F.pts = static_cast<const double*>(d_pts);
  F.k0 = p->k0;
  F.omega = p->omega;
  F.mu0 = p->mu0.real();
  return MSV_OK;
}

inline double2 d2(cplx z) { return make_double2(z.real(), z.imag()); }

}  // namespace

msv_status msv_far_field(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_vec, const msv_c128* d_x,
                         int32_t n_dirs, const double* d_dirs, msv_c128* d_out, void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  if (!d_out) return fail(p, MSV_EINVAL, "null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  msv::FieldParams F{};
  void* buf = nullptr;
  msv_status st = field_common(p, m_lo, m_hi, n_vec, d_x, n_dirs, d_dirs, p->k0, 2.0, 64.0, 1, 0, F, &buf, s);
  if (st != MSV_OK) return st;
  F.out = reinterpret_cast<double2*>(d_out);
  hipError_t e = msv::launch_surface_grid(F, s);
  if (e == hipSuccess) e = msv::launch_far_field(F, s);
  hipError_t ef = hipFreeAsync(buf, s);
  if (e != hipSuccess || ef != hipSuccess) return fail(p, MSV_EHIP, "far-field launch failed");
  return MSV_OK;
}

// Sub-panel geometry for msv_fields: each panel's r, z, dr/du, dz/du
// interpolated (Legendre, from its 16 nodes) to U sub-panels of 16
// Gauss-Legendre nodes, sub-panel q spanning u in [-1 + 2q/U, -1 + 2(q+1)/U].
static msv_status ensure_upsampled(msv_plan* p, int U, hipStream_t s) {
  if (p->up_U == U && p->d_up) return MSV_OK;
  std::vector<double> ug, wg;
  gauss_legendre(kOrder, ug, wg);
  std::vector<double> bw(kOrder, 1.0);
  for (int j = 0; j < kOrder; ++j)
    for (int k = 0; k < kOrder; ++k)
      if (k != j) bw[j] /= (ug[j] - ug[k]);
  const int F = kOrder * U, NU = p->N * U;
  std::vector<double> h(5 * (size_t)NU + (size_t)F * kOrder);
  double* L = h.data() + 5 * (size_t)NU;
  for (int q = 0; q < U; ++q)
    for (int v = 0; v < kOrder; ++v) lagrange_row(ug, bw, -1.0 + (2.0 * q + ug[v] + 1.0) / U, L + (q * kOrder + v) * kOrder);
  for (int pn = 0; pn < p->npan; ++pn)
    for (int f = 0; f < F; ++f) {
      double r = 0, z = 0, ru = 0, zu = 0;
      for (int j = 0; j < kOrder; ++j) {
        const int n = pn * kOrder + j;
        const double l = L[f * kOrder + j];
        r += l * p->h_r[n];
        z += l * p->h_z[n];
        ru += l * p->h_dru[n];
        zu += l * p->h_dzu[n];
      }
      const double sp = std::hypot(ru, zu);
      const size_t nf = (size_t)pn * F + f;
      h[nf] = r;
      h[NU + nf] = z;
      h[2 * (size_t)NU + nf] = ru / sp;
      h[3 * (size_t)NU + nf] = zu / sp;
      h[4 * (size_t)NU + nf] = wg[f % kOrder] * sp / U;
    }
  // the previous sub-panel geometry may still be read by work on `s`
  if (hipStreamSynchronize(s) != hipSuccess) return fail(p, MSV_EHIP, "stream synchronize failed");
  if (p->d_up) dev_free(p->d_up);
  p->d_up = nullptr;
  p->up_bytes = 0;
  p->up_U = 0;
  if (dev_alloc((void**)&p->d_up, h.size() * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();  // clear the sticky error of the failed allocation
    p->d_up = nullptr;
    return fail(p, MSV_ENOMEM, "sub-panel geometry allocation failed");
  }
  if (hipMemcpy(p->d_up, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return fail(p, MSV_EHIP, "sub-panel geometry upload failed");
  p->up_bytes = h.size() * sizeof(double);
  p->up_U = U;
  return MSV_OK;
}

msv_status msv_fields(msv_plan* p, int32_t m_lo, int32_t m_hi, int32_t n_vec, const msv_c128* d_x,
                      int32_t n_points, const double* d_points, int32_t region, int32_t upsample, msv_c128* d_E,
                      msv_c128* d_H, void* stream) {
  if (!p) return fail(nullptr, MSV_EINVAL, "null plan");
  if (!d_E || !d_H) return fail(p, MSV_EINVAL, "null buffer");
  if (region != 0 && region != 1) return fail(p, MSV_EINVAL, "region must be 0 (exterior) or 1 (interior)");
  if (upsample < 1 || upsample > 8) return fail(p, MSV_EINVAL, "upsample must be in [1, 8]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const cplx k = region == 0 ? cplx(p->k0, 0.0) : p->k1;
  if (upsample > 1) {
    msv_status su = ensure_upsampled(p, upsample, s);
    if (su != MSV_OK) return su;
  }
  msv::FieldParams F{};
  void* buf = nullptr;
  const size_t x_elems = (size_t)(m_hi - m_lo + 1) * n_vec * 4 * p->N * upsample;
  msv_status st = field_common(p, m_lo, m_hi, n_vec, d_x, n_points, d_points, std::abs(k), 4.0, 128.0, upsample,
                               upsample > 1 ? x_elems : 0, F, &buf, s);
  if (st != MSV_OK) return st;
  if (upsample > 1) {
    const int NU = p->N * upsample;
    double2* xf = F.tw + F.T;
    hipError_t ei = msv::launch_interp_currents(F.x, xf, p->d_up + 5 * (size_t)NU, p->N, upsample,
                                                (m_hi - m_lo + 1) * n_vec, s);
    if (ei != hipSuccess) {
      (void)hipFreeAsync(buf, s);
      return fail(p, MSV_EHIP, "current interpolation launch failed");
    }
    F.x = xf;
    F.r = p->d_up;
    F.z = p->d_up + NU;
    F.tr = p->d_up + 2 * (size_t)NU;
    F.tz = p->d_up + 3 * (size_t)NU;
    F.w = p->d_up + 4 * (size_t)NU;
  }
  F.kr = k.real();
  F.ki = k.imag();
  // E = aE curl curl S J + bE curl S M, H = aH curl curl S M + bH curl S J
  const cplx iw(0.0, p->omega);
  cplx aE, bE, aH, bH;
  if (region == 0) {  // eq. exteriorfield
    aE = -1.0 / (iw * p->eps0);
    bE = 1.0;
    aH = 1.0 / (iw * p->mu0);
    bH = 1.0;
  } else if (p->formulation == 0) {  // eq. interiorfield
    aE = 1.0 / (iw * p->eps1);
    bE = -1.0;
    aH = -1.0 / (iw * p->mu1);
    bH = -1.0;
  } else {  // eq. interior_dual
    aE = -1.0 / (iw * p->eps0);
    bE = p->mu1 / p->mu0;
    aH = 1.0 / (iw * p->mu0);
    bH = p->eps1 / p->eps0;
  }
  F.aE = d2(aE);
  F.bE = d2(bE);
  F.aH = d2(aH);
  F.bH = d2(bH);
  F.out = reinterpret_cast<double2*>(d_E);
  F.out2 = reinterpret_cast<double2*>(d_H);
  hipError_t e = msv::launch_surface_grid(F, s);
  if (e == hipSuccess) e = msv::launch_fields(F, s);
  hipError_t ef = hipFreeAsync(buf, s);
  if (e != hipSuccess || ef != hipSuccess) return fail(p, MSV_EHIP, "field launch failed");
  return MSV_OK;
}

}  // extern "C"
