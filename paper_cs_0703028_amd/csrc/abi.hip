// abi.hip -- host side of the C ABI declared in include/rtlbl.h: argument
// validation, device memory owned by the handle, launch sequencing on the
// borrowed stream, timing with HIP events.  Every failure is reported as a
// status code plus a message; nothing aborts.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "adaptive.h"
#include "rt_internal.h"

namespace {

thread_local std::string g_create_error;

// Device scratch of rt_trace_rays_noalloc: one batch of rays' segments,
// counts, coherent-order keys and permutation, and the order's histogram.
// Each GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: rt_create looks up
// the device address once per device (hipGetSymbolAddress, device current)
// and every launch takes that address.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device index, nullptr until looked up

// The device address of `scratch` on `device` (which must be current).
hipError_t scratch_address(int device, int n_devices, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() < n_devices) g_scratch_ptr.resize(n_devices, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

rt_status fail(rt_ctx c, rt_status s, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

// Reports a HIP failure and clears it from the runtime's last error, so that
// the next call's launch checks do not report it again.
rt_status hip_fail(rt_ctx c, hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(c, (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? RT_ENOMEM : RT_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define RT_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);  \
  } while (0)

// A failed hipMalloc also leaves its error as the runtime's last error, which
// the next launch check (hipGetLastError) would report; it is cleared here and
// returned once.
template <class T>
hipError_t dev_alloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// v as an FP32 pair hi + lo (hi = v rounded, lo = the rest rounded).
float2 split_pair(double v) {
  const float h = (float)v;
  return make_float2(h, (float)(v - (double)h));
}

// The precision form's per-cell inputs (see rt::CellSet), formed on the host
// from the FP64 gas state and uploaded: u/(pi dnu), log2(T_ref/T), p/dnu,
// 1/T_ref - 1/T and c2/T, and each further gas's u/(pi dnu).
rt_status upload_cells32(rt_ctx c) {
  const int64_t n = c->n_cells;
  const double c2 = rt::second_radiation_cm_K();
  std::vector<float> uf(n), lam(n), P(n);
  std::vector<float2> beta(n), theta(n);
  auto dens = [&](double T, double x, double p) {
    return x * p * rt::kAtm / (rt::kBoltzmann * T) * 1e-6 / (M_PI * c->dnu);
  };
  for (int64_t i = 0; i < n; ++i) {
    const double T = c->hT[i];
    uf[i] = (float)dens(T, c->hx[i], c->hp[i]);
    lam[i] = (float)std::log2(c->T_ref / T);
    P[i] = (float)(c->hp[i] / c->dnu);
    beta[i] = split_pair(1.0 / c->T_ref - 1.0 / T);
    theta[i] = split_pair(c2 / T);
  }
  RT_HIP(c, hipMemcpy(c->cells.uf, uf.data(), n * sizeof(float), hipMemcpyHostToDevice));
  RT_HIP(c, hipMemcpy(c->cells.lamf, lam.data(), n * sizeof(float), hipMemcpyHostToDevice));
  RT_HIP(c, hipMemcpy(c->cells.Pf, P.data(), n * sizeof(float), hipMemcpyHostToDevice));
  RT_HIP(c, hipMemcpy(c->cells.beta2, beta.data(), n * sizeof(float2), hipMemcpyHostToDevice));
  RT_HIP(c, hipMemcpy(c->cells.theta2, theta.data(), n * sizeof(float2), hipMemcpyHostToDevice));
  for (auto& g : c->gas) {
    if (!g.active) continue;
    for (int64_t i = 0; i < n; ++i) uf[i] = (float)dens(c->hT[i], g.hx[i], c->hp[i]);
    RT_HIP(c, hipMemcpy(g.uf, uf.data(), n * sizeof(float), hipMemcpyHostToDevice));
  }
  return RT_OK;
}

bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

void free_lineset(rt::LineSet& L) {
  dev_free(L.m); dev_free(L.phi); dev_free(L.wlo); dev_free(L.whi); dev_free(L.S);
  dev_free(L.E2); dev_free(L.nu); dev_free(L.gamma); dev_free(L.nexp); dev_free(L.prof16);
  dev_free(L.tile16);
  dev_free(L.span4);
  dev_free(L.r64); dev_free(L.S64); dev_free(L.g64); dev_free(L.n64);
  dev_free(L.aE); dev_free(L.rN);
  dev_free(L.E2p); dev_free(L.nup);
  L.n = 0;
  L.n_tiles16 = 0;
  L.n_spans = 0;
}

void free_lines(rt_ctx c) { free_lineset(c->lines); }

int n_gases(rt_ctx c) {
  int n = 1;
  for (const auto& g : c->gas) n += g.active ? 1 : 0;
  return n;
}

// Removes gases 1..kMaxGases-1 (their lines and per-cell arrays).
void free_gases(rt_ctx c) {
  for (auto& g : c->gas) {
    free_lineset(g.lines);
    dev_free(g.x);
    dev_free(g.G);
    dev_free(g.uf);
    dev_free(g.Gq);
    g = rt::ExtraGas();
  }
}

void free_cells(rt_ctx c) {
  rt::CellSet& C = c->cells;
  dev_free(C.G); dev_free(C.beta); dev_free(C.theta); dev_free(C.lam2); dev_free(C.P);
  dev_free(C.uf); dev_free(C.lamf); dev_free(C.Pf); dev_free(C.beta2); dev_free(C.theta2);
  dev_free(C.Gq);
}

void free_events(std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
  for (auto& e : v) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  v.clear();
}

rt_status record_begin(rt_ctx c, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
  hipEvent_t a, b;
  RT_HIP(c, hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  if (e != hipSuccess) { (void)hipEventDestroy(a); return hip_fail(c, e, "hipEventCreate"); }
  v.emplace_back(a, b);
  RT_HIP(c, hipEventRecord(a, c->stream));
  return RT_OK;
}

rt_status record_end(rt_ctx c, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
  RT_HIP(c, hipEventRecord(v.back().second, c->stream));
  return RT_OK;
}

// Sum of elapsed times of completed event pairs (ms); the list is emptied.
rt_status drain_events(rt_ctx c, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double* ms) {
  double t = 0;
  for (auto& e : v) {
    RT_HIP(c, hipEventSynchronize(e.second));
    float f = 0;
    RT_HIP(c, hipEventElapsedTime(&f, e.first, e.second));
    t += f;
  }
  free_events(v);
  *ms += t;
  return RT_OK;
}

// Makes the handle's device current; a host-only handle has none.
rt_status set_device(rt_ctx c) {
  if (c->device < 0)
    return fail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_HIP(c, hipSetDevice(c->device));
  return RT_OK;
}

// Ray scratch: per-ray segment lists for one batch of rays.
// Batch scratch for `need` rays, up to the cap: at most ~1 GiB of segments
// per batch (large batches make the coherent ray order denser), at least
// 4096 and at most 2^21 rays.  Grows, never shrinks, for one grid shape.
rt_status ensure_batch(rt_ctx c, int64_t need) {
  const int max_segs = c->nx + c->ny + c->nz;
  int64_t cap = std::max<int64_t>(4096, (int64_t)(1ll << 30) / (8ll * max_segs));
  cap = std::min<int64_t>(cap, 1 << 21) / 4096 * 4096;
  const int64_t want = std::min<int64_t>(cap, (std::max<int64_t>(need, 1) + 4095) / 4096 * 4096);
  if (c->d_segs && c->max_segs == max_segs && c->batch_rays >= want) return RT_OK;
  dev_free(c->d_segs);
  dev_free(c->d_counts);
  dev_free(c->d_keys);
  dev_free(c->d_perm);
  c->max_segs = max_segs;
  c->batch_rays = want;
  RT_HIP(c, dev_alloc(&c->d_segs, (size_t)want * max_segs));
  RT_HIP(c, dev_alloc(&c->d_counts, (size_t)want));
  RT_HIP(c, dev_alloc(&c->d_keys, (size_t)want));
  RT_HIP(c, dev_alloc(&c->d_perm, (size_t)want));
  if (!c->d_hist) RT_HIP(c, dev_alloc(&c->d_hist, (size_t)rt::kOrderBuckets));
  return RT_OK;
}

double ray_weight(rt_ctx c, double n_rays_total) {
  const double h = c->cell_m;
  const double area = 2.0 * h * h *
                      ((double)c->nx * c->ny + (double)c->ny * c->nz + (double)c->nz * c->nx);
  return M_PI * area * c->dnu / n_rays_total;
}

}  // namespace

extern "C" {

rt_status rt_create(rt_ctx* out, int hip_device, void* hip_stream) {
  if (!out) return fail(nullptr, RT_EINVAL, "rt_create: out is NULL");
  *out = nullptr;
  if (hip_device == RT_NO_DEVICE) {  // argument and call-order checks only
    if (hip_stream) return fail(nullptr, RT_EINVAL, "rt_create: a host-only handle takes no stream");
    rt_ctx c = new (std::nothrow) rt_ctx_s();
    if (!c) return fail(nullptr, RT_ENOMEM, "rt_create: out of host memory");
    c->device = RT_NO_DEVICE;
    *out = c;
    return RT_OK;
  }
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0)
    return fail(nullptr, RT_EDEVICE, std::string("rt_create: no HIP device: ") + hipGetErrorString(e));
  if (hip_device < 0 || hip_device >= n)
    return fail(nullptr, RT_EINVAL, "rt_create: device index out of range");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, hip_device);
  if (e != hipSuccess) return fail(nullptr, RT_EDEVICE, "rt_create: hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, RT_EUNSUPPORTED,
                std::string("rt_create: built for gfx950 only, device is ") + prop.gcnArchName);
  rt_ctx c = new (std::nothrow) rt_ctx_s();
  if (!c) return fail(nullptr, RT_ENOMEM, "rt_create: out of host memory");
  c->device = hip_device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  e = hipSetDevice(hip_device);
  if (e == hipSuccess) e = scratch_address(hip_device, n, &c->noalloc_scratch);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->d_balance), 4 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->d_segcount), sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->d_adapt_evals), sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->d_adapt_evals, 0, sizeof(unsigned long long));
  if (e != hipSuccess) {
    (void)hipGetLastError();  // not left for the next launch check
    rt_destroy(c);
    return fail(nullptr, RT_ENOMEM, std::string("rt_create: ") + hipGetErrorString(e));
  }
  *out = c;
  return RT_OK;
}

rt_status rt_destroy(rt_ctx c) {
  if (!c) return RT_OK;
  if (c->device < 0) {  // host-only: no device memory, nothing in flight
    delete c;
    return RT_OK;
  }
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  free_lines(c);
  free_gases(c);
  free_cells(c);
  dev_free(c->d_T); dev_free(c->d_x); dev_free(c->d_p);
  dev_free(c->d_bwall);
  dev_free(c->d_abs); dev_free(c->d_emi); dev_free(c->d_acc); dev_free(c->d_balance);
  dev_free(c->d_segcount);
  dev_free(c->d_sbar); dev_free(c->d_win); dev_free(c->d_adapt_evals); dev_free(c->d_und);
  dev_free(c->d_segs); dev_free(c->d_counts); dev_free(c->d_rays_explicit); dev_free(c->d_exit);
  dev_free(c->d_keys); dev_free(c->d_perm); dev_free(c->d_hist);
  free_events(c->trace_events); free_events(c->march_events); free_events(c->kappa_events);
  free_events(c->batch_events);
  rt::destroy_batch(c);
  rt::free_surrogate(c);
  delete c;
  return RT_OK;
}

const char* rt_last_error(rt_ctx c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

rt_status rt_setup_grid(rt_ctx c, int nx, int ny, int nz, double cell_m, const double* T,
                        const double* x, const double* p, double T_wall) {
  if (!c) return fail(c, RT_EINVAL, "rt_setup_grid: NULL handle");
  if (nx < 1 || ny < 1 || nz < 1 || nx > rt::kMaxAxis || ny > rt::kMaxAxis || nz > rt::kMaxAxis)
    return fail(c, RT_EINVAL, "rt_setup_grid: each of nx, ny, nz must be in [1, 2^20]");
  const int64_t n = (int64_t)nx * ny * nz;
  if (n >= (int64_t(1) << 31)) return fail(c, RT_EINVAL, "rt_setup_grid: nx*ny*nz must be < 2^31");
  if (!(cell_m > 0) || !std::isfinite(cell_m)) return fail(c, RT_EINVAL, "rt_setup_grid: cell_m must be > 0");
  if (!T || !x || !p) return fail(c, RT_EINVAL, "rt_setup_grid: NULL array");
  if (!(T_wall >= 0) || !std::isfinite(T_wall)) return fail(c, RT_EINVAL, "rt_setup_grid: T_wall must be >= 0");
  if (!finite_all(T, n) || !finite_all(x, n) || !finite_all(p, n))
    return fail(c, RT_EINVAL, "rt_setup_grid: non-finite cell value");
  for (int64_t i = 0; i < n; ++i) {
    if (!(T[i] > 0)) return fail(c, RT_EINVAL, "rt_setup_grid: T must be > 0");
    if (!(x[i] >= 0 && x[i] <= 1)) return fail(c, RT_EINVAL, "rt_setup_grid: x_h2o must be in [0, 1]");
    if (!(p[i] > 0)) return fail(c, RT_EINVAL, "rt_setup_grid: p must be > 0");
  }
  if (c->device < 0) {  // host-only: record the grid, allocate nothing
    free_gases(c);
    c->nx = nx; c->ny = ny; c->nz = nz;
    c->n_cells = n;
    c->cell_m = cell_m;
    c->T_wall = T_wall;
    c->have_grid = true;
    c->have_kappa = false;
    c->cells_valid = false;
    c->cells32_valid = false;
    return RT_OK;
  }
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, hipStreamSynchronize(c->stream));
  dev_free(c->d_T); dev_free(c->d_x); dev_free(c->d_p);
  dev_free(c->d_abs); dev_free(c->d_emi); dev_free(c->d_acc);
  c->d_ovf = nullptr;
  free_cells(c);
  free_gases(c);
  c->have_grid = false;
  c->have_kappa = false;
  c->cells_valid = false;
  c->cells32_valid = false;
  RT_HIP(c, dev_alloc(&c->d_T, n));
  RT_HIP(c, dev_alloc(&c->d_x, n));
  RT_HIP(c, dev_alloc(&c->d_p, n));
  RT_HIP(c, dev_alloc(&c->d_abs, n));
  RT_HIP(c, dev_alloc(&c->d_emi, n));
  // accumulator rows of the cells and the balance, then the overflow flag
  RT_HIP(c, dev_alloc(&c->d_acc, (size_t)((n + rt::kBalRows) * rt::kAccRow + 1)));
  c->d_ovf = reinterpret_cast<unsigned*>(c->d_acc + (n + rt::kBalRows) * rt::kAccRow);
  RT_HIP(c, dev_alloc(&c->cells.G, n));
  RT_HIP(c, dev_alloc(&c->cells.beta, n));
  RT_HIP(c, dev_alloc(&c->cells.theta, n));
  RT_HIP(c, dev_alloc(&c->cells.lam2, n));
  RT_HIP(c, dev_alloc(&c->cells.P, n));
  RT_HIP(c, dev_alloc(&c->cells.uf, n));
  RT_HIP(c, dev_alloc(&c->cells.lamf, n));
  RT_HIP(c, dev_alloc(&c->cells.Pf, n));
  RT_HIP(c, dev_alloc(&c->cells.beta2, n));
  RT_HIP(c, dev_alloc(&c->cells.theta2, n));
  RT_HIP(c, dev_alloc(&c->cells.Gq, n));
  RT_HIP(c, hipMemcpyAsync(c->d_T, T, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  RT_HIP(c, hipMemcpyAsync(c->d_x, x, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  RT_HIP(c, hipMemcpyAsync(c->d_p, p, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  c->hT.assign(T, T + n);
  c->hx.assign(x, x + n);
  c->hp.assign(p, p + n);
  RT_HIP(c, hipStreamSynchronize(c->stream));  // host arrays may be freed on return
  c->nx = nx; c->ny = ny; c->nz = nz;
  c->n_cells = n;
  c->cell_m = cell_m;
  c->T_wall = T_wall;
  c->T_argmin = std::min_element(T, T + n) - T;
  c->T_argmax = std::max_element(T, T + n) - T;
  c->T_min = T[c->T_argmin];
  c->T_max = T[c->T_argmax];
  c->grid_epoch += 1;
  c->have_grid = true;
  c->stats = rt::Stats();
  RT_HIP(c, rt::launch_zero(c));
  return RT_OK;
}

// The per-line checks of rt_setup_lines and rt_setup_gas.
rt_status check_line_arrays(rt_ctx c, const char* who, int n_lines, const double* nu,
                            const double* S, const double* gamma, const double* n_T,
                            const double* E) {
  const std::string w(who);
  if (n_lines < 0) return fail(c, RT_EINVAL, w + ": n_lines must be >= 0");
  if (n_lines > 0 && (!nu || !S || !gamma || !n_T))
    return fail(c, RT_EINVAL, w + ": NULL line array");
  if (n_lines > 0) {
    if (!finite_all(nu, n_lines) || !finite_all(S, n_lines) || !finite_all(gamma, n_lines) ||
        !finite_all(n_T, n_lines) || (E && !finite_all(E, n_lines)))
      return fail(c, RT_EINVAL, w + ": non-finite line parameter");
    for (int i = 0; i < n_lines; ++i) {
      if (!(S[i] >= 0)) return fail(c, RT_EINVAL, w + ": S_ref must be >= 0");
      if (!(gamma[i] > 0)) return fail(c, RT_EINVAL, w + ": gamma_ref must be > 0");
      if (E && !(E[i] >= 0)) return fail(c, RT_EINVAL, w + ": E_lower must be >= 0");
    }
  }
  return RT_OK;
}

// Validates one line list, keeps the lines whose window [m - K + [phi > 0],
// m + K] meets [0, n_nu - 1], sorts them by r = (nu - nu0)/dnu = m + phi and
// uploads them into L (device arrays allocated here; L must be empty).
// evals: in-grid window points summed over the kept lines.
rt_status build_lines(rt_ctx c, const char* who, int n_lines, const double* nu, const double* S,
                      const double* gamma, const double* n_T, const double* E, double T_ref,
                      int K, double nu0, double dnu, int n_nu, rt::LineSet& L, double& evals) {
  const std::string w(who);
  if (rt_status s = check_line_arrays(c, who, n_lines, nu, S, gamma, n_T, E)) return s;
  const double c2 = rt::second_radiation_cm_K();
  struct Rec { double r; int64_t m; double phi; int src; };
  std::vector<Rec> recs;
  recs.reserve(n_lines);
  evals = 0;
  for (int i = 0; i < n_lines; ++i) {
    const double r = (nu[i] - nu0) / dnu;
    const double fm = std::floor(r);
    if (!(std::fabs(fm) < 4.0e15)) continue;
    const int64_t m = (int64_t)fm;
    const double phi = r - fm;
    const int64_t lo = m - K + (phi > 0 ? 1 : 0), hi = m + K;
    if (hi < 0 || lo > n_nu - 1) continue;
    recs.push_back({r, m, phi, i});
    evals += (double)(std::min<int64_t>(hi, n_nu - 1) - std::max<int64_t>(lo, 0) + 1);
  }
  std::stable_sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) { return a.r < b.r; });
  const int nl = (int)recs.size();
  std::vector<int32_t> hm(nl), hwlo(nl), hwhi(nl);
  std::vector<float> hphi(nl), hS(nl), hg(nl), hn(nl);
  std::vector<double> hE2(nl), hnu(nl);
  std::vector<float2> hE2p(nl), hnup(nl);
  std::vector<double> hr64(nl), hS64(nl), hg64(nl), hn64(nl), haE(nl), hrN(nl);
  std::vector<float> hprof((size_t)nl * 16);
  for (int k = 0; k < nl; ++k) {
    // the 16 tabulated points j = m - 7 .. m + 8, at distance j - r from the
    // centre, of the reference-state Lorentz shape
    const Rec& q16 = recs[k];
    const double g = gamma[q16.src];
    for (int t = 0; t < 16; ++t) {
      const double d = ((double)(t - 7) - q16.phi) * dnu;
      hprof[(size_t)k * 16 + t] = (float)(g / (M_PI * (d * d + g * g)));
    }
  }
  for (int k = 0; k < nl; ++k) {
    const Rec& q = recs[k];
    const int i = q.src;
    hm[k] = (int32_t)q.m;
    hphi[k] = (float)q.phi;
    hwlo[k] = (int32_t)(q.m - K + (q.phi > 0 ? 1 : 0));
    hwhi[k] = (int32_t)(q.m + K);
    // with energies, S / (1 - exp(-c2 nu / T_ref)) (the reference-state
    // stimulated-emission factor of Eq. (1) is a per-line constant)
    hS[k] = (float)(E ? S[i] / (-std::expm1(-c2 * nu[i] / T_ref)) : S[i]);
    hE2[k] = E ? c2 * E[i] : 0.0;
    hnu[k] = nu[i];
    hE2p[k] = split_pair(hE2[k]);
    hnup[k] = split_pair(nu[i]);
    hg[k] = (float)gamma[i];
    hn[k] = (float)n_T[i];
    // binary64 data of the adaptive windows: the centre in grid units as
    // placed above, the line constants, -c2 E and the reciprocal of the
    // reference-state factor expm1(-c2 nu / T_ref) of Eq. (1)
    hr64[k] = q.r;
    hS64[k] = S[i];
    hg64[k] = gamma[i];
    hn64[k] = n_T[i];
    haE[k] = E ? -c2 * E[i] : 0.0;
    hrN[k] = 1.0 / std::expm1(-c2 * nu[i] / T_ref);
  }
  RT_HIP(c, dev_alloc(&L.m, nl));
  RT_HIP(c, dev_alloc(&L.phi, nl));
  RT_HIP(c, dev_alloc(&L.wlo, nl));
  RT_HIP(c, dev_alloc(&L.whi, nl));
  RT_HIP(c, dev_alloc(&L.S, nl));
  RT_HIP(c, dev_alloc(&L.E2, nl));
  RT_HIP(c, dev_alloc(&L.nu, nl));
  RT_HIP(c, dev_alloc(&L.gamma, nl));
  RT_HIP(c, dev_alloc(&L.nexp, nl));
  RT_HIP(c, dev_alloc(&L.prof16, (size_t)nl * 16));
  RT_HIP(c, dev_alloc(&L.E2p, nl));
  RT_HIP(c, dev_alloc(&L.nup, nl));
  {
    double** d64[6] = {&L.r64, &L.S64, &L.g64, &L.n64, &L.aE, &L.rN};
    const std::vector<double>* h64[6] = {&hr64, &hS64, &hg64, &hn64, &haE, &hrN};
    for (int k = 0; k < 6; ++k) {
      RT_HIP(c, dev_alloc(d64[k], nl));
      if (nl > 0)
        RT_HIP(c, hipMemcpy(*d64[k], h64[k]->data(), nl * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  // per 256-point tile, the lines with m in [256 t - 8, 256 t + 255 + 7]
  const int n_t16 = (n_nu + 255) / 256;
  std::vector<int2> ht16(n_t16);
  for (int t = 0, lo = 0, hi = 0; t < n_t16; ++t) {
    while (lo < nl && hm[lo] < 256 * t - 8) ++lo;
    if (hi < lo) hi = lo;
    while (hi < nl && hm[hi] <= 256 * t + 262) ++hi;
    ht16[t] = make_int2(lo, hi);
  }
  RT_HIP(c, dev_alloc(&L.tile16, (size_t)n_t16));
  RT_HIP(c, hipMemcpy(L.tile16, ht16.data(), (size_t)n_t16 * sizeof(int2), hipMemcpyHostToDevice));
  L.n_tiles16 = n_t16;
  // per 64-point span, the four line-range bounds of LineSet::span4 (the
  // window bounds are non-decreasing along the sorted list)
  const int n_sp = (nl > 0 ? std::max(0, hwhi[nl - 1]) : 0) / 64 + 2;
  std::vector<int4> hsp(n_sp);
  for (int b = 0; b < n_sp; ++b) {
    const int v0 = 64 * b, v1 = 64 * b + 63;
    auto ge = [&](const std::vector<int32_t>& a, int v) {
      return (int)(std::lower_bound(a.begin(), a.end(), v) - a.begin());
    };
    auto gt = [&](const std::vector<int32_t>& a, int v) {
      return (int)(std::upper_bound(a.begin(), a.end(), v) - a.begin());
    };
    hsp[b] = make_int4(ge(hwhi, v0), gt(hwlo, v1), ge(hwhi, v1), gt(hwlo, v0));
  }
  RT_HIP(c, dev_alloc(&L.span4, (size_t)n_sp));
  RT_HIP(c, hipMemcpy(L.span4, hsp.data(), (size_t)n_sp * sizeof(int4), hipMemcpyHostToDevice));
  L.n_spans = n_sp;
  if (nl > 0) {
    RT_HIP(c, hipMemcpy(L.prof16, hprof.data(), (size_t)nl * 16 * sizeof(float), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.m, hm.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.phi, hphi.data(), nl * sizeof(float), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.wlo, hwlo.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.whi, hwhi.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.S, hS.data(), nl * sizeof(float), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.E2, hE2.data(), nl * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.nu, hnu.data(), nl * sizeof(double), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.gamma, hg.data(), nl * sizeof(float), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.nexp, hn.data(), nl * sizeof(float), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.E2p, hE2p.data(), nl * sizeof(float2), hipMemcpyHostToDevice));
    RT_HIP(c, hipMemcpy(L.nup, hnup.data(), nl * sizeof(float2), hipMemcpyHostToDevice));
  }
  L.n = nl;
  return RT_OK;
}

rt_status rt_setup_lines(rt_ctx c, int n_lines, const double* nu, const double* S,
                         const double* gamma, const double* n_T, const double* E,
                         double T_ref, double cutoff, double nu0, double dnu, int n_nu) {
  if (!c) return fail(c, RT_EINVAL, "rt_setup_lines: NULL handle");
  if (n_lines < 0) return fail(c, RT_EINVAL, "rt_setup_lines: n_lines must be >= 0");
  if (n_nu < 1) return fail(c, RT_EINVAL, "rt_setup_lines: n_nu must be >= 1");
  if (!(dnu > 0) || !std::isfinite(dnu) || !(nu0 > 0) || !std::isfinite(nu0))
    return fail(c, RT_EINVAL, "rt_setup_lines: dnu and nu0 must be finite and > 0");
  if (!(T_ref > 0) || !std::isfinite(T_ref)) return fail(c, RT_EINVAL, "rt_setup_lines: T_ref must be > 0");
  if (!(cutoff >= 0) || !std::isfinite(cutoff)) return fail(c, RT_EINVAL, "rt_setup_lines: cutoff must be >= 0");
  const double Kd = cutoff / dnu;
  const double Kr = std::floor(Kd + 0.5);
  if (std::fabs(Kd - Kr) > 1e-9 * std::max(Kr, 1.0))
    return fail(c, RT_EINVAL, "rt_setup_lines: cutoff/dnu must be an integer");
  if ((double)n_nu + 2.0 * Kr + 2.0 >= 16777216.0)
    return fail(c, RT_EINVAL, "rt_setup_lines: n_nu + 2*cutoff/dnu must stay below 2^24");
  const int K = (int)Kr;
  if (c->device < 0) {  // host-only: check the lines, record the spectral grid
    if (rt_status s = check_line_arrays(c, "rt_setup_lines", n_lines, nu, S, gamma, n_T, E))
      return s;
    free_gases(c);
    c->have_E = E != nullptr;
    c->n_nu = n_nu;
    c->K = K;
    c->nu0 = nu0;
    c->dnu = dnu;
    c->T_ref = T_ref;
    c->have_lines = true;
    c->have_kappa = false;
    c->cells_valid = false;
    c->cells32_valid = false;
    return RT_OK;
  }
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, hipStreamSynchronize(c->stream));
  free_lines(c);
  free_gases(c);  // their lines were placed on the previous spectral grid
  c->have_lines = false;
  c->have_kappa = false;
  c->cells_valid = false;
  c->cells32_valid = false;
  double evals = 0;
  if (rt_status s = build_lines(c, "rt_setup_lines", n_lines, nu, S, gamma, n_T, E, T_ref, K,
                                nu0, dnu, n_nu, c->lines, evals)) {
    free_lines(c);
    return s;
  }
  c->have_E = E != nullptr;
  c->n_nu = n_nu;
  c->K = K;
  c->nu0 = nu0;
  c->dnu = dnu;
  c->T_ref = T_ref;
  c->line_evals_per_cell = evals;
  c->have_lines = true;
  return RT_OK;
}

rt_status rt_setup_gas(rt_ctx c, int gas, const double* x, int n_lines, const double* nu,
                       const double* S, const double* gamma, const double* n_T,
                       const double* E) {
  if (!c) return fail(c, RT_EINVAL, "rt_setup_gas: NULL handle");
  if (gas < 1 || gas >= rt::kMaxGases)
    return fail(c, RT_EINVAL, "rt_setup_gas: gas must be in 1.." + std::to_string(rt::kMaxGases - 1));
  if (!c->have_grid || !c->have_lines)
    return fail(c, RT_ESTATE, "rt_setup_gas: call rt_setup_grid and rt_setup_lines first");
  if (n_lines < 0) return fail(c, RT_EINVAL, "rt_setup_gas: n_lines must be >= 0");
  if (n_lines > 0) {
    if (!x) return fail(c, RT_EINVAL, "rt_setup_gas: NULL mole fractions");
    for (int64_t k = 0; k < c->n_cells; ++k)
      if (!(x[k] >= 0 && x[k] <= 1))
        return fail(c, RT_EINVAL, "rt_setup_gas: mole fractions must be in [0, 1]");
  }
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, hipStreamSynchronize(c->stream));
  rt::ExtraGas& g = c->gas[gas - 1];
  free_lineset(g.lines);
  dev_free(g.x);
  dev_free(g.G);
  dev_free(g.uf);
  dev_free(g.Gq);
  g = rt::ExtraGas();
  c->have_kappa = false;
  c->cells_valid = false;
  c->cells32_valid = false;
  if (n_lines == 0) return RT_OK;  // gas removed
  double evals = 0;
  rt_status st = build_lines(c, "rt_setup_gas", n_lines, nu, S, gamma, n_T, E, c->T_ref, c->K,
                             c->nu0, c->dnu, c->n_nu, g.lines, evals);
  if (st == RT_OK) {
    hipError_t e = dev_alloc(&g.x, (size_t)c->n_cells);
    if (e == hipSuccess) e = dev_alloc(&g.G, (size_t)c->n_cells);
    if (e == hipSuccess) e = dev_alloc(&g.uf, (size_t)c->n_cells);
    if (e == hipSuccess) e = dev_alloc(&g.Gq, (size_t)c->n_cells);
    if (e == hipSuccess)
      e = hipMemcpy(g.x, x, (size_t)c->n_cells * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) st = hip_fail(c, e, "rt_setup_gas: device arrays");
  }
  if (st != RT_OK) {
    free_lineset(g.lines);
    dev_free(g.x);
    dev_free(g.G);
    dev_free(g.uf);
    dev_free(g.Gq);
    g = rt::ExtraGas();
    return st;
  }
  g.hx.assign(x, x + c->n_cells);
  g.have_E = E != nullptr;
  g.line_evals_per_cell = evals;
  g.active = true;
  return RT_OK;
}

int rt_march_chunk(void) { return rt::kChunk; }

rt_status rt_arith_eval(rt_ctx c, int op, const float* a, const float* b, const float* z,
                        float* out, int64_t n) {
  if (!c) return fail(c, RT_EINVAL, "rt_arith_eval: NULL handle");
  const int k = rt::arith_operands(op);
  if (k == 0) return fail(c, RT_EINVAL, "rt_arith_eval: unknown op");
  if (n < 0) return fail(c, RT_EINVAL, "rt_arith_eval: n < 0");
  if (n == 0) return RT_OK;
  if (!out || !a || (k >= 2 && !b) || (k >= 3 && !z))
    return fail(c, RT_EINVAL, "rt_arith_eval: NULL operand or output");
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, rt::launch_arith(c, op, a, k >= 2 ? b : nullptr, k >= 3 ? z : nullptr, out, n));
  return RT_OK;
}

int64_t rt_required_pitch(rt_ctx c) {
  if (!c || !c->have_lines) return -1;
  return ((int64_t)c->n_nu + rt::kChunk - 1) / rt::kChunk * rt::kChunk;
}

rt_status rt_set_line_tolerance(rt_ctx c, double eps) {
  if (!c) return fail(c, RT_EINVAL, "rt_set_line_tolerance: NULL handle");
  if (!(eps > 0 && eps < 1)) return fail(c, RT_EINVAL, "rt_set_line_tolerance: eps must be in (0, 1)");
  c->line_tol = eps;
  return RT_OK;
}

// The FP64-derived cell factors (c->cells: G, beta, theta, lam2, P and the
// further gases' G), formed once per grid and line list.
static rt_status ensure_cells(rt_ctx c) {
  if (c->cells_valid) return RT_OK;
  RT_HIP(c, rt::launch_cell_params(c));
  for (int g = 1; g < rt::kMaxGases; ++g)
    if (c->gas[g - 1].active) RT_HIP(c, rt::launch_gas_factor(c, g));
  c->cells_valid = true;
  return RT_OK;
}

rt_status rt_compute_kappa(rt_ctx c, int mode, float* kappa_dev, float* planck_dev, int64_t ld) {
  if (!c) return fail(c, RT_EINVAL, "rt_compute_kappa: NULL handle");
  if (!c->have_grid || !c->have_lines)
    return fail(c, RT_ESTATE, "rt_compute_kappa: call rt_setup_grid and rt_setup_lines first");
  if (mode != RT_KAPPA_PLAIN && mode != RT_KAPPA_COMPENSATED && mode != RT_KAPPA_SURROGATE &&
      mode != RT_KAPPA_TABLE16 && mode != RT_KAPPA_ADAPTIVE && mode != RT_KAPPA_ADAPTIVE_WINGS)
    return fail(c, RT_EINVAL, "rt_compute_kappa: unknown mode");
  const bool adaptive = mode == RT_KAPPA_ADAPTIVE || mode == RT_KAPPA_ADAPTIVE_WINGS;
  if (adaptive) {
    if (!(c->line_tol > 0))
      return fail(c, RT_ESTATE, "rt_compute_kappa: call rt_set_line_tolerance before the adaptive mode");
    if (n_gases(c) > 1)
      return fail(c, RT_EUNSUPPORTED, "rt_compute_kappa: the adaptive windows cover gas 0 only");
    if (c->K > 32767)
      return fail(c, RT_EUNSUPPORTED, "rt_compute_kappa: the adaptive windows need cutoff/dnu <= 32767");
  }
  if (mode == RT_KAPPA_SURROGATE &&
      (!c->surrogate || !rt::surrogate_ready(c)))
    return fail(c, RT_ESTATE, "rt_compute_kappa: no trained surrogate for this spectral grid");
  if (mode == RT_KAPPA_TABLE16 && c->K < 8)
    return fail(c, RT_EUNSUPPORTED, "rt_compute_kappa: the 16-point form needs cutoff >= 8 dnu "
                                    "(its points must lie within the kept lines' windows)");
  if (mode == RT_KAPPA_SURROGATE && n_gases(c) > 1)
    return fail(c, RT_EUNSUPPORTED, "rt_compute_kappa: the surrogate covers gas 0 only");
  if (!kappa_dev) return fail(c, RT_EINVAL, "rt_compute_kappa: NULL kappa buffer");
  if (ld < rt_required_pitch(c) || ld % rt::kChunk != 0)
    return fail(c, RT_EINVAL, "rt_compute_kappa: ld must be a multiple of the march chunk (rt_required_pitch) and >= it");
  if ((reinterpret_cast<uintptr_t>(kappa_dev) | reinterpret_cast<uintptr_t>(planck_dev)) & 15)
    return fail(c, RT_EINVAL, "rt_compute_kappa: buffers must be 16-byte aligned");
  if (rt_status s = set_device(c)) return s;
  c->have_kappa = false;
  if (c->bwall_len < ld) {
    dev_free(c->d_bwall);
    RT_HIP(c, dev_alloc(&c->d_bwall, (size_t)ld));
    c->bwall_len = ld;
  }
  if (adaptive) {
    const int64_t runs = (c->n_cells + RT_ADAPTIVE_GROUP - 1) / RT_ADAPTIVE_GROUP;
    const int64_t win = runs * (int64_t)std::max(c->lines.n, 1);
    if (c->sbar_cap < c->n_cells) {  // per cell: 2 doubles, an 8-float record, the wing constant
      dev_free(c->d_sbar);
      c->sbar_cap = 0;
      RT_HIP(c, dev_alloc(&c->d_sbar, (size_t)(rt::kAdaptiveCellDoubles * c->n_cells)));
      c->sbar_cap = c->n_cells;
    }
    // room for 1/16 of the windows to be left to binary64 (about 0.3% are
    // at eps = 1e-5 on a 32^3 grid); any beyond are found by a scan
    const int64_t und = std::max<int64_t>(4096, win / 16);
    if (c->und_cap < und) {
      dev_free(c->d_und);
      c->und_cap = 0;
      RT_HIP(c, dev_alloc(&c->d_und, (size_t)(und + 1)));
      c->und_cap = und;
    }
    if (c->win_cap < win) {
      dev_free(c->d_win);
      c->win_cap = 0;
      RT_HIP(c, dev_alloc(&c->d_win, (size_t)win));
      c->win_cap = win;
    }
  }
  c->kappa = kappa_dev;
  c->planck = planck_dev;
  c->ld = ld;
  if (!c->cells32_valid) {  // the precision form's line sum, the Planck table, the walls
    if (rt_status s = upload_cells32(c)) return s;
    RT_HIP(c, rt::launch_cell_params32(c));
    c->cells32_valid = true;
  }
  if (rt_status s = record_begin(c, c->kappa_events)) return s;
  // the FP64-derived cell factors serve every form but the precision form,
  // whose line sum runs on its FP32 inputs alone
  if (mode != RT_KAPPA_COMPENSATED)
    if (rt_status s = ensure_cells(c)) return s;
  if (mode == RT_KAPPA_SURROGATE) {
    if (rt_status s = rt::surrogate_kappa(c)) return s;
  } else if (mode == RT_KAPPA_TABLE16) {
    RT_HIP(c, rt::launch_kappa_table16(c));
  } else if (mode == RT_KAPPA_ADAPTIVE) {
    RT_HIP(c, rt::launch_kappa_adaptive(c));
  } else if (mode == RT_KAPPA_ADAPTIVE_WINGS) {
    RT_HIP(c, rt::launch_kappa_adaptive_wings(c));
  } else {
    RT_HIP(c, rt::launch_kappa(c, mode == RT_KAPPA_COMPENSATED));
  }
  if (rt_status s = record_end(c, c->kappa_events)) return s;
  // wall row always (the learned form writes it in its first launch); cell
  // table if requested
  if (mode != RT_KAPPA_SURROGATE || c->planck) RT_HIP(c, rt::launch_planck(c));
  if (mode == RT_KAPPA_TABLE16) {
    double lines = c->lines.n;
    for (const auto& g : c->gas)
      if (g.active) lines += g.lines.n;
    c->stats.line_evals += 16.0 * lines * (double)c->n_cells;
  } else if (mode != RT_KAPPA_SURROGATE && !adaptive) {
    // (the adaptive windows count their kept evaluations on the device)
    double per_cell = c->line_evals_per_cell;
    for (const auto& g : c->gas)
      if (g.active) per_cell += g.line_evals_per_cell;
    c->stats.line_evals += per_cell * (double)c->n_cells;
  }
  c->have_kappa = true;
  return RT_OK;
}

// Traces rays [begin, begin + count) batch by batch through the ray scratch
// rs.  timed: record the HIP events rt_get_stats reads (the entry point that
// allocates nothing records none).
static rt_status trace_with(rt_ctx c, const rt::RayScratch& rs, uint64_t seed, uint64_t begin,
                            uint64_t count, double weight, bool f64, bool explicit_rays,
                            float* exit_dev, bool timed) {
  if (timed)
    if (rt_status s = record_begin(c, c->trace_events)) return s;
  // A launch adds at most (rays x chunks) terms to one accumulator word
  // (a ray crosses a cell once); the words are normalised after every launch.
  const int64_t n_chunks = std::max<int64_t>(1, c->ld / rt::kChunk);
  const int64_t per_launch =
      std::max<int64_t>(1, std::min<int64_t>(rs.cap, rt::kAccMaxTerms / n_chunks));
  for (uint64_t off = 0; off < count; off += (uint64_t)per_launch) {
    const int64_t n = (int64_t)std::min<uint64_t>((uint64_t)per_launch, count - off);
    if (explicit_rays && off > 0) return fail(c, RT_EINVAL, "explicit rays exceed one batch");
    const bool order = !explicit_rays && n >= rt::kOrderMinRays;
    if (order) RT_HIP(c, rt::launch_order(c, rs, seed, begin + off, n));
    RT_HIP(c, rt::launch_raygen(c, rs, seed, begin + off, n, explicit_rays, nullptr, true,
                                order ? rs.perm : nullptr));
    if (timed)
      if (rt_status s = record_begin(c, c->march_events)) return s;
    RT_HIP(c, rt::launch_march(c, rs, n, weight, f64, exit_dev));
    if (timed)
      if (rt_status s = record_end(c, c->march_events)) return s;
    c->stats.march_launches += 1;
  }
  if (timed)
    if (rt_status s = record_end(c, c->trace_events)) return s;
  c->stats.rays += (double)count;
  return RT_OK;
}

static rt_status trace_batches(rt_ctx c, uint64_t seed, uint64_t begin, uint64_t count,
                               double weight, bool f64, bool explicit_rays, float* exit_dev) {
  if (rt_status s = ensure_batch(c, (int64_t)count)) return s;
  return trace_with(c, rt::owned_rays(c), seed, begin, count, weight, f64, explicit_rays,
                    exit_dev, true);
}

// Checks shared by rt_trace_rays and rt_trace_rays_noalloc.  The plain march
// reads c2/T of the FP64-derived cell factors, which a compute_kappa in the
// precision form does not form.
static rt_status check_trace(rt_ctx c, const char* who, uint64_t n_rays_total,
                             uint64_t ray_begin, uint64_t ray_count, int tally_prec) {
  const std::string w(who);
  if (!c->have_kappa) return fail(c, RT_ESTATE, w + ": call rt_compute_kappa first");
  if (n_rays_total == 0) return fail(c, RT_EINVAL, w + ": n_rays_total must be >= 1");
  if (ray_begin > n_rays_total || ray_count > n_rays_total - ray_begin)
    return fail(c, RT_EINVAL, w + ": ray range outside [0, n_rays_total)");
  if (tally_prec != RT_TALLY_F32 && tally_prec != RT_TALLY_F64)
    return fail(c, RT_EINVAL, w + ": unknown tally precision");
  if (tally_prec == RT_TALLY_F64 && !c->planck)
    return fail(c, RT_ESTATE, w + ": the precision form needs the Planck table "
                                  "(pass planck_dev to rt_compute_kappa)");
  if (tally_prec == RT_TALLY_F32)
    if (rt_status s = set_device(c)) return s;
  return tally_prec == RT_TALLY_F32 ? ensure_cells(c) : RT_OK;
}

rt_status rt_trace_rays(rt_ctx c, uint64_t seed, uint64_t n_rays_total, uint64_t ray_begin,
                        uint64_t ray_count, int tally_prec) {
  if (!c) return fail(c, RT_EINVAL, "rt_trace_rays: NULL handle");
  if (rt_status s = check_trace(c, "rt_trace_rays", n_rays_total, ray_begin, ray_count, tally_prec))
    return s;
  if (ray_count == 0) return RT_OK;
  if (rt_status s = set_device(c)) return s;
  return trace_batches(c, seed, ray_begin, ray_count, ray_weight(c, (double)n_rays_total),
                       tally_prec == RT_TALLY_F64, false, nullptr);
}

rt_status rt_trace_rays_noalloc(rt_ctx c, uint64_t seed, uint64_t n_rays_total,
                                uint64_t ray_begin, uint64_t ray_count, int tally_prec) {
  if (!c) return fail(c, RT_EINVAL, "rt_trace_rays_noalloc: NULL handle");
  if (rt_status s = check_trace(c, "rt_trace_rays_noalloc", n_rays_total, ray_begin, ray_count,
                                tally_prec))
    return s;
  if (!c->noalloc_scratch)
    return fail(c, RT_ESTATE, "rt_trace_rays_noalloc: no device scratch for this handle");
  // carve the static scratch: histogram, then per ray count, key and
  // permutation words, then the segments
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  const int max_segs = c->nx + c->ny + c->nz;
  const size_t hist_bytes = up((size_t)rt::kOrderBuckets * 4);
  const size_t per_ray = 12 + 8 * (size_t)max_segs;
  const size_t room = kNoAllocBytes - hist_bytes - 3 * 256;  // 3 alignment gaps
  const int64_t cap = std::min<int64_t>((int64_t)(room / per_ray), int64_t(1) << 21) / 256 * 256;
  if (cap < 256)
    return fail(c, RT_EINVAL, "rt_trace_rays_noalloc: the grid's traversals (nx+ny+nz = " +
                                  std::to_string(max_segs) + " segments per ray) do not fit 256 rays "
                                  "in the 64 MiB device scratch");
  if (ray_count == 0) return RT_OK;
  if (rt_status s = set_device(c)) return s;
  char* base = static_cast<char*>(c->noalloc_scratch);
  rt::RayScratch rs;
  size_t off = 0;
  rs.hist = reinterpret_cast<uint32_t*>(base + off);
  off += hist_bytes;
  rs.counts = reinterpret_cast<int32_t*>(base + off);
  off += up((size_t)cap * 4);
  rs.keys = reinterpret_cast<uint32_t*>(base + off);
  off += up((size_t)cap * 4);
  rs.perm = reinterpret_cast<uint32_t*>(base + off);
  off += up((size_t)cap * 4);
  rs.segs = reinterpret_cast<int2*>(base + off);
  off += (size_t)cap * max_segs * 8;
  if (off > kNoAllocBytes) return fail(c, RT_EINVAL, "rt_trace_rays_noalloc: scratch layout");
  rs.max_segs = max_segs;
  rs.cap = cap;
  return trace_with(c, rs, seed, ray_begin, ray_count, ray_weight(c, (double)n_rays_total),
                    tally_prec == RT_TALLY_F64, false, nullptr, false);
}

rt_status rt_trace_explicit(rt_ctx c, int n_rays, const int64_t* O, const int64_t* D,
                            double weight, int tally_prec, double* exit_I) {
  if (!c) return fail(c, RT_EINVAL, "rt_trace_explicit: NULL handle");
  if (!c->have_kappa) return fail(c, RT_ESTATE, "rt_trace_explicit: call rt_compute_kappa first");
  if (n_rays < 1 || !O || !D) return fail(c, RT_EINVAL, "rt_trace_explicit: bad ray arrays");
  if (!(weight >= 0 && weight <= 0x1p40))
    return fail(c, RT_EINVAL, "rt_trace_explicit: weight must be in [0, 2^40]");
  if (tally_prec != RT_TALLY_F32 && tally_prec != RT_TALLY_F64)
    return fail(c, RT_EINVAL, "rt_trace_explicit: unknown tally precision");
  if (tally_prec == RT_TALLY_F64 && !c->planck)
    return fail(c, RT_ESTATE, "rt_trace_explicit: the precision form needs the Planck table");
  if (rt_status s = ensure_batch(c, n_rays)) return s;
  if (n_rays > c->batch_rays) return fail(c, RT_EINVAL, "rt_trace_explicit: too many rays");
  const int64_t lim[3] = {c->nx * rt::kCellUnits, c->ny * rt::kCellUnits, c->nz * rt::kCellUnits};
  std::vector<int64_t> buf((size_t)n_rays * 6);
  for (int r = 0; r < n_rays; ++r) {
    bool on_face = false, inward = false, any = false;
    for (int k = 0; k < 3; ++k) {
      const int64_t o = O[3 * r + k], d = D[3 * r + k];
      if (o < 0 || o > lim[k]) return fail(c, RT_EINVAL, "rt_trace_explicit: origin outside the box");
      if (d < -rt::kCellUnits || d > rt::kCellUnits)
        return fail(c, RT_EINVAL, "rt_trace_explicit: |D| components must be <= 2^21");
      if (d != 0) any = true;
      if (o == 0 || o == lim[k]) {
        on_face = true;
        if ((o == 0 && d > 0) || (o == lim[k] && d < 0)) inward = true;
      }
      buf[6 * r + k] = o;
      buf[6 * r + 3 + k] = d;
    }
    if (!any || !on_face || !inward)
      return fail(c, RT_EINVAL, "rt_trace_explicit: rays must start on a face and point inward");
    for (int k = 0; k < 3; ++k) {
      const int64_t o = O[3 * r + k], d = D[3 * r + k];
      if ((o == 0 && d < 0) || (o == lim[k] && d > 0))
        return fail(c, RT_EINVAL, "rt_trace_explicit: ray leaves through its own face");
    }
  }
  if (rt_status s = set_device(c)) return s;
  if (tally_prec == RT_TALLY_F32)
    if (rt_status s = ensure_cells(c)) return s;
  if (c->explicit_cap < n_rays) {
    dev_free(c->d_rays_explicit);
    RT_HIP(c, dev_alloc(&c->d_rays_explicit, (size_t)n_rays * 6));
    c->explicit_cap = n_rays;
  }
  RT_HIP(c, hipMemcpyAsync(c->d_rays_explicit, buf.data(), buf.size() * sizeof(int64_t),
                           hipMemcpyHostToDevice, c->stream));
  float* exit_dev = nullptr;
  if (exit_I) {
    const int64_t need = (int64_t)n_rays * c->ld;
    if (c->exit_cap < need) {
      dev_free(c->d_exit);
      RT_HIP(c, dev_alloc(&c->d_exit, (size_t)need));
      c->exit_cap = need;
    }
    exit_dev = c->d_exit;
  }
  if (rt_status s = trace_batches(c, 0, 0, (uint64_t)n_rays, weight, tally_prec == RT_TALLY_F64,
                                  true, exit_dev))
    return s;
  RT_HIP(c, hipStreamSynchronize(c->stream));  // the host ray buffer goes out of scope
  if (exit_I) {
    std::vector<float> tmp((size_t)n_rays * c->ld);
    RT_HIP(c, hipMemcpy(tmp.data(), exit_dev, tmp.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int r = 0; r < n_rays; ++r)
      for (int j = 0; j < c->n_nu; ++j) exit_I[(size_t)r * c->n_nu + j] = tmp[(size_t)r * c->ld + j];
  }
  return RT_OK;
}

rt_status rt_tally(rt_ctx c, double* absorbed, double* emitted, double* balance) {
  if (!c) return fail(c, RT_EINVAL, "rt_tally: NULL handle");
  if (!c->have_grid) return fail(c, RT_ESTATE, "rt_tally: call rt_setup_grid first");
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, rt::launch_tally(c));
  if (absorbed)
    RT_HIP(c, hipMemcpyAsync(absorbed, c->d_abs, c->n_cells * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (emitted)
    RT_HIP(c, hipMemcpyAsync(emitted, c->d_emi, c->n_cells * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  double bal[4];
  unsigned ovf = 0;
  RT_HIP(c, hipMemcpyAsync(bal, c->d_balance, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  RT_HIP(c, hipMemcpyAsync(&ovf, c->d_ovf, sizeof(ovf), hipMemcpyDeviceToHost, c->stream));
  RT_HIP(c, hipStreamSynchronize(c->stream));
  if (ovf)
    return fail(c, RT_EDEVICE, "rt_tally: a tallied power was negative, not finite or not below 2^80 W");
  if (balance) std::memcpy(balance, bal, sizeof(bal));
  return RT_OK;
}

rt_status rt_reset_tally(rt_ctx c) {
  if (!c) return fail(c, RT_EINVAL, "rt_reset_tally: NULL handle");
  if (!c->have_grid) return fail(c, RT_ESTATE, "rt_reset_tally: call rt_setup_grid first");
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, rt::launch_zero(c));
  RT_HIP(c, hipMemsetAsync(c->d_adapt_evals, 0, sizeof(unsigned long long), c->stream));
  double tmp = 0;
  if (rt_status s = drain_events(c, c->trace_events, &tmp)) return s;
  if (rt_status s = drain_events(c, c->march_events, &tmp)) return s;
  if (rt_status s = drain_events(c, c->kappa_events, &tmp)) return s;
  c->stats.kappa_ms = 0;
  c->stats.line_evals = 0;
  c->stats.trace_ms = 0;
  c->stats.march_ms = 0;
  c->stats.rays = 0;
  c->stats.march_launches = 0;
  return RT_OK;
}

rt_status rt_debug_segments(rt_ctx c, uint64_t seed, uint64_t ray_begin, uint64_t count,
                            int max_segs, int32_t* counts, int32_t* cells, float* len_cm,
                            int64_t* O, int64_t* D) {
  if (!c) return fail(c, RT_EINVAL, "rt_debug_segments: NULL handle");
  if (!c->have_grid) return fail(c, RT_ESTATE, "rt_debug_segments: call rt_setup_grid first");
  if (!counts || !cells || !len_cm) return fail(c, RT_EINVAL, "rt_debug_segments: NULL output");
  if (max_segs < c->nx + c->ny + c->nz) return fail(c, RT_EINVAL, "rt_debug_segments: max_segs < nx+ny+nz");
  if (rt_status s = set_device(c)) return s;
  if (rt_status s = ensure_batch(c, (int64_t)count)) return s;
  if (c->explicit_cap < c->batch_rays) {
    dev_free(c->d_rays_explicit);
    RT_HIP(c, dev_alloc(&c->d_rays_explicit, (size_t)c->batch_rays * 6));
    c->explicit_cap = c->batch_rays;
  }
  std::vector<int2> seg;
  std::vector<int32_t> cnt;
  std::vector<int64_t> rays;
  for (uint64_t off = 0; off < count; off += (uint64_t)c->batch_rays) {
    const int64_t n = (int64_t)std::min<uint64_t>((uint64_t)c->batch_rays, count - off);
    RT_HIP(c, rt::launch_raygen(c, rt::owned_rays(c), seed, ray_begin + off, n, false,
                                c->d_rays_explicit, false,
                                nullptr));
    seg.resize((size_t)n * c->max_segs);
    cnt.resize((size_t)n);
    rays.resize((size_t)n * 6);
    RT_HIP(c, hipMemcpyAsync(seg.data(), c->d_segs, seg.size() * sizeof(int2), hipMemcpyDeviceToHost, c->stream));
    RT_HIP(c, hipMemcpyAsync(cnt.data(), c->d_counts, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    RT_HIP(c, hipMemcpyAsync(rays.data(), c->d_rays_explicit, rays.size() * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    RT_HIP(c, hipStreamSynchronize(c->stream));
    for (int64_t r = 0; r < n; ++r) {
      const int64_t g = (int64_t)off + r;
      counts[g] = cnt[r];
      for (int k = 0; k < cnt[r]; ++k) {
        cells[g * max_segs + k] = seg[r * c->max_segs + k].x;
        int bits = seg[r * c->max_segs + k].y;
        std::memcpy(&len_cm[g * max_segs + k], &bits, sizeof(float));
      }
      for (int k = 0; k < 3; ++k) {
        if (O) O[3 * g + k] = rays[6 * r + k];
        if (D) D[3 * g + k] = rays[6 * r + 3 + k];
      }
    }
  }
  return RT_OK;
}

rt_status rt_get_stats(rt_ctx c, rt_stats* out) {
  if (!c || !out) return fail(c, RT_EINVAL, "rt_get_stats: NULL argument");
  if (rt_status s = set_device(c)) return s;
  RT_HIP(c, hipStreamSynchronize(c->stream));
  if (rt_status s = drain_events(c, c->kappa_events, &c->stats.kappa_ms)) return s;
  if (rt_status s = drain_events(c, c->trace_events, &c->stats.trace_ms)) return s;
  if (rt_status s = drain_events(c, c->march_events, &c->stats.march_ms)) return s;
  unsigned long long segs = 0, kept = 0;
  if (c->d_segcount)
    RT_HIP(c, hipMemcpy(&segs, c->d_segcount, sizeof(segs), hipMemcpyDeviceToHost));
  if (c->d_adapt_evals)
    RT_HIP(c, hipMemcpy(&kept, c->d_adapt_evals, sizeof(kept), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->line_evals = c->stats.line_evals + (double)kept;
  out->kappa_ms = c->stats.kappa_ms;
  out->segments = (double)segs;
  out->updates = (double)segs * (double)c->n_nu;
  out->trace_ms = c->stats.trace_ms;
  out->march_ms = c->stats.march_ms;
  out->rays = c->stats.rays;
  out->march_launches = c->stats.march_launches;
  out->batch_line_evals = c->stats.batch_line_evals;
  out->batch_updates = c->stats.batch_updates;
  out->batch_ms = c->stats.batch_ms;
  return RT_OK;
}

}  // extern "C"
