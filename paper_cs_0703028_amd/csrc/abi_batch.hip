// abi_batch.hip -- host side of the batched form: validation, the work
// plan, carving of the caller's workspace, HIP graph capture of the launch
// sequence, and the autotuner with its JSON cache.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "batch_plan.h"
#include "device_common.h"

namespace {

using namespace rt;

rt_status bfail(rt_ctx c, rt_status s, const std::string& m) {
  c->err = m;
  return s;
}

#define RT_BHIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return (void)hipGetLastError(), /* not left for the next launch check */          \
             bfail(ctx, (e_ == hipErrorOutOfMemory) ? RT_ENOMEM : RT_EDEVICE,           \
                   std::string(#call) + ": " + hipGetErrorString(e_));                  \
  } while (0)

rt_batch_tuning default_tuning() {
  rt_batch_tuning t;
  t.chunk_points = 2 * kChunk;
  t.kappa_groups = 16;
  t.march_rays = 64;
  t.blocks_per_cu = 2;
  t.slots = 1;
  t.mode = RT_BATCH_CHUNKED;
  return t;
}

rt_status check_tuning(rt_ctx c, const rt_batch_tuning& t) {
  if (t.chunk_points < kChunk || t.chunk_points % kChunk != 0 || t.chunk_points > (1 << 20))
    return bfail(c, RT_EINVAL, "rt_batch: chunk_points must be a positive multiple of " +
                                   std::to_string(kChunk));
  if (t.mode != RT_BATCH_CHUNKED && t.mode != RT_BATCH_PERSISTENT)
    return bfail(c, RT_EINVAL, "rt_batch: mode must be RT_BATCH_CHUNKED or RT_BATCH_PERSISTENT");
  if (t.mode == RT_BATCH_CHUNKED) {  // kappa_groups, march_rays, blocks_per_cu unused
    if (t.slots < 1 || t.slots > 8) return bfail(c, RT_EINVAL, "rt_batch: slots must be in 1..8");
    return RT_OK;
  }
  if (t.kappa_groups < 1 || t.kappa_groups > (1 << 20))
    return bfail(c, RT_EINVAL, "rt_batch: kappa_groups must be >= 1");
  if (t.march_rays < 4 || t.march_rays % 4 != 0 || t.march_rays > (1 << 20))
    return bfail(c, RT_EINVAL, "rt_batch: march_rays must be a positive multiple of 4");
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 8)
    return bfail(c, RT_EINVAL, "rt_batch: blocks_per_cu must be in 1..8");
  if (t.slots < 2 || t.slots > 8) return bfail(c, RT_EINVAL, "rt_batch: slots must be in 2..8");
  return RT_OK;
}

rt_status check_cases(rt_ctx c, int n_cases, const rt_case* cases) {
  if (n_cases < 1 || !cases) return bfail(c, RT_EINVAL, "rt_batch: need at least one case");
  if (!c->have_lines) return bfail(c, RT_ESTATE, "rt_batch: call rt_setup_lines first");
  int64_t total = 0;
  for (int k = 0; k < n_cases; ++k) {
    const rt_case& q = cases[k];
    if (q.nx < 1 || q.ny < 1 || q.nz < 1 || q.nx > kMaxAxis || q.ny > kMaxAxis || q.nz > kMaxAxis)
      return bfail(c, RT_EINVAL, "rt_batch: case grid sizes must be in [1, 2^20]");
    const int64_t n = (int64_t)q.nx * q.ny * q.nz;
    total += n;
    if (!(q.cell_m > 0) || !std::isfinite(q.cell_m)) return bfail(c, RT_EINVAL, "rt_batch: cell_m must be > 0");
    if (!(q.T_wall_K >= 0) || !std::isfinite(q.T_wall_K)) return bfail(c, RT_EINVAL, "rt_batch: T_wall must be >= 0");
    if (!q.T_K || !q.x_h2o || !q.p_atm) return bfail(c, RT_EINVAL, "rt_batch: NULL case array");
    if (q.n_rays < 1 || q.n_rays > (uint64_t(1) << 31)) return bfail(c, RT_EINVAL, "rt_batch: n_rays must be in [1, 2^31]");
    for (int64_t i = 0; i < n; ++i) {
      if (!(q.T_K[i] > 0) || !std::isfinite(q.T_K[i])) return bfail(c, RT_EINVAL, "rt_batch: T must be finite and > 0");
      if (!(q.x_h2o[i] >= 0 && q.x_h2o[i] <= 1)) return bfail(c, RT_EINVAL, "rt_batch: x_h2o must be in [0, 1]");
      if (!(q.p_atm[i] > 0) || !std::isfinite(q.p_atm[i])) return bfail(c, RT_EINVAL, "rt_batch: p must be finite and > 0");
    }
  }
  if (total >= (int64_t(1) << 31)) return bfail(c, RT_EINVAL, "rt_batch: total cells must be < 2^31");
  return RT_OK;
}

int64_t align_up(int64_t v) { return (v + 255) / 256 * 256; }

// Builds the plan (sizes, stages) without touching device memory; returns
// the workspace bytes through *bytes.  limit_points > 0 restricts the
// spectral range to the first limit_points points (autotuner trials).
rt_status build_plan(rt_ctx c, int n_cases, const rt_case* cases, const rt_batch_tuning& t,
                     int64_t limit_points, BatchPlan& pl, int64_t* bytes) {
  pl.tuning = t;
  pl.chunked = t.mode == RT_BATCH_CHUNKED;
  pl.n_cases = n_cases;
  const int64_t n_nu = limit_points > 0 ? std::min<int64_t>(limit_points, c->n_nu) : c->n_nu;
  pl.n_chunks = (int)((n_nu + t.chunk_points - 1) / t.chunk_points);
  pl.bwall_ld = (int64_t)pl.n_chunks * t.chunk_points;
  pl.cases.assign(n_cases, BatchCase());
  int64_t cell_off = 0, seg_off = 0, ray_off = 0, blk_off = 0, max_cells = 0;
  double evals = 0;
  double T_min = INFINITY, T_max = 0;
  for (int k = 0; k < n_cases; ++k) {
    const rt_case& q = cases[k];
    BatchCase& b = pl.cases[k];
    const int64_t nc = (int64_t)q.nx * q.ny * q.nz;
    T_min = std::min(T_min, *std::min_element(q.T_K, q.T_K + nc));
    T_max = std::max(T_max, *std::max_element(q.T_K, q.T_K + nc));
    b.nx = q.nx; b.ny = q.ny; b.nz = q.nz;
    b.max_segs = q.nx + q.ny + q.nz;
    b.n_cells = (int64_t)q.nx * q.ny * q.nz;
    b.cell_off = cell_off;
    b.n_rays = (int64_t)q.n_rays;
    // one launch adds up to rays x spectral chunks terms to a case's
    // accumulator words, which hold kAccMaxTerms until normalised
    if ((double)q.n_rays * (double)((c->n_nu + kChunk - 1) / kChunk) > (double)kAccMaxTerms)
      return bfail(c, RT_EINVAL, "rt_batch: n_rays x spectral chunks of a case must be <= 2^35");
    b.seg_off = seg_off;
    b.ray_off = ray_off;
    b.blk_off = blk_off;
    b.seed = q.seed;
    const double h = q.cell_m;
    const double area = 2.0 * h * h * ((double)q.nx * q.ny + (double)q.ny * q.nz + (double)q.nz * q.nx);
    b.weight = M_PI * area * c->dnu / (double)q.n_rays;
    b.unit_cm = q.cell_m * 100.0 / (double)kCellUnits;
    if (q.T_wall_K > 0) {
      const double th = second_radiation_cm_K() / q.T_wall_K;
      const float h = (float)th;
      b.theta_wall = make_float2(h, (float)(th - (double)h));
    } else {
      b.theta_wall = make_float2(0.f, 0.f);
    }
    cell_off += b.n_cells;
    seg_off += b.n_rays * b.max_segs;
    ray_off += b.n_rays;
    // march blocks of 4 rays, an eighth per XCD, for each kChunk part
    blk_off += (int64_t)(t.chunk_points / kChunk) * (((b.n_rays + 3) / 4 + 7) / 8);
    max_cells = std::max(max_cells, b.n_cells);
    evals += c->line_evals_per_cell * (double)b.n_cells;
  }
  pl.total_cells = cell_off;
  pl.total_rays = ray_off;
  pl.ray_blocks = blk_off;
  if (pl.chunked && 8 * blk_off > 0x7fffffffLL)
    return bfail(c, RT_EINVAL, "rt_batch: too many rays for one chunked march launch "
                               "(use RT_BATCH_PERSISTENT or fewer chunk_points)");
  pl.planck_quad = planck_needs_quadratic(T_min, T_max, c->nu0, c->dnu, c->n_nu);
  pl.max_cells = max_cells;
  pl.line_evals = limit_points > 0 ? 0.0 : evals;
  pl.slab_stride = (pl.chunked ? cell_off : max_cells) * t.chunk_points;
  const int n_slabs = t.slots;
  pl.n_pairs = n_cases * pl.n_chunks;

  // stages of the persistent queue
  pl.stages.clear();
  std::vector<int> rg_stage(n_cases), k_stage(pl.n_pairs), m_stage(pl.n_pairs);
  const int tiles = t.chunk_points / dev::kKappaTilePoints;
  auto add = [&](int kind, int cas, int chunk, int pair, int64_t count) {
    BatchStage s;
    s.kind = kind; s.cas = cas; s.chunk = chunk; s.pair = pair;
    s.slot = pair >= 0 ? pair % t.slots : 0;
    s.wait_pair = -1; s.wait_stage = -1; s.raygen_stage = -1;
    s.first = 0; s.count = count;
    pl.stages.push_back(s);
    return (int)pl.stages.size() - 1;
  };
  if (!pl.chunked)
    for (int k = 0; k < n_cases; ++k)
      rg_stage[k] = add(kStageRaygen, k, 0, -1, (pl.cases[k].n_rays + 255) / 256);
  auto pair_case = [&](int p) { return p / pl.n_chunks; };
  auto pair_chunk = [&](int p) { return p % pl.n_chunks; };
  auto add_k = [&](int p) {
    const BatchCase& b = pl.cases[pair_case(p)];
    const int64_t groups = (b.n_cells + dev::kKappaCells - 1) / dev::kKappaCells;
    k_stage[p] = add(kStageKappa, pair_case(p), pair_chunk(p), p,
                     (int64_t)tiles * ((groups + t.kappa_groups - 1) / t.kappa_groups));
  };
  auto add_m = [&](int p) {
    const BatchCase& b = pl.cases[pair_case(p)];
    m_stage[p] = add(kStageMarch, pair_case(p), pair_chunk(p), p, (b.n_rays + t.march_rays - 1) / t.march_rays);
  };
  // software pipeline over the slab ring: the line sums run slots - 1 pairs
  // ahead of the march, K(0) .. K(L-1), then K(p + L) M(p) for every p, with
  // L = slots - 1; K(p + L) reuses the slab of M(p - 1), which precedes it
  const int L = std::max(1, t.slots - 1);
  if (pl.chunked) pl.n_pairs = 0;  // no queue
  for (int p = 0; p < std::min(L, pl.n_pairs); ++p) add_k(p);
  for (int p = 0; p < pl.n_pairs; ++p) {
    if (p + L < pl.n_pairs) add_k(p + L);
    add_m(p);
  }
  for (int p = 0; p < pl.n_pairs; ++p) {
    BatchStage& ks = pl.stages[k_stage[p]];
    if (p >= t.slots) {
      ks.wait_pair = p - t.slots;
      ks.wait_stage = m_stage[p - t.slots];
    }
    BatchStage& ms = pl.stages[m_stage[p]];
    ms.wait_stage = k_stage[p];
    ms.raygen_stage = rg_stage[pair_case(p)];
  }
  int64_t first = 0;
  for (auto& s : pl.stages) { s.first = first; first += s.count; }
  pl.total_items = first;
  pl.n_stages = (int)pl.stages.size();
  pl.n_counters = 4 + n_cases + 2 * (int64_t)pl.n_pairs;

  // workspace layout
  int64_t off = 0;
  auto take = [&](int64_t b) { const int64_t o = off; off += align_up(b); return o; };
  const int64_t nc = pl.total_cells;
  int64_t o_T = take(nc * 8), o_x = take(nc * 8), o_p = take(nc * 8), o_Tw = take(n_cases * 8);
  int64_t o_G = take(nc * 4), o_beta = take(nc * 8), o_theta = take(nc * 8), o_lam2 = take(nc * 4),
          o_P = take(nc * 4);
  int64_t o_abs = take(nc * 8), o_emi = take(nc * 8);
  int64_t o_acc = take(((nc + (int64_t)n_cases * kCaseBalRows) * kAccRow + 1) * 8), o_bal = take((int64_t)n_cases * 4 * 8);
  int64_t o_bw = take((int64_t)n_cases * pl.bwall_ld * 4);
  int64_t o_segs = take(seg_off * 8), o_cnt = take(ray_off * 4);
  int64_t o_keys = take(ray_off * 4), o_perm = take(ray_off * 4);
  int64_t o_hist = take((int64_t)n_cases * kOrderBuckets * 4);
  int64_t o_slab = take((int64_t)n_slabs * pl.slab_stride * 4);
  int64_t o_ctr = take(pl.n_counters * 4);
  int64_t o_st = take((int64_t)pl.n_stages * sizeof(BatchStage));
  int64_t o_cases = take((int64_t)n_cases * sizeof(BatchCase));
  *bytes = off;
  // offsets are stored as pointers relative to a null base until carved
  pl.d_T = reinterpret_cast<double*>(o_T);
  pl.d_x = reinterpret_cast<double*>(o_x);
  pl.d_p = reinterpret_cast<double*>(o_p);
  pl.d_T_wall = reinterpret_cast<double*>(o_Tw);
  pl.cells.G = reinterpret_cast<float*>(o_G);
  pl.cells.beta = reinterpret_cast<double*>(o_beta);
  pl.cells.theta = reinterpret_cast<double*>(o_theta);
  pl.cells.lam2 = reinterpret_cast<float*>(o_lam2);
  pl.cells.P = reinterpret_cast<float*>(o_P);
  pl.d_abs = reinterpret_cast<double*>(o_abs);
  pl.d_emi = reinterpret_cast<double*>(o_emi);
  pl.d_acc = reinterpret_cast<unsigned long long*>(o_acc);
  pl.d_balance = reinterpret_cast<double*>(o_bal);
  pl.d_bwall = reinterpret_cast<float*>(o_bw);
  pl.d_segs = reinterpret_cast<int2*>(o_segs);
  pl.d_counts = reinterpret_cast<int32_t*>(o_cnt);
  pl.d_keys = reinterpret_cast<uint32_t*>(o_keys);
  pl.d_perm = reinterpret_cast<uint32_t*>(o_perm);
  pl.d_hist = reinterpret_cast<uint32_t*>(o_hist);
  pl.d_slabs = reinterpret_cast<float*>(o_slab);
  pl.d_counters = reinterpret_cast<unsigned*>(o_ctr);
  pl.d_stages = reinterpret_cast<BatchStage*>(o_st);
  pl.d_cases = reinterpret_cast<BatchCase*>(o_cases);
  return RT_OK;
}

template <class T>
void rebase(T*& p, char* base) { p = reinterpret_cast<T*>(base + reinterpret_cast<intptr_t>(p)); }

void carve(BatchPlan& pl, void* ws) {
  char* b = static_cast<char*>(ws);
  rebase(pl.d_T, b); rebase(pl.d_x, b); rebase(pl.d_p, b); rebase(pl.d_T_wall, b);
  rebase(pl.cells.G, b); rebase(pl.cells.beta, b); rebase(pl.cells.theta, b);
  rebase(pl.cells.lam2, b); rebase(pl.cells.P, b);
  rebase(pl.d_abs, b); rebase(pl.d_emi, b); rebase(pl.d_acc, b); rebase(pl.d_balance, b);
  rebase(pl.d_bwall, b); rebase(pl.d_segs, b); rebase(pl.d_counts, b); rebase(pl.d_slabs, b);
  rebase(pl.d_keys, b); rebase(pl.d_perm, b); rebase(pl.d_hist, b);
  rebase(pl.d_counters, b); rebase(pl.d_stages, b); rebase(pl.d_cases, b);
}

void release_plan(rt_ctx c) {
  if (!c->batch) return;
  BatchPlan* pl = c->batch;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->capture_stream) (void)hipStreamDestroy(pl->capture_stream);
  if (pl->side_stream) (void)hipStreamDestroy(pl->side_stream);
  for (hipEvent_t e : pl->events) (void)hipEventDestroy(e);
  delete pl;
  c->batch = nullptr;
}

// Copies inputs, derives cell parameters and captures the launch graph.
rt_status materialize(rt_ctx c, int n_cases, const rt_case* cases, BatchPlan& pl, void* ws) {
  carve(pl, ws);
  std::vector<double> T(pl.total_cells), x(pl.total_cells), p(pl.total_cells), Tw(n_cases);
  for (int k = 0; k < n_cases; ++k) {
    const BatchCase& b = pl.cases[k];
    std::memcpy(&T[b.cell_off], cases[k].T_K, b.n_cells * 8);
    std::memcpy(&x[b.cell_off], cases[k].x_h2o, b.n_cells * 8);
    std::memcpy(&p[b.cell_off], cases[k].p_atm, b.n_cells * 8);
    Tw[k] = cases[k].T_wall_K;
  }
  if (c->device < 0) return bfail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_BHIP(c, hipSetDevice(c->device));
  RT_BHIP(c, hipMemcpy(pl.d_T, T.data(), T.size() * 8, hipMemcpyHostToDevice));
  RT_BHIP(c, hipMemcpy(pl.d_x, x.data(), x.size() * 8, hipMemcpyHostToDevice));
  RT_BHIP(c, hipMemcpy(pl.d_p, p.data(), p.size() * 8, hipMemcpyHostToDevice));
  RT_BHIP(c, hipMemcpy(pl.d_T_wall, Tw.data(), Tw.size() * 8, hipMemcpyHostToDevice));
  RT_BHIP(c, hipMemcpy(pl.d_stages, pl.stages.data(), pl.stages.size() * sizeof(BatchStage),
                       hipMemcpyHostToDevice));
  RT_BHIP(c, hipMemcpy(pl.d_cases, pl.cases.data(), pl.cases.size() * sizeof(BatchCase),
                       hipMemcpyHostToDevice));
  RT_BHIP(c, launch_cell_params_on(c, pl.total_cells, pl.d_T, pl.d_x, pl.d_p, pl.cells, c->stream));
  RT_BHIP(c, launch_batch_prep(c, pl, c->stream));
  RT_BHIP(c, hipStreamSynchronize(c->stream));
  int cus = 0;
  RT_BHIP(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  pl.grid_blocks = (int64_t)pl.tuning.blocks_per_cu * cus;
  RT_BHIP(c, hipStreamCreateWithFlags(&pl.capture_stream, hipStreamNonBlocking));
  if (pl.chunked && pl.tuning.slots > 1) {
    // line sums on a second stream (default priority), ordered against the
    // marches by events: one fork, then per chunk "line sum done" and
    // "march done"
    RT_BHIP(c, hipStreamCreateWithFlags(&pl.side_stream, hipStreamNonBlocking));
    pl.events.assign(1 + 2 * (size_t)pl.n_chunks, nullptr);
    for (auto& e : pl.events) RT_BHIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  RT_BHIP(c, hipStreamBeginCapture(pl.capture_stream, hipStreamCaptureModeRelaxed));
  hipError_t le = launch_batch(c, pl, pl.capture_stream);
  hipError_t ce = hipStreamEndCapture(pl.capture_stream, &pl.graph);
  if (le != hipSuccess) return bfail(c, RT_EDEVICE, std::string("rt_batch: launch capture: ") + hipGetErrorString(le));
  if (ce != hipSuccess) return bfail(c, RT_EDEVICE, std::string("rt_batch: end capture: ") + hipGetErrorString(ce));
  RT_BHIP(c, hipGraphInstantiate(&pl.exec, pl.graph, nullptr, nullptr, 0));
  return RT_OK;
}

rt_status prepare_impl(rt_ctx c, int n_cases, const rt_case* cases, int kappa_mode,
                       const rt_batch_tuning& t, void* ws, int64_t bytes, int64_t limit_points) {
  for (const auto& g : c->gas)
    if (g.active)
      return bfail(c, RT_EUNSUPPORTED, "batched form: one gas only (gas 0); remove gases 1.. first");
  release_plan(c);
  BatchPlan* pl = new (std::nothrow) BatchPlan();
  if (!pl) return bfail(c, RT_ENOMEM, "rt_batch: out of host memory");
  int64_t need = 0;
  rt_status s = build_plan(c, n_cases, cases, t, limit_points, *pl, &need);
  if (s == RT_OK && need > bytes) s = bfail(c, RT_EINVAL, "rt_batch: workspace too small");
  pl->comp = kappa_mode == RT_KAPPA_COMPENSATED;
  c->batch = pl;
  if (s == RT_OK) s = materialize(c, n_cases, cases, *pl, ws);
  if (s != RT_OK) release_plan(c);
  return s;
}

std::string arch_name(rt_ctx c) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t k = a.find(':');
  return k == std::string::npos ? a : a.substr(0, k);
}

std::string shape_key(rt_ctx c, int n_cases, const rt_case* cases) {
  double cells = 0, rays = 0;
  for (int k = 0; k < n_cases; ++k) {
    cells += (double)cases[k].nx * cases[k].ny * cases[k].nz;
    rays += (double)cases[k].n_rays;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "v6|%s|cases=%d|log2cells=%d|log2rays=%d|nu=%d|log2lines=%d",
                arch_name(c).c_str(), n_cases, (int)std::lround(std::log2(cells)),
                (int)std::lround(std::log2(rays)), c->n_nu,
                (int)std::lround(std::log2((double)std::max(1, c->lines.n))));
  return buf;
}

// cache file: one line per entry, wrapped as a JSON object
// {"<key>": [chunk, groups, rays, bpc, slots, mode], ...}
bool cache_lookup(const char* path, const std::string& key, rt_batch_tuning* t) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    const size_t q = line.find('"');
    const size_t q2 = line.find('"', q + 1);
    if (q == std::string::npos || q2 == std::string::npos) continue;
    if (line.substr(q + 1, q2 - q - 1) != key) continue;
    rt_batch_tuning v;
    if (std::sscanf(line.c_str() + q2 + 1, " : [%d, %d, %d, %d, %d, %d]", &v.chunk_points,
                    &v.kappa_groups, &v.march_rays, &v.blocks_per_cu, &v.slots, &v.mode) == 6) {
      *t = v;
      return true;
    }
  }
  return false;
}

void cache_store(const char* path, const std::string& key, const rt_batch_tuning& t) {
  if (!path) return;
  std::vector<std::string> entries;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      const size_t q = line.find('"');
      const size_t q2 = line.find('"', q + 1);
      if (q == std::string::npos || q2 == std::string::npos) continue;
      if (line.substr(q + 1, q2 - q - 1) == key) continue;
      std::string e = line.substr(q);
      while (!e.empty() && (e.back() == ',' || e.back() == ' ')) e.pop_back();
      entries.push_back(e);
    }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf), "\"%s\": [%d, %d, %d, %d, %d, %d]", key.c_str(),
                t.chunk_points, t.kappa_groups, t.march_rays, t.blocks_per_cu, t.slots, t.mode);
  entries.push_back(buf);
  std::ofstream o(path, std::ios::trunc);
  o << "{\n";
  for (size_t i = 0; i < entries.size(); ++i)
    o << "  " << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  o << "}\n";
}

}  // namespace

extern "C" {

rt_status rt_batch_default_tuning(rt_batch_tuning* out) {
  if (!out) return RT_EINVAL;
  *out = default_tuning();
  return RT_OK;
}

rt_status rt_batch_workspace_size(rt_ctx c, int n_cases, const rt_case* cases,
                                  const rt_batch_tuning* tuning, int64_t* bytes) {
  if (!c || !bytes) return RT_EINVAL;
  const rt_batch_tuning t = tuning ? *tuning : default_tuning();
  if (rt_status s = check_tuning(c, t)) return s;
  if (rt_status s = check_cases(c, n_cases, cases)) return s;
  BatchPlan pl;
  return build_plan(c, n_cases, cases, t, 0, pl, bytes);
}

rt_status rt_batch_prepare(rt_ctx c, int n_cases, const rt_case* cases, int kappa_mode,
                           const rt_batch_tuning* tuning, void* ws, int64_t bytes) {
  if (!c) return RT_EINVAL;
  if (kappa_mode != RT_KAPPA_PLAIN && kappa_mode != RT_KAPPA_COMPENSATED)
    return bfail(c, RT_EINVAL, "rt_batch_prepare: unknown kappa mode");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
    return bfail(c, RT_EINVAL, "rt_batch_prepare: workspace must be 256-byte aligned device memory");
  const rt_batch_tuning t = tuning ? *tuning : default_tuning();
  if (rt_status s = check_tuning(c, t)) return s;
  if (rt_status s = check_cases(c, n_cases, cases)) return s;
  return prepare_impl(c, n_cases, cases, kappa_mode, t, ws, bytes, 0);
}

rt_status rt_batch_launch(rt_ctx c) {
  if (!c) return RT_EINVAL;
  if (!c->batch || !c->batch->exec) return bfail(c, RT_ESTATE, "rt_batch_launch: call rt_batch_prepare first");
  if (c->device < 0) return bfail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_BHIP(c, hipSetDevice(c->device));
  hipEvent_t a, b;
  RT_BHIP(c, hipEventCreate(&a));
  RT_BHIP(c, hipEventCreate(&b));
  c->batch_events.emplace_back(a, b);
  RT_BHIP(c, hipEventRecord(a, c->stream));
  RT_BHIP(c, hipGraphLaunch(c->batch->exec, c->stream));
  RT_BHIP(c, hipEventRecord(b, c->stream));
  return RT_OK;
}

rt_status rt_batch_results(rt_ctx c, double* absorbed, double* emitted, double* balance) {
  if (!c) return RT_EINVAL;
  if (!c->batch) return bfail(c, RT_ESTATE, "rt_batch_results: call rt_batch_prepare first");
  BatchPlan& pl = *c->batch;
  if (c->device < 0) return bfail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_BHIP(c, hipSetDevice(c->device));
  RT_BHIP(c, hipStreamSynchronize(c->stream));
  unsigned err = 0, ovf = 0;
  RT_BHIP(c, hipMemcpy(&err, pl.d_counters + 2, sizeof(unsigned), hipMemcpyDeviceToHost));
  RT_BHIP(c, hipMemcpy(&ovf, pl.d_acc + (pl.total_cells + (int64_t)pl.n_cases * kCaseBalRows) * kAccRow, sizeof(unsigned),
                       hipMemcpyDeviceToHost));
  if (ovf)
    return bfail(c, RT_EDEVICE, "rt_batch_results: a tallied power was negative, not finite or not below 2^80 W");
  if (absorbed)
    RT_BHIP(c, hipMemcpy(absorbed, pl.d_abs, pl.total_cells * 8, hipMemcpyDeviceToHost));
  if (emitted)
    RT_BHIP(c, hipMemcpy(emitted, pl.d_emi, pl.total_cells * 8, hipMemcpyDeviceToHost));
  if (balance)
    RT_BHIP(c, hipMemcpy(balance, pl.d_balance, (size_t)pl.n_cases * 4 * 8, hipMemcpyDeviceToHost));
  // work counters of the batch
  std::vector<int32_t> counts(pl.total_rays);
  RT_BHIP(c, hipMemcpy(counts.data(), pl.d_counts, counts.size() * 4, hipMemcpyDeviceToHost));
  double segs = 0;
  for (int32_t v : counts) segs += v;
  const double pts = (double)std::min<int64_t>((int64_t)pl.n_chunks * pl.tuning.chunk_points, c->n_nu);
  c->stats.batch_updates = segs * pts;
  c->stats.batch_line_evals = pl.line_evals;
  double ms = 0;
  for (auto& e : c->batch_events) {
    float f = 0;
    RT_BHIP(c, hipEventElapsedTime(&f, e.first, e.second));
    ms = f;  // last launch
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  c->batch_events.clear();
  c->stats.batch_ms = ms;
  if (err) return bfail(c, RT_EDEVICE, "rt_batch_results: a dependency wait in the persistent kernel timed out");
  return RT_OK;
}

rt_status rt_batch_run(rt_ctx c, int n_cases, const rt_case* cases, int kappa_mode,
                       const rt_batch_tuning* tuning, double* absorbed, double* emitted,
                       double* balance) {
  if (!c) return RT_EINVAL;
  int64_t bytes = 0;
  if (rt_status s = rt_batch_workspace_size(c, n_cases, cases, tuning, &bytes)) return s;
  if (c->device < 0) return bfail(c, RT_EUNSUPPORTED, "host-only handle (RT_NO_DEVICE): the call needs a device");
  RT_BHIP(c, hipSetDevice(c->device));
  void* ws = nullptr;
  hipError_t e = hipMalloc(&ws, (size_t)bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // not left for the next launch check
    return bfail(c, RT_ENOMEM, std::string("rt_batch_run: workspace of ") + std::to_string(bytes) +
                                   " bytes: " + hipGetErrorString(e));
  }
  rt_status s = rt_batch_prepare(c, n_cases, cases, kappa_mode, tuning, ws, bytes);
  if (s == RT_OK) s = rt_batch_launch(c);
  if (s == RT_OK) s = rt_batch_results(c, absorbed, emitted, balance);
  (void)hipStreamSynchronize(c->stream);  // nothing may still read the workspace
  release_plan(c);
  (void)hipFree(ws);
  return s;
}

rt_status rt_batch_autotune(rt_ctx c, int n_cases, const rt_case* cases, int kappa_mode, void* ws,
                            int64_t bytes, const char* cache_path, rt_batch_tuning* best) {
  if (!c || !best) return RT_EINVAL;
  if (rt_status s = check_cases(c, n_cases, cases)) return s;
  const std::string key = shape_key(c, n_cases, cases);
  if (cache_lookup(cache_path, key, best)) return RT_OK;
  const int64_t trial_points =
      std::min<int64_t>(4 * kChunk, ((int64_t)c->n_nu + kChunk - 1) / kChunk * kChunk);
  rt_batch_tuning cur = default_tuning();
  double cur_ms = -1;
  auto trial = [&](const rt_batch_tuning& t, double* ms) -> rt_status {
    BatchPlan probe;
    int64_t need = 0;
    if (build_plan(c, n_cases, cases, t, trial_points, probe, &need) != RT_OK || need > bytes) {
      *ms = -1;
      return RT_OK;  // does not fit: skip
    }
    if (rt_status s = prepare_impl(c, n_cases, cases, kappa_mode, t, ws, bytes, trial_points)) return s;
    for (int rep = 0; rep < 2; ++rep) {
      if (rt_status s = rt_batch_launch(c)) return s;
      if (rt_status s = rt_batch_results(c, nullptr, nullptr, nullptr)) return s;
    }
    *ms = c->stats.batch_ms;
    return RT_OK;
  };
  if (rt_status s = trial(cur, &cur_ms)) return s;
  if (cur_ms < 0) return bfail(c, RT_EINVAL, "rt_batch_autotune: workspace too small for the default tuning");
  // coordinate descent, repeated while a pass improves (at most 3 passes):
  // the best value of one parameter moves when the others change
  // (the persistent kernel's own parameters are swept only in its mode)
  const int modes[] = {RT_BATCH_CHUNKED, RT_BATCH_PERSISTENT};
  const int chunks[] = {kChunk, 2 * kChunk, 4 * kChunk};
  const int groups[] = {16, 32, 64, 128};
  const int rays[] = {16, 64, 256};
  const int bpc[] = {2, 4, 5, 8};
  const int slots[] = {1, 2, 4, 8};
  const int* values[6] = {modes, chunks, groups, rays, bpc, slots};
  const int n_values[6] = {2, 3, 4, 3, 4, 4};
  for (int pass = 0; pass < 3; ++pass) {
    bool improved = false;
    for (int param = 0; param < 6; ++param) {
      if (param >= 2 && param <= 4 && cur.mode == RT_BATCH_CHUNKED) continue;
      for (int v = 0; v < n_values[param]; ++v) {
        rt_batch_tuning t = cur;
        const int x = values[param][v];
        if (param == 0) t.mode = x;
        if (param == 1) t.chunk_points = x;
        if (param == 2) t.kappa_groups = x;
        if (param == 3) t.march_rays = x;
        if (param == 4) t.blocks_per_cu = x;
        if (param == 5) t.slots = x;
        if (std::memcmp(&t, &cur, sizeof(t)) == 0) continue;
        if (check_tuning(c, t) != RT_OK) continue;  // e.g. one slab for the queue
        double ms = -1;
        if (rt_status s = trial(t, &ms)) return s;
        if (ms > 0 && ms < cur_ms) { cur = t; cur_ms = ms; improved = true; }
      }
    }
    if (!improved) break;
  }
  release_plan(c);
  *best = cur;
  cache_store(cache_path, key, cur);
  return RT_OK;
}

}  // extern "C"

namespace rt {
void destroy_batch(rt_ctx c) { release_plan(c); }
}  // namespace rt
