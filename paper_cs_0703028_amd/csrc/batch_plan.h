// batch_plan.h -- work plan of the batched launch (host + device): either
// per-chunk launches over all cases or one persistent work-queue kernel.
#pragma once

#include "rt_internal.h"

namespace rt {

constexpr int kStageRaygen = 0, kStageKappa = 1, kStageMarch = 2;
// balance rows (entering, escaped) per case; a case's rays spread over them
constexpr int kCaseBalRows = 64;

// One contiguous range of queue items of one kind.
struct BatchStage {
  int kind;
  int cas;
  int chunk;
  int pair;          // (case, chunk) pair index in queue order
  int slot;          // kappa slab of the pair
  int wait_pair;     // KAPPA: pair whose march frees the slab (-1: none)
  int wait_stage;    // KAPPA: that pair's MARCH stage; MARCH: this pair's KAPPA stage
  int raygen_stage;  // MARCH: the case's RAYGEN stage
  int64_t first;     // first queue item
  int64_t count;     // items in the stage
};

struct BatchCase {
  int nx, ny, nz, max_segs;
  int64_t n_cells, cell_off, n_rays, seg_off, ray_off;
  int64_t blk_off;  // chunked mode: first row of 8 march blocks of the case
  uint64_t seed;
  double weight, unit_cm;
  float2 theta_wall;  // c2 / T_wall as an FP32 pair (0: cold walls)
};

struct BatchPlan {
  rt_batch_tuning tuning;
  bool comp = false;
  bool chunked = true;      // tuning.mode == RT_BATCH_CHUNKED
  bool planck_quad = true;  // second-order Planck expansion in the march
  int n_cases = 0, n_chunks = 0, n_pairs = 0, n_stages = 0;
  int64_t total_items = 0, total_cells = 0, total_rays = 0, max_cells = 0;
  int64_t ray_blocks = 0;  // chunked mode: rows of 8 march blocks over all cases
  int64_t grid_blocks = 0;
  int64_t bwall_ld = 0, slab_stride = 0;
  int64_t n_counters = 0;
  double line_evals = 0, updates_per_seg = 0;
  std::vector<BatchCase> cases;
  std::vector<BatchStage> stages;
  // device pointers into the caller's workspace
  double *d_T = nullptr, *d_x = nullptr, *d_p = nullptr, *d_T_wall = nullptr;
  CellSet cells;
  // fixed-point accumulator rows: case k's cells from cell_off + k kCaseBalRows,
  // then its kCaseBalRows balance rows (entering, escaped); the overflow flag
  // after the last row
  unsigned long long* d_acc = nullptr;
  double *d_abs = nullptr, *d_emi = nullptr, *d_balance = nullptr;
  float* d_bwall = nullptr;
  int2* d_segs = nullptr;
  int32_t* d_counts = nullptr;
  uint32_t* d_keys = nullptr;  // coherent-order key per ray (all cases)
  uint32_t* d_perm = nullptr;  // case-local slot -> case-local ray index
  uint32_t* d_hist = nullptr;  // [n_cases][kOrderBuckets] counts, then offsets
  float* d_slabs = nullptr;
  unsigned* d_counters = nullptr;  // [queue lo, queue hi, error, pad, rg_done..., k_done..., m_done...]
  BatchStage* d_stages = nullptr;
  BatchCase* d_cases = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture_stream = nullptr;
  // chunked mode with several slabs: the line sums' stream and the events
  // ordering it against the marches (fork, line sum done per chunk, march
  // done per chunk)
  hipStream_t side_stream = nullptr;
  std::vector<hipEvent_t> events;
};

hipError_t launch_batch_prep(rt_ctx c, const BatchPlan& pl, hipStream_t s);
hipError_t launch_batch(rt_ctx c, const BatchPlan& pl, hipStream_t s);
hipError_t launch_cell_params_on(rt_ctx c, int64_t n, const double* T, const double* x,
                                 const double* p, const CellSet& cells, hipStream_t s);

}  // namespace rt
