// surrogate.h -- state of the learned form: an MLP (T, x, p, chunk) -> 256
// values of ln(kappa/u) per spectral chunk, BF16 weights on MFMA with FP32
// accumulation, trained on line-sum spectra.
#pragma once

#include "rt_internal.h"

namespace rt {

typedef __bf16 bf16;

constexpr int kMlpLayers = 4;
constexpr int kMlpWidth = 256;                         // outputs per chunk
constexpr int kMaxCheckCells = 256;                    // sampled cells per check, at most
constexpr int kMlpDims[kMlpLayers + 1] = {4, 512, 512, 512, 256};

struct Surrogate {
  bool trained = false;
  int n_nu = 0, n_chunks = 0;
  double T_min = 0, T_max = 0, x_min = 0, x_max = 0, p_min = 0, p_max = 0;
  int check_cells = 8;
  double tolerance = 1e-3;
  uint64_t check_seed = 0;
  // parameters: FP32 masters W_l [K][N] and b_l [N]; Adam moments; BF16
  // copies for the forward GEMM ([N][K]) and for the input gradient ([K][N])
  float* w[kMlpLayers] = {};
  float* b[kMlpLayers] = {};
  float* mw[kMlpLayers] = {};
  float* vw[kMlpLayers] = {};
  float* mb[kMlpLayers] = {};
  float* vb[kMlpLayers] = {};
  bf16* wt[kMlpLayers] = {};
  bf16* wk[kMlpLayers] = {};
  // inference copies of layers 2-4 in MFMA fragment order: for column tile
  // ct, k-step s (16) and lane l, the 8 values of W^T[32 ct + l % 32]
  // [16 s + 8 (l / 32) ..] are contiguous, so a wavefront's operand load is
  // one contiguous 1 KB read
  bf16* wf[kMlpLayers] = {};
  float* mean = nullptr;  // [n_chunks][256] normalisation of the targets
  float* stdv = nullptr;
  // last inference
  double check_error = 0;       // largest checked relative L1 error of a chunk
  int fallback_chunks = 0;      // chunks recomputed with the line sum
  int exact_chunks = 0;  // last inference: chunks summed exactly beside the network
  int fallback_cells = 0;       // out-of-range cells recomputed
  double infer_ms = 0, check_ms = 0, fallback_ms = 0;
  double train_loss = 0;
  int64_t param_count = 0;
  // inference scratch, kept between calls (sized for the current grid)
  int64_t inf_cells = 0, inf_ld = 0;
  int inf_check = 0, inf_chunks = 0;
  unsigned* d_cell_flag = nullptr;   // = epoch: cell outside the training box
  unsigned* d_group_flag = nullptr;  // = epoch: its line-sum group of cells
  unsigned epoch = 0;                // inference calls so far
  float* d_err = nullptr;            // checked error per chunk
  int32_t* d_check = nullptr;   // sampled cells
  float* d_exact = nullptr;     // their exact rows
  uint64_t pick_epoch = ~0ull;  // grid the sampled cells were drawn for
  hipEvent_t ev[4] = {};
  // with long line lists the check's exact line sum runs on a second
  // stream of the handle's device (default priority), beside the network:
  // forked after the previous work of the handle's stream and joined before
  // the check
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool stats_pending = false;   // counts of the last inference not read yet
  bool time_phases = false;     // attach timing events to the inference kernels
  bool timed_last = false;      // the last inference carried them
};


}  // namespace rt
