// Plan object and host-side helpers shared by the library's C-ABI sources.
#pragma once

#include <string>
#include <vector>

#include "internal.h"

namespace omniseg {

// Records the error text of the calling thread and returns `code`.
int32_t fail(int32_t code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::omniseg::fail(OMNISEG_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct ConvDesc {
  int64_t canon_w, canon_b;
  int cin, cout, cu;
  int cin_p, cout_p, cu_p;
  int64_t pk_w, pk_b;
  int64_t pk_wt;  // data-gradient (transposed, flipped) weights, or -1
  // FP8: packed per-output-channel weight scales (or -1), and the activation
  // table offsets of the input's channel scales (upsampled / plain part, skip
  // part or -1) and of the output's
  int64_t pk_ws = -1;
  int64_t act_in = -1, act_in_e = -1, act_out = -1;
};

inline int elem_size(int precision) {
  return precision == OMNISEG_BF16 ? 2 : precision == OMNISEG_FP8 ? 1 : 4;
}

}  // namespace omniseg

struct omniseg_plan {
  omniseg_config cfg;
  int L = 0;
  int C[8] = {0};
  int Cp[8] = {0};
  int P = 0;
  int G = 0;
  int64_t n_canon = 0;
  omniseg::ConvDesc enc_a[8], enc_b[8], dec_a[8], dec_b[8];
  int64_t canon_first_w = 0, canon_first_b = 0, pk_first_w = 0, pk_first_b = 0;
  int64_t canon_pre_w = -1, canon_pre_b = -1, pk_pre_w = 0, pk_pre_b = 0;
  int64_t canon_ctrl_w = 0, canon_ctrl_b = 0, pk_ctrl_w = 0, pk_ctrl_b = 0;
  int64_t packed_bytes = 0;
  // activation table (per padded channel of every stored activation):
  // offset of (kind, level), kinds OMNISEG_ACT_*; -1 where absent
  int64_t act_off[4][8];
  int64_t n_act = 0;
  // FP8: packed channel scales and their inverses, one per table entry
  int64_t pk_scale = -1, pk_iscale = -1;
  mutable std::vector<omniseg::SlideDev> slide_tab;  // host staging of the device slide table
  mutable std::vector<int32_t> host_tab;             // host staging of tile lists and grids
  // conv tile configuration per (stage, level): stage 0 enc_a, 1 enc_b, 2 dec_a, 3 dec_b; -1 = default
  int tune[4][8];
  // per-launch profiling (off by default); records accumulate over calls
  // until omniseg_read_profile has returned them
  bool profiling = false;
  mutable bool profile_read = false;
  mutable std::vector<hipEvent_t> events;
  mutable std::vector<omniseg_launch_record> recs;
  // captured graphs of omniseg_segment_slide, keyed by a hash of the arguments
  struct GraphEntry {
    uint64_t key;
    hipGraphExec_t exec;
  };
  mutable std::vector<GraphEntry> graphs;
  ~omniseg_plan() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (const GraphEntry& g : graphs) (void)hipGraphExecDestroy(g.exec);
  }
};

namespace omniseg {

// Conv tile configuration for a backbone layer: the tuned one when it is
// valid for the shape, else the default.  stage: 0 enc_a, 1 enc_b, 2 dec_a, 3 dec_b.
inline int layer_config(const omniseg_plan* p, int stage, int level, int H, int W, int cout_p) {
  const int t = p->tune[stage][level];
  if (t >= 0 && conv_config_valid(t, p->cfg.precision, H, W, cout_p)) return t;
  return conv_default_config(p->cfg.precision, H, W, cout_p);
}

// Records a pair of events around each launch when profiling is on.
struct Prof {
  const omniseg_plan* p;
  hipStream_t st;
  size_t next = 0;
  hipError_t begin() {
    if (!p->profiling) return hipSuccess;
    while (p->events.size() < 2 * (next + 1)) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      p->events.push_back(e);
    }
    return hipEventRecord(p->events[2 * next], st);
  }
  hipError_t end(int stage, int level, int tiles, double flops, double bytes, int config = -1) {
    if (!p->profiling) return hipSuccess;
    hipError_t r = hipEventRecord(p->events[2 * next + 1], st);
    omniseg_launch_record rec;
    rec.stage = stage;
    rec.level = level;
    rec.tiles = tiles;
    rec.precision = p->cfg.precision;
    rec.config = config;
    rec.reserved = 0;
    rec.flops = flops;
    rec.bytes = bytes;
    rec.ms = 0.0;
    p->recs.push_back(rec);
    ++next;
    return r;
  }
};

// The profiler of one call: continues the record list of earlier profiled
// calls, or starts a new one once the list has been read.
inline Prof profile_start(const omniseg_plan* p, hipStream_t st) {
  if (p->profiling && p->profile_read) {
    p->recs.clear();
    p->profile_read = false;
  }
  Prof prof{p, st};
  prof.next = p->recs.size();
  return prof;
}

}  // namespace omniseg
