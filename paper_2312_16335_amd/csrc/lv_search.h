// Device-side views shared by the search kernels and their host launchers.
#pragma once

#include <cstdint>

#include "lv_common.h"

namespace lv {

constexpr int kDefaultHashSlots = 1024;

// What the traversal reads of one index (device pointers).
struct IndexView {
  const unsigned char *records;
  int64_t stride;
  int32_t d;
  int32_t code_bytes;
  const float *mu;
  const unsigned char *sec;
  int32_t D;
  int32_t sec_row_bytes;
  int32_t sec_packets;
  int32_t sec_kind;  // LV_F32, LV_F16, LV_LVQ8, LV_F16_RESID or LV_LVQ8_LEVEL2
  const float *sec_mu;  // [D] for LV_LVQ8
  const uint32_t *adj;
  int32_t R;
  uint32_t entry;
  uint32_t N;
  const uint16_t *A;  // bfloat16 [d][D] query projection (may be null)
};

// One request of a batched step: queries [q_begin, q_end) of the step, all
// searched in sub-index `sub` with (k, L); results at element out_off of
// the step's ids / scores arrays (count * k of them).
struct Request {
  int32_t sub;
  int32_t k;
  int32_t L;
  int32_t tile0;   // first 32-row projection tile of this request
  int64_t q_begin;
  int64_t q_end;
  int64_t out_off;
};

// Per-step header, followed in memory by nreq Request entries.
struct StepHeader {
  const float *Q;        // [nq][D]
  float *Qp;             // [nq][qp_stride] projected queries (workspace)
  uint32_t *ids;
  float *scores;
  uint32_t *counters;    // [nq][2] or null
  int64_t nq;
  int64_t qp_stride;
  int32_t nreq;
  int32_t ntiles;        // 32-row projection tiles over all requests
};

// One batch of construction searches (graph construction, Appendix A):
// node order[start + b] for b < B, window L, pool rows of pool_stride
// (>= L + R) ids at pool + b * pool_stride; optional counters [B][2]
// (expansions, scorings).  ix.adj is the graph being built.
struct BuildSearchArgs {
  IndexView ix;
  const uint32_t *order;
  int64_t start;
  int32_t B;
  int32_t L;
  int32_t pool_stride;
  uint32_t *pool;
  uint32_t *counters;
  unsigned long long *stats;  // optional totals: [0] searches, [1] expansions, [2] scorings
  int32_t hash_slots;
  int32_t probes;
};

IndexView make_view(const lv_index *ix);
// Visited set of one query: `slots` slots in LDS (a multiple of 256), up to `probes` slots tried
// before an id replaces the one in its home slot.
// expand: entries expanded per iteration (1: the paper's traversal; more:
// the throughput variant).
struct VisitedCfg {
  int slots;
  int probes;
  int expand;
  bool team = false;  // plain search: kTeamWaves wavefronts per query
};
int visited_config(const lv_search_params *params, VisitedCfg *cfg);
size_t beam_lds_bytes(int L, int slots);
int check_lds(size_t lds, int L, int slots);
int launch_batched(int bits, int group, int vbytes, const StepHeader *hdr,
                      const IndexView *subs, unsigned int *counter, int Lmax, VisitedCfg vc,
                      int grid, hipStream_t stream);
int batched_occupancy(int bits, int group, int vbytes, int Lmax, VisitedCfg vc, int *blocks);
int launch_build_search(int bits, int group, int vbytes, const BuildSearchArgs &a,
                        hipStream_t stream);
int launch_project_grouped(const StepHeader *hdr, const IndexView *subs, int max_tiles, int d,
                           int D, hipStream_t stream);

}  // namespace lv
