// Graph construction on the primary vectors.
//
// Appendix A: per node, search the current graph with the node as the query
// for more than R candidates, prune them to at most R diverse out-neighbours
// and make those the node's out-edges.  Section 2 ("Graph construction"):
// only the primary vectors take part.  Appendix D: Vamana, pruning factor
// alpha.  Distances are the squared Euclidean distances of the LVQ
// reconstructions (lv_l2.h).
//
// Batch-synchronous insertion, so that a parallel build has one result:
// nodes are inserted in a given order, in batches of 1, 2, 4, ... up to
// max_batch in the first pass and of max_batch in later passes.  A batch:
//   1. construction searches on the graph as it stands (one wavefront per
//      node, the search kernel's body): pool row = final window, then the
//      node's current out-neighbours;
//   2. forward pruning (one wavefront per node) writes the node's new row;
//      each new edge p -> j counts one new source of j, and the first count
//      lists j as a touched target;
//   3. every touched target reserves a slice of the source list;
//   4. every new edge writes its source into its target's slice;
//   5. reverse edges (one wavefront per touched target): the new sources in
//      ascending order that are not in the target's row are appended, in
//      registers only (reverse_append_kernel, the common case); a target
//      whose union is longer than R (or that has more than 64 new sources)
//      is listed for reverse_kernel, which prunes the union around it.
// Every row is written by one wavefront, and no row depends on the order in
// which targets were listed, so the graph does not depend on scheduling.
//
// Pruning by one wavefront: the candidates (sentinel and the node itself
// removed) are scored one per pass of the whole wavefront (one coalesced
// load of the record's code words, integer dot products with v_dot4 /
// v_dot8, exact sums), ranked by (distance, id) by counting, and walked in
// that order with repeats skipped.  Lane j holds kept neighbour j (its codes
// in LDS) and tests whether it dominates the candidate:
// alpha^2 f(k, c) <= f(p, c).  The next candidate's code words are loaded
// while the current one is tested.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lv_common.h"
#include "lv_l2.h"
#include "lv_search.h"

namespace lv {
namespace {

constexpr int kMaxR = 64;             // one kept neighbour per lane
constexpr int kMaxCodeWords = 64;     // one code word per lane (d * bits <= 2048)
constexpr int kMaxNewSources = 256;   // new in-edges of one node in one batch

#define LV_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const LV_GLOBAL T *gp(const T *p) {
  return (const LV_GLOBAL T *)p;
}

__device__ __forceinline__ bool better(double as, uint32_t aid, double bs, uint32_t bid) {
  return (as > bs) | ((as == bs) & (aid < bid));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// v moved across lanes by a DPP pattern (rows outside ROWS receive 0).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  if constexpr (ROWS == 0xF)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
  else
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}

// Sum over the wavefront (all lanes active), returned in every lane: sums
// within quads (swap neighbours, swap pairs), within rows (rotate by 4 and
// 8), then rows chained into lane 63 (row broadcasts 15 and 31).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v += dpp_u32<0xB1>(v);
  v += dpp_u32<0x4E>(v);
  v += dpp_u32<0x124>(v);
  v += dpp_u32<0x128>(v);
  v += dpp_u32<0x142, 0xA>(v);
  v += dpp_u32<0x143, 0xC>(v);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Sum of code products over one 32-bit word of two records.
template <int BITS>
__device__ __forceinline__ uint32_t dot_codes(uint32_t a, uint32_t b, uint32_t acc) {
  if constexpr (BITS == 8)
    return __builtin_amdgcn_udot4(a, b, acc, false);
  else
    return __builtin_amdgcn_udot8(a, b, acc, false);
}

template <int BITS>
constexpr uint32_t kOnes = BITS == 8 ? 0x01010101u : 0x11111111u;

struct PruneView {
  const unsigned char *records;
  int64_t stride;
  int32_t d;
  int32_t cw;  // 32-bit code words per record
  uint32_t *adj;
  int32_t R;
  uint32_t N;
  double alpha2;
};

// Bookkeeping of one batch (device memory).
struct BatchState {
  uint32_t *cnt;       // [N] new sources per node in this batch (zero between batches)
  uint32_t *fill;      // [N]
  uint32_t *base;      // [N]
  uint32_t *touched;   // [max_batch * R]
  uint32_t *srcs;      // [max_batch * R]
  uint32_t *deferred;  // [max_batch * R] targets left to reverse_kernel
  uint32_t *misc;      // [0] touched count, [1] source cursor, [2] overflow flag,
                       // [3] deferred count
  unsigned long long *stats;  // optional work totals (LV_BS_* order) or null
};

extern __shared__ __align__(16) unsigned char lv_gsmem[];

// Per-wavefront LDS of the pruning kernels for M candidates and rows of kw
// code words: an odd number of 16-byte chunks (zero padded), so that 16
// lanes reading 16 bytes each from 16 different kept rows cover all banks.
struct PruneLds {
  double *cs;       // [M] -f(p, c)
  uint32_t *cid;    // [M]
  float *cdl;       // [M] delta
  float *clo;       // [M] lo
  uint32_t *csum;   // [M] sum of codes
  uint32_t *csq;    // [M] sum of squared codes
  uint32_t *ord;    // [M] candidate index by rank
  uint32_t *krow;   // [R][kw] codes of kept neighbours
  float *kdl, *klo; // [R]
  uint32_t *ks, *kss, *kid;  // [R]
  uint32_t *stage;  // [kw] codes of the candidate under test
};

__host__ __device__ inline int row_words(int cw) { return 4 * (((cw + 3) / 4) | 1); }

__host__ __device__ inline size_t prune_lds_bytes(int M, int R, int cw) {
  const int kw = row_words(cw);
  return (size_t)M * (8 + 4 * 6) + (size_t)R * kw * 4 + (size_t)R * 4 * 5 + (size_t)kw * 4;
}

__device__ __forceinline__ PruneLds carve_prune(int M, int R, int cw) {
  PruneLds s;
  unsigned char *b = lv_gsmem;
  const int kw = row_words(cw);
  // 16-byte aligned rows first: kept codes, then the staged candidate
  s.krow = reinterpret_cast<uint32_t *>(b);
  s.stage = s.krow + (size_t)R * kw;
  s.cs = reinterpret_cast<double *>(s.stage + kw);
  s.cid = reinterpret_cast<uint32_t *>(s.cs + M);
  s.cdl = reinterpret_cast<float *>(s.cid + M);
  s.clo = s.cdl + M;
  s.csum = reinterpret_cast<uint32_t *>(s.clo + M);
  s.csq = s.csum + M;
  s.ord = s.csq + M;
  s.kdl = reinterpret_cast<float *>(s.ord + M);
  s.klo = s.kdl + R;
  s.ks = reinterpret_cast<uint32_t *>(s.klo + R);
  s.kss = s.ks + R;
  s.kid = s.kss + R;
  return s;
}

// Prune candidates cid[0..m) (no sentinel, not p) around node p; returns
// the number kept, their ids in kid[].
template <int BITS>
__device__ int prune_core(const PruneView &v, uint32_t p, int m, const PruneLds &sm, int lane) {
  const int cw = v.cw;
  const int kw = row_words(cw);
  const double dd = (double)v.d;
  const LV_GLOBAL unsigned char *recs = gp(v.records);
  // the pruned node: its code word of this lane, constants and code sums
  const LV_GLOBAL unsigned char *prec = recs + (size_t)p * (size_t)v.stride;
  const uint32_t pw = lane < cw ? reinterpret_cast<const LV_GLOBAL uint32_t *>(prec)[lane] : 0u;
  const LV_GLOBAL float *pc = reinterpret_cast<const LV_GLOBAL float *>(prec + 4 * cw);
  const double pdl = (double)pc[0], plo = (double)pc[1];
  const double ps = (double)wave_sum(dot_codes<BITS>(pw, kOnes<BITS>, 0u));
  const double pss = (double)wave_sum(dot_codes<BITS>(pw, pw, 0u));

  // score: one candidate per pass of the wavefront, U loads in flight
  constexpr int U = 4;
  for (int i0 = 0; i0 < m; i0 += U) {
    uint32_t x[U];
    float dl[U], lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      x[u] = 0u;
      dl[u] = lo[u] = 0.f;
      if (i < m) {
        const LV_GLOBAL unsigned char *rec = recs + (size_t)sm.cid[i] * (size_t)v.stride;
        if (lane < cw) x[u] = reinterpret_cast<const LV_GLOBAL uint32_t *>(rec)[lane];
        const LV_GLOBAL float *cc = reinterpret_cast<const LV_GLOBAL float *>(rec + 4 * cw);
        dl[u] = cc[0];
        lo[u] = cc[1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u;
      if (i >= m) break;  // uniform
      const uint32_t sab = wave_sum(dot_codes<BITS>(x[u], pw, 0u));
      const uint32_t s1 = wave_sum(dot_codes<BITS>(x[u], kOnes<BITS>, 0u));
      const uint32_t s2 = wave_sum(dot_codes<BITS>(x[u], x[u], 0u));
      if (lane == 0) {
        sm.cs[i] = -lvq_l2(dd, pdl, plo, ps, pss, (double)dl[u], (double)lo[u], (double)s1,
                           (double)s2, (double)sab);
        sm.cdl[i] = dl[u];
        sm.clo[i] = lo[u];
        sm.csum[i] = s1;
        sm.csq[i] = s2;
      }
    }
  }
  wave_sync();
  // rank by (distance ascending, id ascending); equal pairs (repeats of one
  // id) are ordered by position.  ord[] starts as the identity so that it
  // holds valid indices whatever the scores.
  for (int i = lane; i < m; i += 64) sm.ord[i] = (uint32_t)i;
  wave_sync();
  for (int i = lane; i < m; i += 64) {
    const double si = sm.cs[i];
    const uint32_t ii = sm.cid[i];
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double sj = sm.cs[j];
      const uint32_t ij = sm.cid[j];
      r += better(sj, ij, si, ii) | ((sj == si) & (ij == ii) & (j < i));
    }
    sm.ord[r] = (uint32_t)i;
  }
  wave_sync();
  // greedy walk.  Row words past the codes stay zero (written once here;
  // the walk writes code words only).
  const int pad = kw - cw;
  for (int t = lane; t < (v.R + 1) * pad; t += 64)
    sm.krow[(size_t)(t / pad) * kw + cw + t % pad] = 0u;  // row R is the stage
  int nk = 0;
  uint32_t prev = kSentinel;
  int nxt_i = 0;
  uint32_t nxt_x = 0u;
  if (m > 0) {
    nxt_i = (int)sm.ord[0];
    if (lane < cw)
      nxt_x = reinterpret_cast<const LV_GLOBAL uint32_t *>(
          recs + (size_t)sm.cid[nxt_i] * (size_t)v.stride)[lane];
  }
  for (int r = 0; r < m && nk < v.R; ++r) {
    const int i = nxt_i;
    const uint32_t x = nxt_x;
    if (r + 1 < m) {
      nxt_i = (int)sm.ord[r + 1];
      if (lane < cw)
        nxt_x = reinterpret_cast<const LV_GLOBAL uint32_t *>(
            recs + (size_t)sm.cid[nxt_i] * (size_t)v.stride)[lane];
    }
    const uint32_t c = sm.cid[i];
    if (c == prev) continue;
    prev = c;
    if (lane < cw) sm.stage[lane] = x;
    wave_sync();
    bool dom = false;
    if (lane < nk) {
      uint32_t sab = 0u;
      const u32x4 *kr = reinterpret_cast<const u32x4 *>(sm.krow + (size_t)lane * kw);
      const u32x4 *sg = reinterpret_cast<const u32x4 *>(sm.stage);
#pragma unroll 4
      for (int w = 0; w < kw / 4; ++w) {
        const u32x4 a = kr[w], b = sg[w];
        sab = dot_codes<BITS>(a[0], b[0], sab);
        sab = dot_codes<BITS>(a[1], b[1], sab);
        sab = dot_codes<BITS>(a[2], b[2], sab);
        sab = dot_codes<BITS>(a[3], b[3], sab);
      }
      const double f = lvq_l2(dd, (double)sm.kdl[lane], (double)sm.klo[lane],
                              (double)sm.ks[lane], (double)sm.kss[lane], (double)sm.cdl[i],
                              (double)sm.clo[i], (double)sm.csum[i], (double)sm.csq[i],
                              (double)sab);
      dom = v.alpha2 * f <= -sm.cs[i];
    }
    if (__ballot(dom)) continue;
    if (lane < cw) sm.krow[(size_t)nk * kw + lane] = x;
    if (lane == 0) {
      sm.kdl[nk] = sm.cdl[i];
      sm.klo[nk] = sm.clo[i];
      sm.ks[nk] = sm.csum[i];
      sm.kss[nk] = sm.csq[i];
      sm.kid[nk] = c;
    }
    ++nk;
    wave_sync();
  }
  wave_sync();
  return nk;
}

struct ForwardArgs {
  PruneView v;
  const uint32_t *order;
  int64_t start;
  int32_t B;
  const uint32_t *pool;
  int32_t pool_stride;  // L + R
  BatchState st;
};

template <int BITS>
__global__ __launch_bounds__(64) void prune_forward_kernel(ForwardArgs a) {
  const int b = blockIdx.x;
  if (b >= a.B) return;
  const int lane = threadIdx.x;
  const PruneView &v = a.v;
  const uint32_t p = a.order[a.start + b];
  const PruneLds sm = carve_prune(a.pool_stride, v.R, v.cw);
  const uint32_t *row = a.pool + (size_t)b * (size_t)a.pool_stride;
  int m = 0;
  for (int i0 = 0; i0 < a.pool_stride; i0 += 64) {
    const uint32_t c = i0 + lane < a.pool_stride ? row[i0 + lane] : kSentinel;
    const bool ok = c != kSentinel && c != p;
    const uint64_t msk = __ballot(ok);
    if (ok) sm.cid[m + lane_rank(msk)] = c;
    m += __popcll(msk);
  }
  wave_sync();
  const int nk = prune_core<BITS>(v, p, m, sm, lane);
  uint32_t *out = v.adj + (size_t)p * (size_t)v.R;
  for (int j = lane; j < v.R; j += 64) out[j] = j < nk ? sm.kid[j] : kSentinel;
  if (a.st.stats && lane == 0) atomicAdd(&a.st.stats[LV_BS_FWD_CANDS], (unsigned long long)m);
  if (lane < nk) {
    const uint32_t j = sm.kid[lane];
    if (atomicAdd(&a.st.cnt[j], 1u) == 0u) a.st.touched[atomicAdd(&a.st.misc[0], 1u)] = j;
  }
}

__global__ void batch_reset_kernel(uint32_t *misc) {
  misc[0] = 0u;
  misc[1] = 0u;
  misc[3] = 0u;
}

__global__ void alloc_kernel(BatchState st) {
  const uint32_t nt = st.misc[0];
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
    const uint32_t j = st.touched[t];
    st.base[j] = atomicAdd(&st.misc[1], st.cnt[j]);
    st.fill[j] = 0u;
  }
}

__global__ void scatter_kernel(const uint32_t *order, int64_t start, int32_t B, const uint32_t *adj,
                               int32_t R, BatchState st) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * R) return;
  const uint32_t p = order[start + e / R];
  const uint32_t j = adj[(size_t)p * R + e % R];
  if (j == kSentinel) return;
  const uint32_t s = atomicAdd(&st.fill[j], 1u);
  st.srcs[st.base[j] + s] = p;
}

// Reverse edges of one batch, common case (one wavefront per target, no
// LDS): lane i holds new source i (at most 64) and lane k row entry k; the
// sources not in the row (and not j) are appended in ascending order when
// the row has room.  Other targets go to the deferred list.
__global__ __launch_bounds__(64) void reverse_append_kernel(PruneView v, BatchState st) {
  const int lane = threadIdx.x;
  const uint32_t nt = st.misc[0];
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint32_t j = st.touched[t];
    const uint32_t cnt = st.cnt[j];
    if (st.stats && lane == 0) atomicAdd(&st.stats[LV_BS_REV_TARGETS], 1ull);
    if (cnt > 64u) {
      if (lane == 0) st.deferred[atomicAdd(&st.misc[3], 1u)] = j;
      continue;
    }
    uint32_t *row = v.adj + (size_t)j * (size_t)v.R;
    const uint32_t rv = lane < v.R ? row[lane] : kSentinel;
    const int deg = __popcll(__ballot(rv != kSentinel));
    const uint32_t s = lane < (int)cnt ? st.srcs[st.base[j] + lane] : kSentinel;
    bool add = lane < (int)cnt && s != j && s < v.N;
    for (uint32_t t2 = 0; t2 < cnt; ++t2) {  // is source t2 in the row?
      const uint32_t st_ = (uint32_t)__builtin_amdgcn_readlane((int)s, (int)t2);
      if (__ballot(lane < deg && rv == st_) && lane == (int)t2) add = false;
    }
    const uint64_t am = __ballot(add);
    const int u = deg + __popcll(am);
    if (u > v.R) {
      if (lane == 0) st.deferred[atomicAdd(&st.misc[3], 1u)] = j;
      continue;
    }
    int pos = 0;  // rank among the appended sources (ids are distinct)
    for (uint32_t t2 = 0; t2 < cnt; ++t2) {
      const uint32_t st_ = (uint32_t)__builtin_amdgcn_readlane((int)s, (int)t2);
      pos += (int)(((am >> t2) & 1u) && st_ < s);
    }
    if (add) row[deg + pos] = s;
    if (lane == 0) st.cnt[j] = 0u;
  }
}

// Reverse edges of the deferred targets: the union of the row and the new
// sources, pruned around the target when longer than R.
template <int BITS>
__global__ __launch_bounds__(64) void reverse_kernel(PruneView v, BatchState st) {
  const int lane = threadIdx.x;
  const int M = v.R + kMaxNewSources;
  const PruneLds sm = carve_prune(M, v.R, v.cw);
  const uint32_t nt = st.misc[3];
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const uint32_t j = st.deferred[t];
    const uint32_t cnt = st.cnt[j];
    const uint32_t b0 = st.base[j];
    uint32_t *row = v.adj + (size_t)j * (size_t)v.R;
    wave_sync();
    if (cnt > (uint32_t)kMaxNewSources) {
      if (lane == 0) {
        atomicOr(&st.misc[2], 1u);
        st.cnt[j] = 0u;
      }
      continue;
    }
    // current row (valid ids first) into cid[0..deg)
    const uint32_t rv = lane < v.R ? row[lane] : kSentinel;
    const int deg = __popcll(__ballot(rv != kSentinel));
    if (lane < deg) sm.cid[lane] = rv;
    // new sources, ranked ascending (distinct ids) into csum[], staged in csq[]
    for (uint32_t i = lane; i < cnt; i += 64) {
      sm.csq[i] = st.srcs[b0 + i];
      sm.csum[i] = kSentinel;
    }
    wave_sync();
    for (uint32_t i = lane; i < cnt; i += 64) {
      const uint32_t s = sm.csq[i];
      uint32_t r = 0;
      for (uint32_t k = 0; k < cnt; ++k) r += sm.csq[k] < s;
      sm.csum[r] = s;
    }
    wave_sync();
    // append the sources not in the row (and not j itself), in ascending order
    int u = deg;
    for (uint32_t i0 = 0; i0 < cnt; i0 += 64) {
      const uint32_t i = i0 + lane;
      const uint32_t s = i < cnt ? sm.csum[i] : kSentinel;
      bool add = i < cnt && s != j && s < v.N;
      const uint32_t nc = cnt - i0 < 64u ? cnt - i0 : 64u;
      for (uint32_t t = 0; t < nc; ++t) {  // is source t in the row (lane k holds entry k)?
        const uint32_t st_ = (uint32_t)__builtin_amdgcn_readlane((int)s, (int)t);
        if (__ballot(lane < deg && rv == st_) && lane == (int)t) add = false;
      }
      const uint64_t msk = __ballot(add);
      if (add) sm.cid[u + lane_rank(msk)] = s;
      u += __popcll(msk);
    }
    wave_sync();
    if (u <= v.R) {
      for (int k = lane; k < v.R; k += 64) row[k] = k < u ? sm.cid[k] : kSentinel;
    } else {
      const int nk = prune_core<BITS>(v, j, u, sm, lane);
      for (int k = lane; k < v.R; k += 64) row[k] = k < nk ? sm.kid[k] : kSentinel;
      if (st.stats && lane == 0) {
        atomicAdd(&st.stats[LV_BS_REV_PRUNES], 1ull);
        atomicAdd(&st.stats[LV_BS_REV_CANDS], (unsigned long long)u);
      }
    }
    if (lane == 0) st.cnt[j] = 0u;
  }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

int fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return LV_OK;
  const int64_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

// Device allocations of one build, freed on every exit path.
struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  int alloc(T **out, size_t count) {
    void *p = nullptr;
    LV_CHECK_HIP(hipMalloc(&p, count * sizeof(T) > 0 ? count * sizeof(T) : 1));
    ptrs.push_back(p);
    *out = static_cast<T *>(p);
    return LV_OK;
  }
};

int stride_layout(int32_t stride, int *group, int *vbytes) {
  switch (stride) {
    case 64: *group = 16; *vbytes = 4; return 1;
    case 96: *group = 8; *vbytes = 12; return 1;
    case 128: *group = 16; *vbytes = 8; return 1;
    case 192: *group = 16; *vbytes = 12; return 1;
    case 256: *group = 16; *vbytes = 16; return 1;
    case 512: *group = 64; *vbytes = 8; return 1;
    case 768: *group = 64; *vbytes = 12; return 1;
    case 1024: *group = 64; *vbytes = 16; return 1;
    default: return 0;
  }
}

}  // namespace
}  // namespace lv

extern "C" int lv_graph_build(const void *records, int32_t record_stride, int64_t N, int32_t d,
                              int32_t bits, const uint32_t *order, uint32_t entry,
                              const lv_build_params *params, uint32_t *adjacency, void *stream) {
  using namespace lv;
  clear_error();
  if (!records || !order || !params || !adjacency) LV_FAIL(LV_EINVAL, "NULL argument");
  if (N < 1 || N >= 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "N must be in [1, 2^31-2]");
  if (d < 8 || d % 8 != 0) LV_FAIL(LV_EINVAL, "d must be a positive multiple of 8");
  if (bits != 4 && bits != 8) LV_FAIL(LV_EINVAL, "bits must be 4 or 8");
  const int32_t cb = d * bits / 8;
  if (cb > 4 * kMaxCodeWords)
    LV_FAIL(LV_EUNSUPPORTED, "construction supports at most %d code bytes per record (got %d)",
            4 * kMaxCodeWords, cb);
  int group = 0, vbytes = 0;
  if (!stride_layout(record_stride, &group, &vbytes))
    LV_FAIL(LV_EUNSUPPORTED, "record_stride %d unsupported (use lv_record_stride)",
            record_stride);
  if (record_stride < cb + 8) LV_FAIL(LV_EINVAL, "record_stride smaller than codes + 8");
  const lv_build_params &bp = *params;
  if (bp.R < 1 || bp.R > kMaxR) LV_FAIL(LV_EUNSUPPORTED, "R must be in [1, %d]", kMaxR);
  if (bp.L < 1 || bp.L > LV_MAX_L) LV_FAIL(LV_EINVAL, "L must be in [1, %d]", LV_MAX_L);
  if (bp.passes < 1 || bp.passes > LV_MAX_BUILD_PASSES)
    LV_FAIL(LV_EINVAL, "passes must be in [1, %d]", LV_MAX_BUILD_PASSES);
  for (int t = 0; t < bp.passes; ++t)
    if (!std::isfinite(bp.alphas[t]) || bp.alphas[t] < 0.0)
      LV_FAIL(LV_EINVAL, "alphas[%d] must be finite and >= 0", t);
  if (bp.max_batch < 1) LV_FAIL(LV_EINVAL, "max_batch must be >= 1");
  if (bp.stop_after < 0) LV_FAIL(LV_EINVAL, "stop_after must be >= 0");
  if ((uint64_t)entry >= (uint64_t)N) LV_FAIL(LV_EINVAL, "entry out of range");
  lv_search_params sp{};
  sp.hash_slots = bp.hash_slots ? bp.hash_slots : 2048;
  VisitedCfg vc;
  int rc = visited_config(&sp, &vc);
  if (rc != LV_OK) return rc;
  {  // the insertion order must be a permutation (ids index device arrays)
    std::vector<unsigned char> seen((size_t)N, 0);
    for (int64_t i = 0; i < N; ++i) {
      if ((int64_t)order[i] >= N || seen[order[i]])
        LV_FAIL(LV_EINVAL, "order is not a permutation of 0..N-1 (position %lld)",
                (long long)i);
      seen[order[i]] = 1;
    }
  }
  rc = check_lds(beam_lds_bytes(bp.L, vc.slots), bp.L, vc.slots);
  if (rc != LV_OK) return rc;
  const int R = bp.R, L = bp.L, cw = cb / 4;
  const int pool_stride = L + R;
  const int64_t maxb = bp.max_batch < N ? bp.max_batch : N;
  const size_t lds_fwd = prune_lds_bytes(pool_stride, R, cw);
  const size_t lds_rev = prune_lds_bytes(R + kMaxNewSources, R, cw);
  rc = check_lds(lds_fwd > lds_rev ? lds_fwd : lds_rev, L, vc.slots);
  if (rc != LV_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);

  Scratch sc;
  uint32_t *order_d = nullptr, *pool = nullptr;
  BatchState st{};
  if ((rc = sc.alloc(&order_d, (size_t)N)) != LV_OK) return rc;
  if ((rc = sc.alloc(&pool, (size_t)maxb * pool_stride)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.cnt, (size_t)N)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.fill, (size_t)N)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.base, (size_t)N)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.touched, (size_t)maxb * R)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.srcs, (size_t)maxb * R)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.deferred, (size_t)maxb * R)) != LV_OK) return rc;
  if ((rc = sc.alloc(&st.misc, 4)) != LV_OK) return rc;
  uint32_t *counters = nullptr;
  if (bp.stats) {
    if ((rc = sc.alloc(&st.stats, LV_BUILD_STATS)) != LV_OK) return rc;
    if ((rc = sc.alloc(&counters, (size_t)maxb * 2)) != LV_OK) return rc;
    if ((rc = fill_u32(reinterpret_cast<uint32_t *>(st.stats), 2 * LV_BUILD_STATS, 0u, s)) !=
        LV_OK)
      return rc;
  }
  LV_CHECK_HIP(hipMemcpyAsync(order_d, order, (size_t)N * sizeof(uint32_t),
                              hipMemcpyHostToDevice, s));
  if ((rc = fill_u32(adjacency, N * (int64_t)R, kSentinel, s)) != LV_OK) return rc;
  if ((rc = fill_u32(st.cnt, N, 0u, s)) != LV_OK) return rc;
  if ((rc = fill_u32(st.misc, 4, 0u, s)) != LV_OK) return rc;

  BuildSearchArgs sa{};
  sa.ix.records = static_cast<const unsigned char *>(records);
  sa.ix.stride = record_stride;
  sa.ix.d = d;
  sa.ix.code_bytes = cb;
  sa.ix.adj = adjacency;
  sa.ix.R = R;
  sa.ix.entry = entry;
  sa.ix.N = (uint32_t)N;
  sa.order = order_d;
  sa.L = L;
  sa.pool_stride = pool_stride;
  sa.pool = pool;
  sa.counters = counters;
  sa.stats = st.stats;
  sa.hash_slots = vc.slots;
  sa.probes = vc.probes;
  ForwardArgs fa{};
  fa.v.records = sa.ix.records;
  fa.v.stride = record_stride;
  fa.v.d = d;
  fa.v.cw = cw;
  fa.v.adj = adjacency;
  fa.v.R = R;
  fa.v.N = (uint32_t)N;
  fa.order = order_d;
  fa.pool = pool;
  fa.pool_stride = pool_stride;
  fa.st = st;
  const int app_grid = (int)(maxb * R < 16384 ? maxb * R : 16384);
  const int rev_grid = (int)(maxb * R < 2048 ? maxb * R : 2048);
  const int alloc_grid = (int)((maxb * R + 255) / 256 < 1024 ? (maxb * R + 255) / 256 : 1024);

  int64_t batches = 0;
  for (int pass = 0; pass < bp.passes; ++pass) {
    fa.v.alpha2 = bp.alphas[pass] * bp.alphas[pass];
    int64_t bs = pass == 0 ? 1 : maxb;
    for (int64_t start = 0; start < N;) {
      if (bp.stop_after && batches == bp.stop_after) {
        pass = bp.passes;  // ends both loops
        break;
      }
      const int64_t B = start + bs <= N ? bs : N - start;
      hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, st.misc);
      sa.start = start;
      sa.B = (int32_t)B;
      if ((rc = launch_build_search(bits, group, vbytes, sa, s)) != LV_OK) return rc;
      fa.start = start;
      fa.B = (int32_t)B;
      if (bits == 8)
        hipLaunchKernelGGL(prune_forward_kernel<8>, dim3((unsigned)B), dim3(64), lds_fwd, s, fa);
      else
        hipLaunchKernelGGL(prune_forward_kernel<4>, dim3((unsigned)B), dim3(64), lds_fwd, s, fa);
      hipLaunchKernelGGL(alloc_kernel, dim3(alloc_grid), dim3(256), 0, s, st);
      hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((B * R + 255) / 256)), dim3(256), 0, s,
                         order_d, start, (int32_t)B, adjacency, R, st);
      hipLaunchKernelGGL(reverse_append_kernel, dim3(app_grid), dim3(64), 0, s, fa.v, st);
      if (bits == 8)
        hipLaunchKernelGGL(reverse_kernel<8>, dim3(rev_grid), dim3(64), lds_rev, s, fa.v, st);
      else
        hipLaunchKernelGGL(reverse_kernel<4>, dim3(rev_grid), dim3(64), lds_rev, s, fa.v, st);
      LV_CHECK_LAUNCH();
      ++batches;
      start += B;
      bs = 2 * bs < maxb ? 2 * bs : maxb;
    }
  }
  uint32_t misc[4] = {0, 0, 0, 0};
  LV_CHECK_HIP(hipMemcpyAsync(misc, st.misc, sizeof(misc), hipMemcpyDeviceToHost, s));
  unsigned long long tot[LV_BUILD_STATS] = {};
  if (bp.stats)
    LV_CHECK_HIP(hipMemcpyAsync(tot, st.stats, sizeof(tot), hipMemcpyDeviceToHost, s));
  LV_CHECK_HIP(hipStreamSynchronize(s));
  if (bp.stats)
    for (int i = 0; i < LV_BUILD_STATS; ++i) bp.stats[i] = (int64_t)tot[i];
  if (misc[2])
    LV_FAIL(LV_EUNSUPPORTED,
            "a node received more than %d new edges in one batch; use a smaller max_batch",
            kMaxNewSources);
  return LV_OK;
}
