// Graph search on gfx950: one wavefront per query.
//
// Per query (Section 2 "Search"; traversal of Appendix C read as a
// best-first beam with window L):
//   * the candidate window (L entries of float64 score + id, kept sorted by
//     score descending then id ascending) lives in LDS, double-buffered so a
//     batch of new candidates merges in one parallel pass;
//   * the visited set is an LDS open-addressed hash of node ids.  It may
//     forget (bounded probing): a forgotten node is scored again, and the
//     merge drops it if it is already in the window.  A node that left the
//     window earlier was worse than L others and the L-th score never
//     decreases, so the final window is the same as with an exact set;
//   * per expansion the adjacency row is read with one 4-byte id per lane,
//     unvisited ids are compacted with a ballot, and groups of G lanes each
//     gather one primary record (G lanes x V bytes, one load per lane) and
//     dequantise-and-dot it against the projected query held in registers:
//     s(n) = delta_n * sum_j q'_j c_nj + lo_n * sum_j q'_j + <q', mu>, which
//     equals <q', y^_n> for the LVQ reconstruction y^_n;
//   * the batch is sorted across lanes (bitonic), merged with the window by
//     binary search, duplicates dropped, and the window truncated to L;
//   * at the end every window entry is re-ranked with <q, secondary> (the
//     whole wavefront streams one secondary row, several rows in flight)
//     and the best k are selected.
// Scores are accumulated in float64: on gfx950 a float64 FMA issues at the
// same rate as an unpacked float32 FMA, and float64 keeps the traversal
// order equal to a float64 reference except at exact ties.
#include "lv_common.h"

namespace lv {
namespace {

constexpr uint32_t kExpanded = 0x80000000u;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
constexpr int kProbes = 16;

struct BeamArgs {
  const unsigned char *records;
  int64_t stride;
  int32_t d;
  int32_t code_bytes;
  const float *mu;
  const unsigned char *sec;
  int32_t D;
  int32_t sec_row_bytes;
  int32_t sec_packets;
  const uint32_t *adj;
  int32_t R;
  uint32_t entry;
  uint32_t N;
  const float *Q;
  const float *Qp;
  int64_t m;
  int32_t k;
  int32_t L;
  uint32_t *out_ids;
  float *out_scores;
  uint32_t *counters;
  int32_t hash_log2;
  uint32_t max_hops;
};

__device__ __forceinline__ bool better(double as, uint32_t aid, double bs, uint32_t bid) {
  return as > bs || (as == bs && aid < bid);
}

// Order LDS traffic between lanes of one wavefront (the workgroup is one
// wavefront; LDS operations of a wave complete in issue order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int W>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = 1; o < W; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// V-byte chunk of a record: V / 4 dwords.
template <int V>
struct Chunk {
  uint32_t w[V / 4];
};

template <int V>
__device__ __forceinline__ Chunk<V> load_chunk(const unsigned char *p) {
  Chunk<V> c;
  if constexpr (V == 4) {
    c.w[0] = *reinterpret_cast<const uint32_t *>(p);
  } else if constexpr (V == 8) {
    uint2 t = *reinterpret_cast<const uint2 *>(p);
    c.w[0] = t.x; c.w[1] = t.y;
  } else if constexpr (V == 12) {
    uint3 t = *reinterpret_cast<const uint3 *>(p);
    c.w[0] = t.x; c.w[1] = t.y; c.w[2] = t.z;
  } else {
    static_assert(V == 16, "record chunk of 4, 8, 12 or 16 bytes");
    uint4 t = *reinterpret_cast<const uint4 *>(p);
    c.w[0] = t.x; c.w[1] = t.y; c.w[2] = t.z; c.w[3] = t.w;
  }
  return c;
}

template <int BITS, int V>
__device__ __forceinline__ uint32_t code_at(const Chunk<V> &c, int t) {
  if constexpr (BITS == 8) {
    return (c.w[t >> 2] >> (8 * (t & 3))) & 0xFFu;
  } else {
    return (c.w[t >> 3] >> (4 * (t & 7))) & 0xFu;
  }
}

// Score the nc candidate ids in cid[] into cs[].  Group g of G lanes takes
// candidates g, g + 64/G, ...; U records per group are in flight at once.
template <int BITS, int G, int V>
__device__ __forceinline__ void score_batch(const BeamArgs &a, const double (&qv)[V * 8 / BITS],
                                            double sq, double cq, const uint32_t *cid, double *cs,
                                            int nc, int lane) {
  constexpr int NQ = V * 8 / BITS;
  constexpr int RPP = 64 / G;
  constexpr int U = (96 / V) < 2 ? 2 : (96 / V);
  const int gl = lane % G;
  const int grp = lane / G;
  for (int base = 0; base < nc; base += RPP * U) {
    Chunk<V> ch[U];
    uint2 dl[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = base + u * RPP + grp;
      if (c < nc) {
        const unsigned char *rec = a.records + (size_t)cid[c] * (size_t)a.stride;
        ch[u] = load_chunk<V>(rec + gl * V);
        if (gl == 0) {
          const uint32_t *cw = reinterpret_cast<const uint32_t *>(rec + a.code_bytes);
          dl[u] = make_uint2(cw[0], cw[1]);
        }
      } else {
#pragma unroll
        for (int w = 0; w < V / 4; ++w) ch[u].w[w] = 0u;
        dl[u] = make_uint2(0u, 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double acc = 0.0;
#pragma unroll
      for (int t = 0; t < NQ; ++t) acc = fma((double)code_at<BITS, V>(ch[u], t), qv[t], acc);
      acc = group_sum<G>(acc);
      const int c = base + u * RPP + grp;
      if (gl == 0 && c < nc) {
        const double delta = (double)__uint_as_float(dl[u].x);
        const double lo = (double)__uint_as_float(dl[u].y);
        cs[c] = delta * acc + lo * sq + cq;
      }
    }
  }
}

// Bitonic sort of one (score, id) pair per lane, best first.
__device__ __forceinline__ void sort64(double &s, uint32_t &id, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const double ps = __shfl_xor(s, j, 64);
      const uint32_t pid = (uint32_t)__shfl_xor((int)id, j, 64);
      const bool keep_better = ((lane & k) == 0) == ((lane & j) == 0);
      const bool pb = better(ps, pid, s, id);
      if (keep_better == pb) {
        s = ps;
        id = pid;
      }
    }
  }
}

__device__ __forceinline__ bool hash_visit(uint32_t *hash, int log2h, uint32_t n) {
  const uint32_t mask = (1u << log2h) - 1u;
  uint32_t h = (n * 2654435761u) >> (32 - log2h);
#pragma unroll 1
  for (int t = 0; t < kProbes; ++t) {
    const uint32_t old = atomicCAS(&hash[h], kEmpty, n);
    if (old == kEmpty) return true;
    if (old == n) return false;
    h = (h + 1u) & mask;
  }
  return true;  // unknown: score it; the merge drops it if it is in the window
}

template <bool F16>
__device__ __forceinline__ void rerank_rows(const BeamArgs &a, const float *q, const uint32_t *ids,
                                            double *out, int nl, int lane) {
  constexpr int E = F16 ? 8 : 4;  // elements per 16-byte packet
  constexpr int PPL = 2;          // packets per lane (rows up to 2 KiB)
  constexpr int UR = 4;           // rows in flight
  float qq[PPL][E];
#pragma unroll
  for (int pk = 0; pk < PPL; ++pk) {
    const int packet = lane + 64 * pk;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = packet * E + e;
      qq[pk][e] = (packet < a.sec_packets && j < a.D) ? q[j] : 0.f;
    }
  }
  for (int base = 0; base < nl; base += UR) {
    uint4 v[UR][PPL];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int idx = base + u;
      const uint32_t id = idx < nl ? (ids[idx] & kIdMask) : 0u;
      const unsigned char *row = a.sec + (size_t)id * (size_t)a.sec_row_bytes;
#pragma unroll
      for (int pk = 0; pk < PPL; ++pk) {
        const int packet = lane + 64 * pk;
        if (idx < nl && packet < a.sec_packets)
          v[u][pk] = *reinterpret_cast<const uint4 *>(row + (size_t)packet * 16);
        else
          v[u][pk] = make_uint4(0u, 0u, 0u, 0u);
      }
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      double acc = 0.0;
#pragma unroll
      for (int pk = 0; pk < PPL; ++pk) {
        const uint32_t w[4] = {v[u][pk].x, v[u][pk].y, v[u][pk].z, v[u][pk].w};
#pragma unroll
        for (int e = 0; e < E; ++e) {
          float x;
          if constexpr (F16) {
            const uint16_t hbits = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
            x = (float)__builtin_bit_cast(_Float16, hbits);
          } else {
            x = __uint_as_float(w[e]);
          }
          acc = fma((double)x, (double)qq[pk][e], acc);
        }
      }
      acc = group_sum<64>(acc);
      if (lane == 0 && base + u < nl) out[base + u] = acc;
    }
  }
}

template <int BITS, int G, int V>
__global__ __launch_bounds__(64) void beam_kernel(BeamArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NQ = V * 8 / BITS;
  const int lane = threadIdx.x;
  const int64_t qi = blockIdx.x;
  if (qi >= a.m) return;
  const int L = a.L;
  double *ls_buf[2];
  uint32_t *lid_buf[2];
  ls_buf[0] = reinterpret_cast<double *>(smem);
  ls_buf[1] = ls_buf[0] + L;
  double *cs = ls_buf[1] + L;
  lid_buf[0] = reinterpret_cast<uint32_t *>(cs + 64);
  lid_buf[1] = lid_buf[0] + L;
  uint32_t *cid = lid_buf[1] + L;
  int32_t *lbc = reinterpret_cast<int32_t *>(cid + 64);
  uint32_t *hash = reinterpret_cast<uint32_t *>(lbc + 64);
  const int hslots = 1 << a.hash_log2;

  // projected query slice of this lane, float64
  const int gl = lane % G;
  double qv[NQ];
  double sq = 0.0, cq = 0.0;
  {
    const float *qp = a.Qp + qi * a.d;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int j = gl * NQ + t;
      const double x = j < a.d ? (double)qp[j] : 0.0;
      qv[t] = x;
      sq += x;
      if (j < a.d) cq = fma(x, (double)a.mu[j], cq);
    }
    sq = group_sum<G>(sq);
    cq = group_sum<G>(cq);
  }
  for (int i = lane; i < hslots; i += 64) hash[i] = kEmpty;
  wave_sync();

  // seed the window with the entry node
  if (lane == 0) {
    cid[0] = a.entry;
    hash_visit(hash, a.hash_log2, a.entry);
  }
  wave_sync();
  score_batch<BITS, G, V>(a, qv, sq, cq, cid, cs, 1, lane);
  wave_sync();
  if (lane == 0) {
    ls_buf[0][0] = cs[0];
    lid_buf[0][0] = a.entry;
  }
  wave_sync();
  int nl = 1;
  int cur = 0;
  uint32_t n_exp = 0, n_dist = 1;

  for (uint32_t hop = 0; hop < a.max_hops; ++hop) {
    double *ls = ls_buf[cur];
    uint32_t *lid = lid_buf[cur];
    // best unexpanded entry = first unexpanded position of the sorted window
    int pos = -1;
    for (int base = 0; base < nl; base += 64) {
      const int i = base + lane;
      const bool un = i < nl && !(lid[i] & kExpanded);
      const uint64_t msk = __ballot(un);
      if (msk) {
        pos = base + __ffsll((unsigned long long)msk) - 1;
        break;
      }
    }
    if (pos < 0) break;
    const uint32_t p = lid[pos];
    wave_sync();
    if (lane == 0) lid[pos] = p | kExpanded;
    wave_sync();
    ++n_exp;
    const uint32_t *row = a.adj + (size_t)p * (size_t)a.R;
    for (int rb = 0; rb < a.R; rb += 64) {
      uint32_t n = kSentinel;
      if (rb + lane < a.R) n = row[rb + lane];
      bool fresh = false;
      if (n < a.N) fresh = hash_visit(hash, a.hash_log2, n);
      const uint64_t fm = __ballot(fresh);
      const int nc = __popcll(fm);
      if (nc == 0) continue;
      if (fresh) cid[lane_rank(fm)] = n;
      wave_sync();
      score_batch<BITS, G, V>(a, qv, sq, cq, cid, cs, nc, lane);
      wave_sync();
      n_dist += nc;

      // merge the scored batch into the window
      ls = ls_buf[cur];
      lid = lid_buf[cur];
      double bs = -INFINITY;
      uint32_t bid = kSentinel;
      if (lane < nc) {
        bs = cs[lane];
        bid = cid[lane];
      }
      if (nl == L && bid != kSentinel &&
          !better(bs, bid, ls[L - 1], lid[L - 1] & kIdMask)) {
        bs = -INFINITY;
        bid = kSentinel;
      }
      if (__ballot(bid != kSentinel) == 0) continue;
      sort64(bs, bid, lane);
      int lb = 0;
      bool valid = bid != kSentinel;
      if (valid) {
        int lo = 0, hi = nl;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (better(ls[mid], lid[mid] & kIdMask, bs, bid))
            lo = mid + 1;
          else
            hi = mid;
        }
        lb = lo;
        if (lo < nl && (lid[lo] & kIdMask) == bid) valid = false;  // already in the window
      }
      const uint64_t vm = __ballot(valid);
      const int nv = __popcll(vm);
      if (nv == 0) continue;
      const int r = lane_rank(vm);
      if (valid) lbc[r] = lb;
      wave_sync();
      double *ls_n = ls_buf[cur ^ 1];
      uint32_t *lid_n = lid_buf[cur ^ 1];
      for (int j = lane; j < nl; j += 64) {
        int lo = 0, hi = nv;  // count of new entries placed before window entry j
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (lbc[mid] <= j)
            lo = mid + 1;
          else
            hi = mid;
        }
        const int np = j + lo;
        if (np < L) {
          ls_n[np] = ls[j];
          lid_n[np] = lid[j];
        }
      }
      if (valid && lb + r < L) {
        ls_n[lb + r] = bs;
        lid_n[lb + r] = bid;
      }
      nl = nl + nv < L ? nl + nv : L;
      cur ^= 1;
      wave_sync();
    }
  }

  // re-rank the window with the secondary vectors
  {
    const uint32_t *lid = lid_buf[cur];
    double *s2 = ls_buf[cur ^ 1];
    uint32_t *id2 = lid_buf[cur ^ 1];
    const float *q = a.Q + qi * a.D;
    if (a.sec_row_bytes == a.D * 2)
      rerank_rows<true>(a, q, lid, s2, nl, lane);
    else
      rerank_rows<false>(a, q, lid, s2, nl, lane);
    for (int j = lane; j < nl; j += 64) id2[j] = lid[j] & kIdMask;
    wave_sync();
    // selection of the best k
    for (int t = 0; t < a.k; ++t) {
      double bs = -INFINITY;
      uint32_t bid = kSentinel;
      for (int j = lane; j < nl; j += 64) {
        const uint32_t id = id2[j];
        if (id != kSentinel && better(s2[j], id, bs, bid)) {
          bs = s2[j];
          bid = id;
        }
      }
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const double ps = __shfl_xor(bs, o, 64);
        const uint32_t pid = (uint32_t)__shfl_xor((int)bid, o, 64);
        if (better(ps, pid, bs, bid)) {
          bs = ps;
          bid = pid;
        }
      }
      if (lane == 0) {
        a.out_ids[qi * a.k + t] = bid;
        a.out_scores[qi * a.k + t] = bid == kSentinel ? -INFINITY : (float)bs;
      }
      if (bid == kSentinel) {
        for (int t2 = t + 1 + lane; t2 < a.k; t2 += 64) {
          a.out_ids[qi * a.k + t2] = kSentinel;
          a.out_scores[qi * a.k + t2] = -INFINITY;
        }
        break;
      }
      for (int j = lane; j < nl; j += 64)
        if (id2[j] == bid) id2[j] = kSentinel;
      wave_sync();
    }
  }
  if (a.counters && lane == 0) {
    a.counters[2 * qi] = n_exp;
    a.counters[2 * qi + 1] = n_dist;
  }
}

size_t beam_lds_bytes(int L, int log2h) {
  return (size_t)L * 24 + 64 * 16 + ((size_t)4 << log2h);
}

template <int BITS, int G, int V>
int launch_t(const BeamArgs &args, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((beam_kernel<BITS, G, V>), dim3((unsigned)args.m), dim3(64), lds, stream,
                     args);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

}  // namespace

int launch_beam(const lv_index *ix, const float *Q, const float *Qp, int64_t m, int32_t k,
                int32_t L, uint32_t *ids, float *scores, uint32_t *counters,
                const lv_search_params *params, hipStream_t stream) {
  const lv_index_desc &dsc = ix->desc;
  int hs = params && params->hash_slots ? params->hash_slots : 4096;
  if (hs < 256 || hs > 65536 || (hs & (hs - 1)))
    LV_FAIL(LV_EINVAL, "hash_slots must be a power of two in [256, 65536] (got %d)", hs);
  int log2h = 0;
  while ((1 << log2h) < hs) ++log2h;
  if (m == 0) return LV_OK;
  if (m > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "at most 2^31-1 queries per call");
  BeamArgs a;
  a.records = static_cast<const unsigned char *>(dsc.records);
  a.stride = dsc.record_stride;
  a.d = dsc.d;
  a.code_bytes = ix->code_bytes;
  a.mu = dsc.mu;
  a.sec = static_cast<const unsigned char *>(dsc.secondaries);
  a.D = dsc.D;
  a.sec_row_bytes = dsc.D * (dsc.sec_dtype == LV_F16 ? 2 : 4);
  a.sec_packets = ix->sec_packets;
  a.adj = dsc.adjacency;
  a.R = dsc.R;
  a.entry = dsc.entry;
  a.N = (uint32_t)dsc.N;
  a.Q = Q;
  a.Qp = Qp;
  a.m = m;
  a.k = k;
  a.L = L;
  a.out_ids = ids;
  a.out_scores = scores;
  a.counters = counters;
  a.hash_log2 = log2h;
  a.max_hops = (uint32_t)dsc.N + 1u;  // every node is expanded at most once
  const size_t lds = beam_lds_bytes(L, log2h);
  int dev = 0, lds_max = 0;
  LV_CHECK_HIP(hipGetDevice(&dev));
  LV_CHECK_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (lds > (size_t)lds_max)
    LV_FAIL(LV_EINVAL, "window %d with %d hash slots needs %zu bytes of LDS (limit %d)", L, hs,
            lds, lds_max);
  const int key = ix->group * 100 + ix->vbytes;
  if (dsc.bits == 8) {
    switch (key) {
      case 1604: return launch_t<8, 16, 4>(a, lds, stream);
      case 1608: return launch_t<8, 16, 8>(a, lds, stream);
      case 1612: return launch_t<8, 16, 12>(a, lds, stream);
      case 1616: return launch_t<8, 16, 16>(a, lds, stream);
      case 6408: return launch_t<8, 64, 8>(a, lds, stream);
      case 6412: return launch_t<8, 64, 12>(a, lds, stream);
      case 6416: return launch_t<8, 64, 16>(a, lds, stream);
    }
  } else {
    switch (key) {
      case 1604: return launch_t<4, 16, 4>(a, lds, stream);
      case 1608: return launch_t<4, 16, 8>(a, lds, stream);
      case 1612: return launch_t<4, 16, 12>(a, lds, stream);
      case 1616: return launch_t<4, 16, 16>(a, lds, stream);
      case 6408: return launch_t<4, 64, 8>(a, lds, stream);
      case 6412: return launch_t<4, 64, 12>(a, lds, stream);
      case 6416: return launch_t<4, 64, 16>(a, lds, stream);
    }
  }
  LV_FAIL(LV_EUNSUPPORTED, "no search kernel for record stride %d", dsc.record_stride);
}

}  // namespace lv
