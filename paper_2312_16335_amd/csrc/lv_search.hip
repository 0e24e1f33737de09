// Graph search on gfx950: one wavefront per query.
//
// Per query (Section 2 "Search"; traversal of Appendix D read as a
// best-first beam with window L):
//   * the candidate window (L entries of float64 score + id, kept sorted by
//     score descending then id ascending) lives in LDS as one buffer that a
//     batch of new candidates is merged into in place: an entry only moves
//     towards the end, by a shift that does not decrease along the window,
//     so 64-entry chunks taken from the end, each read before it is written,
//     never overwrite an entry not yet read;
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
//   * while a hop is processed, the adjacency row of the runner-up
//     unexpanded candidate is already being fetched; when it is still the
//     best candidate at the next hop (the common case late in a search) that
//     hop skips one dependent memory round trip.  Results do not change;
//   * at the end every window entry is re-ranked with <q, secondary> (the
//     whole wavefront streams one secondary row, several rows in flight)
//     and the best k are selected.
// Scores are accumulated in float64: on gfx950 a float64 FMA issues at the
// same rate as an unpacked float32 FMA, and float64 keeps the traversal
// order equal to a float64 reference except at exact ties.
//
// Two kernels share the per-query body: a plain launch with one workgroup
// per query of one request, and a batched launch over the queries of many
// requests (each with its own sub-index, k and L), either one workgroup per
// query or resident wavefronts pulling queries from a device counter.
//
// For batches too small to fill the GPU a third, team launch gives each
// query a workgroup of kTeamWaves wavefronts: the first runs the traversal
// of the multi-expansion body (with one expansion per iteration it is the
// paper's traversal), and every batch of candidates is scored by all of
// them, each wavefront a slice, as is the final re-ranking of the window;
// the others wait at workgroup barriers between batches.  Scores, order and
// results are those of the one-wavefront body.
//
// Graph construction (Appendix A) runs the same body with a database node as
// the query: its own codes take the place of the projected query, a record
// is scored with minus the squared distance of the two LVQ reconstructions,
// and the final window is the result (no re-ranking).
#include "lv_common.h"
#include "lv_l2.h"
#include "lv_search.h"

namespace lv {
namespace {

constexpr uint32_t kExpanded = 0x80000000u;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
constexpr int kFastMerge = 8;  // survivors merged by counting instead of sorting
constexpr int kMaxExpand = 8;  // entries expanded per iteration by the throughput variant
constexpr int kTeamWaves = 4;  // wavefronts per query of the team launch
constexpr size_t kTeamLdsBytes = 16;  // the team's command word, after the visited set

// Everything one query needs besides the index.
struct Job {
  const float *q;    // [D] original query
  const float *qp;   // [d] projected query
  int32_t k, L;
  uint32_t *ids;     // [k]
  float *scores;     // [k]
  uint32_t *counters;  // [2] or nullptr
  uint32_t node;     // construction: the database node searched for
};

// Query-side constants of a construction search: d, the node's delta and
// lo, and the integer sums of its codes and of their squares.
struct BuildQ {
  double d, da, lo, s, ss;
};

// Dynamic LDS of the search kernels.  All per-query LDS state is addressed
// from this array by offsets, so every access compiles to an LDS
// instruction (a pointer chosen at run time between two buffers would
// otherwise fall back to flat addressing).
extern __shared__ __align__(16) unsigned char lv_smem[];

// Layout: window scores [Lmax] f64, batch scores [64] f64, window ids
// [Lmax] u32, batch ids [64] u32, ids being expanded [kMaxExpand] u32,
// visited hash.  The merge positions of the
// sorting merge reuse the batch scores' space (read into registers first).
struct Lds {
  int Lmax;
  __device__ __forceinline__ double *ls() const { return reinterpret_cast<double *>(lv_smem); }
  __device__ __forceinline__ double *cs() const { return ls() + Lmax; }
  __device__ __forceinline__ uint32_t *lid() const {
    return reinterpret_cast<uint32_t *>(cs() + 64);
  }
  __device__ __forceinline__ uint32_t *cid() const { return lid() + Lmax; }
  __device__ __forceinline__ int32_t *lbc() const { return reinterpret_cast<int32_t *>(cs()); }
  __device__ __forceinline__ uint32_t *xid() const { return cid() + 64; }
  __device__ __forceinline__ uint32_t *hash() const { return xid() + kMaxExpand; }
};

__device__ __forceinline__ Lds carve(int Lmax) {
  Lds s;
  s.Lmax = Lmax;
  return s;
}

// Total order of candidates: higher score first, then smaller id.  Bitwise
// operators keep it branch-free across lanes.
__device__ __forceinline__ bool better(double as, uint32_t aid, double bs, uint32_t bid) {
  return (as > bs) | ((as == bs) & (aid < bid));
}

// Order LDS traffic between lanes of one wavefront (a workgroup is one
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

// Index data arrive through memory in the persistent kernel; marking the
// pointers global keeps the loads global (not flat) instructions.
#define LV_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const LV_GLOBAL T *gp(const T *p) {
  return (const LV_GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ LV_GLOBAL T *gpw(T *p) {
  return (LV_GLOBAL T *)p;
}

__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int j) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
}

__device__ __forceinline__ double lane_f64(double v, int j) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = lane_u32((uint32_t)b, j), hi = lane_u32((uint32_t)(b >> 32), j);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// DPP lane patterns (a row is 16 lanes): swap neighbours and pairs within
// each quad, rotate a row right by 4 and by 8 lanes.
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;  // lane i of a half row from lane 7 - i
constexpr int kDppRowRor4 = 0x124;
constexpr int kDppRowRor8 = 0x128;
constexpr int kDppRowBcast15 = 0x142;  // last lane of a row to the next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3

// v moved across lanes by a DPP pattern; rows outside ROWS receive +0.0.
// With all rows enabled every lane is written, so no initial value is needed.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  uint32_t lo, hi;
  if constexpr (ROWS == 0xF) {
    lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  } else {
    lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
    hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF,
                                               false);
  }
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each aligned group of W lanes (8: half a row; 16: one row; 64:
// the wavefront), with DPP moves only (no LDS round trip).  W = 8, 16: every
// lane of a group ends with the group's sum (possibly differing in the last
// bit between lanes, so callers read one fixed lane).  W = 64: row sums are chained
// into lane 63 and broadcast, so every lane returns the same value.
template <int W>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(W == 8 || W == 16 || W == 64, "groups of 8, 16 or 64 lanes");
  v += dpp_f64<kDppQuadXor1>(v);
  v += dpp_f64<kDppQuadXor2>(v);
  if constexpr (W == 8) {
    v += dpp_f64<kDppRowHalfMirror>(v);  // the other quad of the half row
    return v;
  }
  v += dpp_f64<kDppRowRor4>(v);
  v += dpp_f64<kDppRowRor8>(v);
  if constexpr (W == 64) {
    v += dpp_f64<kDppRowBcast15, 0xA>(v);  // rows 1, 3: + previous row
    v += dpp_f64<kDppRowBcast31, 0xC>(v);  // rows 2, 3: + rows 0..1
    v = lane_f64(v, 63);
  }
  return v;
}

// Sum over each aligned group of W lanes (8, 16 or 64) of 32-bit integers
// (modulo 2^32), with DPP adds; every lane of a group ends with its sum.
template <int W>
__device__ __forceinline__ uint32_t group_sum_u32(uint32_t v) {
  static_assert(W == 8 || W == 16 || W == 64, "groups of 8, 16 or 64 lanes");
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppQuadXor1, 0xF, 0xF, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppQuadXor2, 0xF, 0xF, true);
  if constexpr (W == 8) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowHalfMirror, 0xF, 0xF, true);
    return v;
  }
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowRor4, 0xF, 0xF, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowRor8, 0xF, 0xF, true);
  if constexpr (W == 64) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast15, 0xA, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppRowBcast31, 0xC, 0xF, false);
    v = lane_u32(v, 63);
  }
  return v;
}

// Largest value over each aligned group of W lanes, for v >= 0.
template <int W>
__device__ __forceinline__ float group_max_nonneg(float v) {
  static_assert(W == 8 || W == 16 || W == 64, "groups of 8, 16 or 64 lanes");
  auto mx = [](float a, int b) { return fmaxf(a, __int_as_float(b)); };
  v = mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppQuadXor1, 0xF, 0xF, true));
  v = mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppQuadXor2, 0xF, 0xF, true));
  if constexpr (W == 8) {
    return mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppRowHalfMirror, 0xF, 0xF,
                                             true));
  }
  v = mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppRowRor4, 0xF, 0xF, true));
  v = mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppRowRor8, 0xF, 0xF, true));
  if constexpr (W == 64) {  // rows that receive nothing take max(v, +0.0) = v
    v = mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppRowBcast15, 0xA, 0xF,
                                          false));
    v = mx(v, __builtin_amdgcn_update_dpp(0, __float_as_int(v), kDppRowBcast31, 0xC, 0xF,
                                          false));
    v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  }
  return v;
}

template <int V>
struct Chunk {
  uint32_t w[V / 4];
};

constexpr uint32_t kOnes = 0x01010101u;  // one per byte: udot4 with it sums the bytes
constexpr uint32_t kNib = 0x0F0F0F0Fu;   // the low nibble of every byte

__device__ __forceinline__ uint32_t udot4(uint32_t a, uint32_t b, uint32_t acc) {
  return __builtin_amdgcn_udot4(a, b, acc, false);
}

// Query side of the primary scoring in one lane: its code slots t = 0..NQ-1
// are components gl NQ + t.
//
// Search: the projected query on its grid, q~_t = Q_t 2^-s with integers
// |Q_t| <= 2^22 (s from the largest |q_j|: the largest is below 2^(22 - s)),
// held as the three bytes of Q_t + 2^23 (at most 3 * 2^22 < 2^24).  For
// 8-bit codes l[k][w] packs byte k of the offset values of slots 4w..4w+3,
// so that udot4(code dword w, l[k][w]) sums code * byte k over four slots;
// for 4-bit codes l[k][w] (k < 3) covers the low nibbles of dword w (slots
// 8w, 8w+2, 8w+4, 8w+6) and l[3 + k][w] the high nibbles.  Then
// sum_t c_t Q_t = A0 + 2^8 A1 + 2^16 A2 - 2^23 sum_t c_t with Ak the sums of
// code * byte k: integers, exact.  Slots past d have Q_t = 0 (offset bytes
// only), whatever their record bytes hold.
//
// Construction: the searched node's own codes (zero past d) in l[0] (8-bit)
// or its low / high nibbles in l[0] / l[1] (4-bit), and in m the mask of the
// code bits below d, applied to a candidate's bytes for its code sums.
template <int BITS, int V, bool BUILD>
struct QCode {
  static constexpr int NW = V / 4;
  static constexpr int NL = BUILD ? (BITS == 8 ? 1 : 2) : (BITS == 8 ? 3 : 6);
  uint32_t l[NL][NW];
  uint32_t m[BUILD ? NW : 1];
};

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int V>
__device__ __forceinline__ Chunk<V> load_chunk(const LV_GLOBAL unsigned char *p) {
  Chunk<V> c;
  if constexpr (V == 16) {
    const u32x4 t = *reinterpret_cast<const LV_GLOBAL u32x4 *>(p);
    c.w[0] = t[0]; c.w[1] = t[1]; c.w[2] = t[2]; c.w[3] = t[3];
  } else if constexpr (V == 8) {
    const u32x2 t = *reinterpret_cast<const LV_GLOBAL u32x2 *>(p);
    c.w[0] = t[0]; c.w[1] = t[1];
  } else {
    static_assert(V == 4 || V == 12, "record chunk of 4, 8, 12 or 16 bytes");
    const LV_GLOBAL uint32_t *w = reinterpret_cast<const LV_GLOBAL uint32_t *>(p);
#pragma unroll
    for (int i = 0; i < V / 4; ++i) c.w[i] = w[i];
  }
  return c;
}

// Score the nc candidate ids in cid[] into cs[].  Group g of G lanes takes
// candidates g, g + 64/G, ...; U records per group are in flight at once.
// Search: score = delta <c, q~> + lo sum(q~) + <q~, mu> with <c, q~> =
// 2^-s sum_t c_t Q_t (scale = 2^-s; sq, cq the other two terms): the
// integer sum is exact (see QCode), so <c, q~> is exact in float64.
// Groups of 8 or 16 lanes add its parts as 32-bit integers (with 8-bit
// codes a record of at most 256 bytes keeps the low part below 2^32);
// 64-lane groups (records up to 1 KiB) join the parts in float64 per lane
// first, exactly (integers below 2^53).
// BUILD: the query is the searched node's codes, so the sum is the integer
// S_ab; the candidate's S_b and S_bb are summed alongside and the score is
// minus the squared distance.
template <int BITS, int G, int V, bool BUILD = false>
__device__ __forceinline__ void score_batch(const IndexView &ix, const QCode<BITS, V, BUILD> &qc,
                                            double scale, double sq, double cq, const BuildQ &bq,
                                            const uint32_t *cid, double *cs, int nc, int lane) {
  constexpr int NW = V / 4;
  constexpr int RPP = 64 / G;
  constexpr int U = (48 / V) < 2 ? 2 : (48 / V);
  const int gl = lane % G;
  const int grp = lane / G;
  // The record's delta and lo follow its codes.  When both lie in one lane's
  // chunk, that lane (whose code slots past d meet zero query components)
  // writes the score; otherwise lane 0 loads them separately.
  const int cl = ix.code_bytes / V;
  const int cw0 = (ix.code_bytes % V) / 4;
  const bool in_chunk = (ix.code_bytes % V) + 8 <= V && cl < G;
  const int wl = in_chunk ? cl : 0;
  for (int base = 0; base < nc; base += RPP * U) {
    Chunk<V> ch[U];
    uint32_t dlw[U], low[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = base + u * RPP + grp;
      dlw[u] = low[u] = 0u;
      if (base + u * RPP < nc && c < nc) {
        const LV_GLOBAL unsigned char *rec = gp(ix.records) + (size_t)cid[c] * (size_t)ix.stride;
        ch[u] = load_chunk<V>(rec + gl * V);
        if (!in_chunk && gl == 0) {
          const LV_GLOBAL uint32_t *cw =
              reinterpret_cast<const LV_GLOBAL uint32_t *>(rec + ix.code_bytes);
          dlw[u] = cw[0];
          low[u] = cw[1];
        }
      } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) ch[u].w[w] = 0u;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * RPP >= nc) break;  // uniform: no record in this pass
      double acc;
      double sb = 0.0, sbb = 0.0;
      if constexpr (BUILD) {
        uint32_t ab = 0u, s1 = 0u, s2 = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = ch[u].w[w], cm = c & qc.m[w];
          if constexpr (BITS == 8) {
            ab = udot4(c, qc.l[0][w], ab);
            s1 = udot4(cm, kOnes, s1);
            s2 = udot4(cm, cm, s2);
          } else {
            ab = udot4(c & kNib, qc.l[0][w], ab);
            ab = udot4((c >> 4) & kNib, qc.l[1][w], ab);
            const uint32_t e = cm & kNib, o = (cm >> 4) & kNib;
            s1 = udot4(e + o, kOnes, s1);
            s2 = udot4(e, e, s2);
            s2 = udot4(o, o, s2);
          }
        }
        acc = (double)group_sum_u32<G>(ab);
        sb = (double)group_sum_u32<G>(s1);
        sbb = (double)group_sum_u32<G>(s2);
      } else {
        uint32_t a0 = 0u, a1 = 0u, a2 = 0u, as = 0u;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = ch[u].w[w];
          if constexpr (BITS == 8) {
            a0 = udot4(c, qc.l[0][w], a0);
            a1 = udot4(c, qc.l[1][w], a1);
            a2 = udot4(c, qc.l[2][w], a2);
            as = udot4(c, kOnes, as);
          } else {
            const uint32_t e = c & kNib, o = (c >> 4) & kNib;
            a0 = udot4(o, qc.l[3][w], udot4(e, qc.l[0][w], a0));
            a1 = udot4(o, qc.l[4][w], udot4(e, qc.l[1][w], a1));
            a2 = udot4(o, qc.l[5][w], udot4(e, qc.l[2][w], a2));
            as = udot4(e + o, kOnes, as);
          }
        }
        const uint32_t lo32 = a0 + (a1 << 8);   // < 2^32 over the group (G <= 16)
        const uint32_t hi32 = a2 - (as << 7);   // A2 - 2^7 sum(c): a signed 32-bit value
        double S;
        if constexpr (G == 64) {
          S = group_sum<64>(fma((double)(int32_t)hi32, 65536.0, (double)lo32));
        } else {
          S = fma((double)(int32_t)group_sum_u32<G>(hi32), 65536.0,
                  (double)group_sum_u32<G>(lo32));
        }
        acc = S * scale;
      }
      const int c = base + u * RPP + grp;
      if (in_chunk) {  // cw0 is uniform: scalar branches, plain moves
#pragma unroll
        for (int w = 0; w + 1 < NW; ++w) {
          if (cw0 == w) {
            dlw[u] = ch[u].w[w];
            low[u] = ch[u].w[w + 1];
          }
        }
      }
      if (gl == wl && c < nc) {
        const double delta = (double)__uint_as_float(dlw[u]);
        const double lo = (double)__uint_as_float(low[u]);
        if constexpr (BUILD) {
          cs[c] = -lvq_l2(bq.d, bq.da, bq.lo, bq.s, bq.ss, delta, lo, sb, sbb, acc);
        } else {
          cs[c] = delta * acc + lo * sq + cq;
        }
      }
    }
  }
}

// Bitonic sort of one (score, id) pair per lane, best first.  Entries sit
// in lanes [0, n) and the other lanes hold padding (-inf, sentinel), so the
// phases that merge blocks larger than the smallest power of two >= n only
// move padding and are skipped.
__device__ __forceinline__ void sort64(double &s, uint32_t &id, int lane, int n) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
    // lanes from n on hold only padding: once a block of k/2 lanes holds
    // every entry, block 0 is already sorted best first and stays so
    if ((k >> 1) >= n) break;  // uniform
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

// Visited test-and-set.  After `probes` occupied slots the id replaces the
// one in its home slot (the set forgets an older id) and counts as unknown:
// it is scored, and the merge drops it if it is in the window.
// The home slot is the high half of (Knuth's multiplicative hash of n) x
// slots, which for 2^k slots is the hash's top k bits.
__device__ __forceinline__ bool hash_visit(uint32_t *hash, uint32_t slots, int probes,
                                           uint32_t n) {
  const uint32_t h0 = __umulhi(n * 2654435761u, slots);
  uint32_t h = h0;
#pragma unroll 1
  for (int t = 0; t < probes; ++t) {
    const uint32_t old = atomicCAS(&hash[h], kEmpty, n);
    if (old == kEmpty) return true;
    if (old == n) return false;
    h = h + 1u == slots ? 0u : h + 1u;
  }
  atomicExch(&hash[h0], n);
  return true;
}

// Secondary scores of window entries ids[0..nl) into out[], one row at a
// time across the wavefront (16-byte packets, UR rows in flight).  KIND is
// LV_F32, LV_F16, LV_LVQ8, LV_F16_RESID or LV_LVQ8_LEVEL2; an LVQ-8 row is
// scored as delta * <q, c> + lo * sum(q) + <q, sec_mu>, which equals <q, x^>
// for its reconstruction x^ = sec_mu + lo + delta * c.  The packet after the
// codes holds delta and lo; its query components are zero.  A residual row
// (D - d float16 coordinates, q = P_perp q) and a second-level row (d codes,
// q = A q, no centring) add their inner product to the primary score
// already in out[].
template <int KIND>
__device__ __forceinline__ void rerank_rows(const IndexView &ix, const float *q,
                                            const uint32_t *ids, double *out, int nl, int lane) {
  constexpr bool F16 = KIND == LV_F16 || KIND == LV_F16_RESID;
  constexpr bool LVQ = KIND == LV_LVQ8 || KIND == LV_LVQ8_LEVEL2;
  constexpr bool ADD = KIND == LV_F16_RESID || KIND == LV_LVQ8_LEVEL2;
  constexpr int E = F16 ? 8 : (KIND == LV_F32 ? 4 : 16);  // elements per packet
  // components per row
  const int dim = KIND == LV_F16_RESID ? ix.D - ix.d : (KIND == LV_LVQ8_LEVEL2 ? ix.d : ix.D);
  // packets per lane: rows up to 2 KiB (LVQ rows up to 1 KiB)
  constexpr int PPL = LVQ ? 1 : 2;
  constexpr int UR = 4;   // rows in flight
  float qq[PPL][E];
  double sq = 0.0, cq = 0.0;
#pragma unroll
  for (int pk = 0; pk < PPL; ++pk) {
    const int packet = lane + 64 * pk;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = packet * E + e;
      const bool in = packet < ix.sec_packets && j < dim;
      qq[pk][e] = in ? gp(q)[j] : 0.f;
      if constexpr (LVQ) sq += (double)qq[pk][e];
      if constexpr (KIND == LV_LVQ8)
        cq = fma((double)qq[pk][e], in ? (double)gp(ix.sec_mu)[j] : 0.0, cq);
    }
  }
  int cl = 0, cpk = 0;  // lane and packet slot holding an LVQ row's delta and lo
  if constexpr (LVQ) {
    sq = group_sum<64>(sq);
    if constexpr (KIND == LV_LVQ8) cq = group_sum<64>(cq);
    cl = ((dim + 15) / 16) % 64;
    cpk = ((dim + 15) / 16) / 64;
  }
  for (int base = 0; base < nl; base += UR) {
    u32x4 v[UR][PPL];
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      const int idx = base + u;
      const uint32_t id = idx < nl ? (ids[idx] & kIdMask) : 0u;
      const LV_GLOBAL unsigned char *row = gp(ix.sec) + (size_t)id * (size_t)ix.sec_row_bytes;
#pragma unroll
      for (int pk = 0; pk < PPL; ++pk) {
        const int packet = lane + 64 * pk;
        if (idx < nl && packet < ix.sec_packets)
          v[u][pk] = *reinterpret_cast<const LV_GLOBAL u32x4 *>(row + (size_t)packet * 16);
        else
          v[u][pk] = u32x4{0u, 0u, 0u, 0u};
      }
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
      double acc = 0.0;
#pragma unroll
      for (int pk = 0; pk < PPL; ++pk) {
        const uint32_t w[4] = {v[u][pk][0], v[u][pk][1], v[u][pk][2], v[u][pk][3]};
#pragma unroll
        for (int e = 0; e < E; ++e) {
          double x;
          if constexpr (F16)
            x = (double)(float)__builtin_bit_cast(_Float16, (uint16_t)(w[e >> 1] >> (16 * (e & 1))));
          else if constexpr (KIND == LV_F32)
            x = (double)__uint_as_float(w[e]);
          else
            x = (double)((w[e >> 2] >> (8 * (e & 3))) & 0xFFu);
          acc = fma(x, (double)qq[pk][e], acc);
        }
      }
      acc = group_sum<64>(acc);
      if constexpr (LVQ) {
        const uint32_t dw = lane_u32(cpk == 0 ? v[u][0][0] : v[u][PPL - 1][0], cl);
        const uint32_t lw = lane_u32(cpk == 0 ? v[u][0][1] : v[u][PPL - 1][1], cl);
        acc = (double)__uint_as_float(dw) * acc + (double)__uint_as_float(lw) * sq + cq;
      }
      if (lane == 0 && base + u < nl) {
        if constexpr (ADD)
          out[base + u] += acc;
        else
          out[base + u] = acc;
      }
    }
  }
}

// Secondary scores of float16 / float32 rows (KIND LV_F16, LV_F16_RESID or
// LV_F32, as rerank_rows) two rows at a time: half wavefront h scores row
// 2 i + h, lane l of the half holding 16-byte packets l, l + 32, ... (PPH
// of them: rows of at most 32 PPH packets).  Every lane does useful work
// for rows whose packet count is not a multiple of 64, a row in flight
// costs 2 PPH registers instead of 8, so UP pairs (2 UP rows) are gathered
// at once, and the two half sums share one reduction.
template <int KIND, int PPH>
__device__ __forceinline__ void rerank_pairs(const IndexView &ix, const float *q,
                                             const uint32_t *ids, double *out, int nl,
                                             int lane) {
  constexpr bool F16 = KIND == LV_F16 || KIND == LV_F16_RESID;
  constexpr int E = F16 ? 8 : 4;                          // elements per packet
  constexpr int UP = PPH <= 2 ? 4 : 2;  // pairs in flight
  const int dim = KIND == LV_F16_RESID ? ix.D - ix.d : ix.D;
  const int h = lane >> 5, hl = lane & 31;
  float qq[PPH][E];
#pragma unroll
  for (int pk = 0; pk < PPH; ++pk) {
    const int packet = hl + 32 * pk;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = packet * E + e;
      qq[pk][e] = packet < ix.sec_packets && j < dim ? gp(q)[j] : 0.f;
    }
  }
  for (int base = 0; base < nl; base += 2 * UP) {
    u32x4 v[UP][PPH];
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      const int idx = base + 2 * u + h;
      const uint32_t id = idx < nl ? (ids[idx] & kIdMask) : 0u;
      const LV_GLOBAL unsigned char *row = gp(ix.sec) + (size_t)id * (size_t)ix.sec_row_bytes;
#pragma unroll
      for (int pk = 0; pk < PPH; ++pk) {
        const int packet = hl + 32 * pk;
        if (idx < nl && packet < ix.sec_packets)
          v[u][pk] = *reinterpret_cast<const LV_GLOBAL u32x4 *>(row + (size_t)packet * 16);
        else
          v[u][pk] = u32x4{0u, 0u, 0u, 0u};
      }
    }
#pragma unroll
    for (int u = 0; u < UP; ++u) {
      if (base + 2 * u >= nl) break;  // uniform: no row left
      double acc = 0.0;
#pragma unroll
      for (int pk = 0; pk < PPH; ++pk) {
        const uint32_t w[4] = {v[u][pk][0], v[u][pk][1], v[u][pk][2], v[u][pk][3]};
#pragma unroll
        for (int e = 0; e < E; ++e) {
          double x;
          if constexpr (F16)
            x = (double)(float)__builtin_bit_cast(_Float16, (uint16_t)(w[e >> 1] >> (16 * (e & 1))));
          else
            x = (double)__uint_as_float(w[e]);
          acc = fma(x, (double)qq[pk][e], acc);
        }
      }
      // row sums, then rows 0 + 1 and 2 + 3: the half sums land in lanes 31, 63
      acc = group_sum<16>(acc);
      acc += dpp_f64<kDppRowBcast15, 0xA>(acc);
      const int idx = base + 2 * u + h;
      if (hl == 31 && idx < nl) {
        if constexpr (KIND == LV_F16_RESID)
          out[idx] += acc;
        else
          out[idx] = acc;
      }
    }
  }
}

// Rows of 65..96 packets (float16 rows of 513..768 components, float32 rows
// of 257..384) are scored in pairs; other rows one at a time.
template <int KIND>
__device__ __forceinline__ void rerank_pairs_any(const IndexView &ix, const float *q,
                                                 const uint32_t *ids, double *out, int n,
                                                 int lane) {
  if (ix.sec_packets > 64 && ix.sec_packets <= 96)  // uniform
    rerank_pairs<KIND, 3>(ix, q, ids, out, n, lane);
  else
    rerank_rows<KIND>(ix, q, ids, out, n, lane);
}

// The query the re-ranking reads: the full query, or the residual part of
// the projected one (P_perp q), or the projected one itself (second level).
__device__ __forceinline__ const float *rerank_query(const IndexView &ix, const float *qp,
                                                     const float *q) {
  if (ix.sec_kind == LV_F16_RESID) return qp + ix.d;
  if (ix.sec_kind == LV_LVQ8_LEVEL2) return qp;
  return q;
}

// Re-rank entries [0, n) of ids/out with the index's kind of secondaries.
// PAIRS = false keeps every row kind on the one-row path (the team launch,
// whose wavefronts re-rank short slices and whose registers the paired path
// would overflow).
template <bool PAIRS = true>
__device__ __forceinline__ void rerank_any(const IndexView &ix, const float *q,
                                           const uint32_t *ids, double *out, int n, int lane) {
  if (ix.sec_kind == LV_F16) {
    if constexpr (PAIRS)
      rerank_pairs_any<LV_F16>(ix, q, ids, out, n, lane);
    else
      rerank_rows<LV_F16>(ix, q, ids, out, n, lane);
  } else if (ix.sec_kind == LV_LVQ8) {
    rerank_rows<LV_LVQ8>(ix, q, ids, out, n, lane);
  } else if (ix.sec_kind == LV_F16_RESID) {
    if constexpr (PAIRS)
      rerank_pairs_any<LV_F16_RESID>(ix, q, ids, out, n, lane);
    else
      rerank_rows<LV_F16_RESID>(ix, q, ids, out, n, lane);
  } else if (ix.sec_kind == LV_LVQ8_LEVEL2) {
    rerank_rows<LV_LVQ8_LEVEL2>(ix, q, ids, out, n, lane);
  } else {
    if constexpr (PAIRS)
      rerank_pairs_any<LV_F32>(ix, q, ids, out, n, lane);
    else
      rerank_rows<LV_F32>(ix, q, ids, out, n, lane);
  }
}

// Merge the scored batch (cid/cs[0..nc)) into the window of nl <= L
// entries, in place; duplicates of window entries are dropped.  DEDUP also
// drops repeats inside the batch (a batch gathered from several rows can hold
// an id twice when the visited set forgot it in between).
template <bool DEDUP = false>
__device__ __forceinline__ void merge_batch(const Lds &sm, int nc, int L, int &nl, int lane) {
  const double *ls = sm.ls();
  uint32_t *lid = sm.lid();
  double bs = -INFINITY;
  uint32_t bid = kSentinel;
  if (lane < nc) {
    bs = sm.cs()[lane];
    bid = sm.cid()[lane];
  }
  if (nl == L && bid != kSentinel && !better(bs, bid, ls[L - 1], lid[L - 1] & kIdMask)) {
    bs = -INFINITY;
    bid = kSentinel;
  }
  const uint64_t surv = __ballot(bid != kSentinel);
  if (surv == 0) return;
  const int nsurv = __popcll(surv);
  if (nsurv <= kFastMerge && nl <= 256) {
    // Few survivors (the common case once the window is full): a survivor
    // lands at (#window entries better) + (#kept survivors better), a
    // window entry moves down by the kept survivors placed at or before it.
    // The window is read into registers; survivors are broadcast one by one,
    // and every per-survivor decision is a wave-wide mask (the compares'
    // own lane masks, combined in scalar registers).
    const int nt = (nl + 63) >> 6;  // 64-entry chunks in use (uniform)
    double es[4];
    uint32_t er[4], ei[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      const bool ok = e < nl;
      es[t] = ok ? ls[e] : -INFINITY;
      er[t] = ok ? lid[e] : kSentinel;
      ei[t] = er[t] & kIdMask;
    }
    uint64_t keepm = 0;  // lanes of the survivors kept
    int my_lb = 0, my_rank = 0;
    uint64_t rem = surv;
    while (rem) {  // uniform loop over survivors
      const int j = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const double cj = lane_f64(bs, j);
      const uint32_t ij = lane_u32(bid, j);
      // empty slots hold (-inf, sentinel): never better, never equal
      int cnt = 0;
      uint64_t dm = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= nt) break;  // uniform
        const uint64_t gt = __ballot(es[t] > cj), eq = __ballot(es[t] == cj);
        const uint64_t lt = __ballot(ei[t] < ij);
        cnt += __popcll(gt | (eq & lt));
        dm |= __ballot(ei[t] == ij);
      }
      bool keep = dm == 0;  // not already in the window
      if constexpr (DEDUP)  // nor kept earlier from this batch
        keep = keep && (keepm & __ballot(bid == ij)) == 0;
      if (keep) {
        keepm |= 1ull << j;
        my_rank += (bid != kSentinel && better(cj, ij, bs, bid)) ? 1 : 0;
      }
      my_lb = lane == j ? cnt : my_lb;
    }
    const int nkeep = __popcll(keepm);
    if (nkeep == 0) return;
    int sh[4] = {0, 0, 0, 0};  // kept survivors placed at or before window entry t
    for (uint64_t km = keepm; km; km &= km - 1) {
      const int lbj = __builtin_amdgcn_readlane(my_lb, __ffsll((unsigned long long)km) - 1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t >= nt) break;  // uniform
        sh[t] += (lane + 64 * t >= lbj) ? 1 : 0;
      }
    }
    const bool my_keep = (keepm >> lane) & 1;
    // in place: the whole window was read into registers above
    double *ls_w = sm.ls();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t;
      if (e < nl && e + sh[t] < L) {
        ls_w[e + sh[t]] = es[t];
        lid[e + sh[t]] = er[t];
      }
    }
    if (my_keep && my_lb + my_rank < L) {
      ls_w[my_lb + my_rank] = bs;
      lid[my_lb + my_rank] = bid;
    }
    nl = nl + nkeep < L ? nl + nkeep : L;
    wave_sync();
    return;
  }
  sort64(bs, bid, lane, nc);
  int lb = 0;
  bool valid = bid != kSentinel;
  if constexpr (DEDUP) {  // repeats are adjacent after the sort
    const uint32_t pid = (uint32_t)__shfl_up((int)bid, 1, 64);
    if (lane > 0 && pid == bid) valid = false;
  }
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
  if (nv == 0) return;
  const int r = lane_rank(vm);
  if (valid) sm.lbc()[r] = lb;
  wave_sync();
  // in place, 64-entry chunks from the end: entry e moves to e + (number
  // of new entries placed before it), never onto an entry not yet read
  double *ls_w = sm.ls();
  for (int c = (nl - 1) >> 6; c >= 0; --c) {
    const int e = 64 * c + lane;
    if (e < nl) {
      const double se = ls[e];
      const uint32_t ie = lid[e];
      int lo = 0, hi = nv;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sm.lbc()[mid] <= e)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int np = e + lo;
      if (np < L) {
        ls_w[np] = se;
        lid[np] = ie;
      }
    }
  }
  if (valid && lb + r < L) {
    ls_w[lb + r] = bs;
    lid[lb + r] = bid;
  }
  nl = nl + nv < L ? nl + nv : L;
  wave_sync();
}

// Start of wavefront w's slice of a batch of nc candidates in the team
// launch: slices are whole passes of 64 / G records, as even as possible,
// in wavefront order (w = WQ gives nc).
template <int G, int WQ>
__device__ __forceinline__ int team_slice(int nc, int w) {
  constexpr int RPP = 64 / G;
  const int passes = (nc + RPP - 1) / RPP;
  const int per = (passes + WQ - 1) / WQ;
  const int o = w * per * RPP;
  return o < nc ? o : nc;
}

// The team's command word: the LDS word after the visited set.
__device__ __forceinline__ int *team_cmd(const Lds &sm, int hslots) {
  return reinterpret_cast<int *>(sm.hash() + hslots);
}

// The whole search of one query by one wavefront.  BUILD: construction
// search for node job.node; the final window goes to job.ids (L entries,
// padded with the sentinel).  MULTI: the throughput variant that expands up
// to `expand` entries per iteration (not the paper's traversal).
//
// WQ > 1 (team launch, MULTI only): the workgroup has WQ wavefronts and
// the LDS word after the visited set is the team's command word
// (kTeamLdsBytes more per workgroup).  Wavefront 0 (the leader) runs the search; at
// every batch it publishes the candidate count in *cmd and the whole
// workgroup scores the batch between two barriers; after the traversal it
// publishes -2 - (window size), the workgroup re-ranks the window between
// two barriers, and the other wavefronts return.  Every wavefront therefore
// passes the same sequence of barriers.
template <int BITS, int G, int V, bool BUILD = false, bool MULTI = false, int WQ = 1>
__device__ void search_query(const IndexView &ix, const Job &job, const Lds &sm, int hslots,
                             int probes, int expand, int lane) {
  static_assert(WQ == 1 || (MULTI && !BUILD), "team search is the multi-expansion body");
  constexpr int NQ = V * 8 / BITS;
  const int L = job.L;

  // this lane's part of the query side of the scoring (see QCode)
  const int gl = lane % G;
  QCode<BITS, V, BUILD> qc;
  double scale = 1.0, sq = 0.0, cq = 0.0;
  BuildQ bq{};
  if constexpr (BUILD) {
    // the node's own codes (small integers), masked past d
    const LV_GLOBAL unsigned char *rec = gp(ix.records) + (size_t)job.node * (size_t)ix.stride;
    const Chunk<V> ch = load_chunk<V>(rec + gl * V);
    constexpr int CPW = 32 / BITS;  // codes per dword
    uint32_t s1 = 0u, s2 = 0u;
#pragma unroll
    for (int w = 0; w < qc.NW; ++w) {
      uint32_t m = 0u;
#pragma unroll
      for (int i = 0; i < CPW; ++i)
        if (gl * NQ + w * CPW + i < ix.d) m |= ((1u << BITS) - 1u) << (BITS * i);
      qc.m[w] = m;
      const uint32_t c = ch.w[w] & m;
      if constexpr (BITS == 8) {
        qc.l[0][w] = c;
        s1 = udot4(c, kOnes, s1);
        s2 = udot4(c, c, s2);
      } else {
        const uint32_t e = c & kNib, o = (c >> 4) & kNib;
        qc.l[0][w] = e;
        qc.l[1][w] = o;
        s1 = udot4(e + o, kOnes, s1);
        s2 = udot4(o, o, udot4(e, e, s2));
      }
    }
    const LV_GLOBAL float *cw = reinterpret_cast<const LV_GLOBAL float *>(rec + ix.code_bytes);
    bq.d = (double)ix.d;
    bq.da = (double)cw[0];
    bq.lo = (double)cw[1];
    bq.s = (double)lane_u32(group_sum_u32<G>(s1), 0);
    bq.ss = (double)lane_u32(group_sum_u32<G>(s2), 0);
  } else {
    float qv[NQ];
    float am = 0.f;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      // unconditional loads (clamped index) so that all of them are in flight
      const int j = gl * NQ + t;
      const float x = gp(job.qp)[j < ix.d ? j : 0];
      qv[t] = j < ix.d ? x : 0.f;
      am = fmaxf(am, fabsf(qv[t]));
    }
    // the grid: s = 22 - e with max |q_j| = f 2^e, f in [0.5, 1) (e = 0 for 0)
    am = group_max_nonneg<G>(am);
    int e = 0;
    (void)frexpf(am, &e);
    const int sh = 22 - __builtin_amdgcn_readfirstlane(e);
    scale = ldexp(1.0, -sh);
    double sumq = 0.0;
#pragma unroll
    for (int w = 0; w < qc.NW; ++w)
#pragma unroll
      for (int k = 0; k < qc.NL; ++k) qc.l[k][w] = 0u;
#pragma unroll
    for (int t = 0; t < NQ; ++t) {
      const int j = gl * NQ + t;
      const double Qt = rint(ldexp((double)qv[t], sh));  // |Qt| <= 2^22, exact
      sumq += Qt;
      const float mj = gp(ix.mu)[j < ix.d ? j : 0];
      cq = fma(Qt * scale, j < ix.d ? (double)mj : 0.0, cq);
      const uint32_t off = (uint32_t)((int32_t)Qt + (1 << 23));
      constexpr int CPW = 32 / BITS;
      const int w = t / CPW, i = t % CPW;
      const int set = BITS == 8 ? 0 : 3 * (i & 1);  // 4-bit: low / high nibbles
      const int b = BITS == 8 ? i : i >> 1;          // byte of the code dword
#pragma unroll
      for (int k = 0; k < 3; ++k) qc.l[set + k][w] |= ((off >> (8 * k)) & 0xFFu) << (8 * b);
    }
    // the same in every lane after the group reduction: keep them scalar
    sq = lane_f64(group_sum<G>(sumq), 0) * scale;  // exact: |sum| < 2^53
    cq = lane_f64(group_sum<G>(cq), 0);
  }
  if constexpr (WQ > 1) {
    // slice of each batch: whole passes of 64 / G records per wavefront
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (wave != 0) {
      for (;;) {
        __syncthreads();  // the leader has published a batch (or the end)
        const int nc = __builtin_amdgcn_readfirstlane(*team_cmd(sm, hslots));
        if (nc < 0) {  // -2 - nl: re-rank this wavefront's slice of the window, end
          const int nl = -2 - nc;
          const int r0 = team_slice<16, WQ>(nl, wave);
          rerank_any<false>(ix, job.q, sm.lid() + r0, sm.ls() + r0,
                     team_slice<16, WQ>(nl, wave + 1) - r0, lane);
          __syncthreads();  // slices re-ranked
          return;
        }
        const int off = team_slice<G, WQ>(nc, wave);
        const int cnt = team_slice<G, WQ>(nc, wave + 1) - off;
        score_batch<BITS, G, V, BUILD>(ix, qc, scale, sq, cq, bq, sm.cid() + off, sm.cs() + off, cnt,
                                       lane);
        __syncthreads();  // scores written
      }
    }
  }
  for (int i = lane; i < hslots; i += 64) sm.hash()[i] = kEmpty;
  wave_sync();

  // seed the window with the entry node
  if (lane == 0) {
    sm.cid()[0] = ix.entry;
    hash_visit(sm.hash(), (uint32_t)hslots, probes, ix.entry);
  }
  wave_sync();
  score_batch<BITS, G, V, BUILD>(ix, qc, scale, sq, cq, bq, sm.cid(), sm.cs(), 1, lane);
  wave_sync();
  if (lane == 0) {
    sm.ls()[0] = sm.cs()[0];
    sm.lid()[0] = ix.entry;
  }
  wave_sync();
  int nl = 1;
  uint32_t n_exp = 0, n_dist = 1;
  uint32_t pf_id = kSentinel;   // node whose first adjacency chunk is in pf_row
  uint32_t pf_row = kSentinel;
  const uint32_t max_hops = ix.N + 1u;  // every node is expanded at most once

  if constexpr (MULTI) {
    for (uint32_t hop = 0; hop < max_hops; ++hop) {
      // the first `expand` unexpanded entries in window order, flagged and
      // listed in xid[]
      uint32_t *lid = sm.lid();
      int ne = 0;
      for (int base = 0; base < nl && ne < expand; base += 64) {
        const int i = base + lane;
        const uint32_t v = i < nl ? lid[i] : kExpanded;
        const bool un = !(v & kExpanded);
        const uint64_t msk = __ballot(un);
        const int r = lane_rank(msk);
        const int need = expand - ne;
        if (un && r < need) {
          lid[i] = v | kExpanded;
          sm.xid()[ne + r] = v;
        }
        const int c = __popcll(msk);
        ne += c < need ? c : need;
      }
      if (ne == 0) break;
      wave_sync();
      n_exp += (uint32_t)ne;
      // the first 64 ids of every row are requested before any is used
      uint32_t first[kMaxExpand];
#pragma unroll
      for (int e = 0; e < kMaxExpand; ++e) {
        first[e] = kSentinel;
        if (e < ne && lane < ix.R)
          first[e] = gp(ix.adj)[(size_t)sm.xid()[e] * (size_t)ix.R + lane];
      }
      // fresh ids of the rows, in order, collected into batches of <= 64;
      // the batch is scored and merged when the next chunk would not fit,
      // and after the last chunk (one scoring / merge site)
      int nc = 0, e = 0, rb = 0;
      for (;;) {
        const bool more = e < ne;  // uniform
        uint32_t n = kSentinel;
        if (more) {
          if (rb == 0)
            n = first[0];
          else if (rb + lane < ix.R)
            n = gp(ix.adj)[(size_t)sm.xid()[e] * (size_t)ix.R + rb + lane];
        }
        bool fresh = false;
        if (n < ix.N) fresh = hash_visit(sm.hash(), (uint32_t)hslots, probes, n);
        const uint64_t fm = __ballot(fresh);
        const int cnt = __popcll(fm);
        if (!more || nc + cnt > 64) {
          if (nc > 0) {
            wave_sync();
            if constexpr (WQ > 1) {
              if (lane == 0) *team_cmd(sm, hslots) = nc;
              __syncthreads();  // batch and count visible to the workgroup
              score_batch<BITS, G, V, BUILD>(ix, qc, scale, sq, cq, bq, sm.cid(), sm.cs(),
                                             team_slice<G, WQ>(nc, 1), lane);
              __syncthreads();  // every slice scored
            } else {
              score_batch<BITS, G, V, BUILD>(ix, qc, scale, sq, cq, bq, sm.cid(), sm.cs(), nc, lane);
            }
            wave_sync();
            n_dist += nc;
            merge_batch<true>(sm, nc, L, nl, lane);
            nc = 0;
          }
          if (!more) break;
        }
        if (fresh) sm.cid()[nc + lane_rank(fm)] = n;
        nc += cnt;
        rb += 64;
        if (rb >= ix.R) {  // next row: its first chunk moves to first[0]
          rb = 0;
          ++e;
#pragma unroll
          for (int t = 0; t + 1 < kMaxExpand; ++t) first[t] = first[t + 1];
        }
      }
    }
    if constexpr (WQ > 1) {  // the window's size: the team's re-ranking order
      if (lane == 0) *team_cmd(sm, hslots) = -2 - nl;
      __syncthreads();
    }
  } else {
    for (uint32_t hop = 0; hop < max_hops; ++hop) {
      uint32_t *lid = sm.lid();
      // best unexpanded entry = first unexpanded position of the sorted window;
      // the next one is the runner-up whose row is prefetched
      int pos = -1;
      uint32_t p = kSentinel, p2 = kSentinel;
      for (int base = 0; base < nl; base += 64) {
        const int i = base + lane;
        const uint32_t v = i < nl ? lid[i] : kExpanded;
        uint64_t msk = __ballot(!(v & kExpanded));
        if (msk) {
          if (pos < 0) {
            const int b = __ffsll((unsigned long long)msk) - 1;
            pos = base + b;
            p = lane_u32(v, b);
            msk &= msk - 1;
          }
          if (msk) {
            p2 = lane_u32(v, __ffsll((unsigned long long)msk) - 1);
            break;
          }
        }
      }
      if (pos < 0) break;
      if (lane == 0) lid[pos] = p | kExpanded;
      wave_sync();
      ++n_exp;
      const LV_GLOBAL uint32_t *row = gp(ix.adj) + (size_t)p * (size_t)ix.R;
      uint32_t first = kSentinel;
      if (p == pf_id)
        first = pf_row;
      else if (lane < ix.R)
        first = row[lane];
      // prefetch the runner-up's first chunk; consumed at the next hop if it is
      // still the best unexpanded candidate then
      pf_id = p2;
      pf_row = (p2 != kSentinel && lane < ix.R) ? gp(ix.adj)[(size_t)p2 * (size_t)ix.R + lane]
                                                : kSentinel;
      for (int rb = 0; rb < ix.R; rb += 64) {
        uint32_t n = rb == 0 ? first : (rb + lane < ix.R ? row[rb + lane] : kSentinel);
        bool fresh = false;
        if (n < ix.N) fresh = hash_visit(sm.hash(), (uint32_t)hslots, probes, n);
        const uint64_t fm = __ballot(fresh);
        const int nc = __popcll(fm);
        if (nc == 0) continue;
        if (fresh) sm.cid()[lane_rank(fm)] = n;
        wave_sync();
        score_batch<BITS, G, V, BUILD>(ix, qc, scale, sq, cq, bq, sm.cid(), sm.cs(), nc, lane);
        wave_sync();
        n_dist += nc;

        merge_batch(sm, nc, L, nl, lane);
      }
    }
  }

  if constexpr (BUILD) {
    for (int j = lane; j < L; j += 64)
      gpw(job.ids)[j] = j < nl ? (sm.lid()[j] & kIdMask) : kSentinel;
    if (job.counters && lane == 0) {
      gpw(job.counters)[0] = n_exp;
      gpw(job.counters)[1] = n_dist;
    }
    wave_sync();
    return;
  }

  // re-rank the window with the secondary vectors, in place: the secondary
  // score of entry j replaces its primary score, its id loses the flag
  uint32_t *id2 = sm.lid();
  double *s2 = sm.ls();
  if constexpr (WQ > 1) {
    // the team re-ranks too, a slice of whole 4-row passes each
    rerank_any<false>(ix, job.q, id2, s2, team_slice<16, WQ>(nl, 1), lane);
    __syncthreads();  // every slice re-ranked
  } else {
    rerank_any(ix, job.q, id2, s2, nl, lane);
  }
  wave_sync();
  for (int j = lane; j < nl; j += 64) id2[j] &= kIdMask;
  wave_sync();
  for (int t = 0; t < job.k; ++t) {
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
      gpw(job.ids)[t] = bid;
      gpw(job.scores)[t] = bid == kSentinel ? -INFINITY : (float)bs;
    }
    if (bid == kSentinel) {
      for (int t2 = t + 1 + lane; t2 < job.k; t2 += 64) {
        gpw(job.ids)[t2] = kSentinel;
        gpw(job.scores)[t2] = -INFINITY;
      }
      break;
    }
    for (int j = lane; j < nl; j += 64)
      if (id2[j] == bid) id2[j] = kSentinel;
    wave_sync();
  }
  if (job.counters && lane == 0) {
    gpw(job.counters)[0] = n_exp;
    gpw(job.counters)[1] = n_dist;
  }
  wave_sync();
}

struct PlainArgs {
  IndexView ix;
  const float *Q;
  const float *Qp;
  int64_t m;
  int32_t k, L;
  uint32_t *ids;
  float *scores;
  uint32_t *counters;
  int32_t hash_slots;
  int32_t probes;
  int32_t expand;
  int32_t qp_stride;  // floats per projected query (d, or D with residual secondaries)
};

template <int BITS, int G, int V, bool MULTI>
__global__ __launch_bounds__(64) void beam_kernel(PlainArgs a) {
  const int64_t qi = blockIdx.x;
  if (qi >= a.m) return;
  const Lds sm = carve(a.L);
  Job job;
  job.qp = a.Qp + qi * a.qp_stride;
  // residual secondaries are scored with P_perp q, stored after P q
  job.q = rerank_query(a.ix, job.qp, a.Q + qi * a.ix.D);
  job.k = a.k;
  job.L = a.L;
  job.ids = a.ids + qi * a.k;
  job.scores = a.scores + qi * a.k;
  job.counters = a.counters ? a.counters + 2 * qi : nullptr;
  search_query<BITS, G, V, false, MULTI>(a.ix, job, sm, a.hash_slots, a.probes, a.expand,
                                         threadIdx.x);
}

// Team launch: one workgroup of kTeamWaves wavefronts per query (the
// multi-expansion body; expand = 1 is the paper's traversal).
template <int BITS, int G, int V>
__global__ __launch_bounds__(64 * kTeamWaves) void team_kernel(PlainArgs a) {
  const int64_t qi = blockIdx.x;
  if (qi >= a.m) return;  // the same for the whole workgroup
  const Lds sm = carve(a.L);
  Job job;
  job.qp = a.Qp + qi * a.qp_stride;
  job.q = rerank_query(a.ix, job.qp, a.Q + qi * a.ix.D);
  job.k = a.k;
  job.L = a.L;
  job.ids = a.ids + qi * a.k;
  job.scores = a.scores + qi * a.k;
  job.counters = a.counters ? a.counters + 2 * qi : nullptr;
  search_query<BITS, G, V, false, true, kTeamWaves>(a.ix, job, sm, a.hash_slots, a.probes,
                                                    a.expand, (int)(threadIdx.x & 63u));
}

// Batched form over a step's request table.  With a counter (persistent
// launch), resident wavefronts take queries from it until the step's queries
// run out; without one, workgroup b searches query b once (one workgroup per
// query slot, scheduled by the hardware).  Requests are sorted by q_begin; a
// query finds its request by binary search.
// Waves per SIMD the register allocation aims at: 5 (at most 102 VGPRs),
// for 4-bit records too now that a lane's query components are held as
// byte limbs (a few spills of per-query values, outside the search loops).
template <int BITS, int V>
constexpr int batched_waves() { return 5; }

template <int BITS, int G, int V, bool MULTI>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(batched_waves<BITS, V>()))) void batched_kernel(
    const StepHeader *__restrict__ hdr, const IndexView *__restrict__ subs,
    unsigned int *__restrict__ counter, int32_t Lmax, int32_t hash_slots, int32_t probes,
    int32_t expand) {
  const int lane = threadIdx.x;
  const Lds sm = carve(Lmax);
  const int64_t nq = hdr->nq;
  const int32_t nreq = hdr->nreq;
  const Request *req = reinterpret_cast<const Request *>(hdr + 1);
  unsigned int own = blockIdx.x;  // without a counter: this block's query, once
  for (;;) {
    unsigned int u = 0;
    if (counter) {
      if (lane == 0) u = atomicAdd(counter, 1u);
    } else {
      u = own;
      own = 0xFFFFFFFFu;
    }
    // wave-uniform from here on, so request and index fields live in SGPRs
    u = __builtin_amdgcn_readfirstlane(__shfl(u, 0, 64));
    if ((int64_t)u >= nq) break;
    int lo = 0, hi = nreq - 1;  // last request with q_begin <= u
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (req[mid].q_begin <= (int64_t)u)
        lo = mid;
      else
        hi = mid - 1;
    }
    const Request r = req[lo];
    const IndexView ix = subs[r.sub];
    const int64_t j = (int64_t)u - r.q_begin;
    // An opaque copy of the lane id: lane-dependent constants of the search
    // are then recomputed per query instead of being hoisted out of this
    // loop, where they would stay live (and spill) for the kernel's lifetime.
    int lane_q = lane;
    asm volatile("" : "+v"(lane_q));
    Job job;
    job.qp = hdr->Qp + (int64_t)u * hdr->qp_stride;
    job.q = rerank_query(ix, job.qp, hdr->Q + (int64_t)u * ix.D);
    job.k = r.k;
    job.L = r.L;
    job.ids = hdr->ids + r.out_off + j * r.k;
    job.scores = hdr->scores + r.out_off + j * r.k;
    job.counters = hdr->counters ? hdr->counters + 2 * (int64_t)u : nullptr;
    search_query<BITS, G, V, false, MULTI>(ix, job, sm, hash_slots, probes, expand, lane_q);
  }
}

// Construction searches of one batch: workgroup b searches node
// order[start + b] on the graph as it stands (no kernel of the batch writes
// it meanwhile) and writes its pool row: the final window (L ids), then the
// node's current out-neighbours (R ids).
template <int BITS, int G, int V>
__global__ __launch_bounds__(64) void build_search_kernel(BuildSearchArgs a) {
  const int b = blockIdx.x;
  if (b >= a.B) return;
  const uint32_t p = a.order[a.start + b];
  Job job;
  job.q = nullptr;
  job.qp = nullptr;
  job.k = 0;
  job.L = a.L;
  job.ids = a.pool + (size_t)b * (size_t)a.pool_stride;
  job.scores = nullptr;
  job.counters = a.counters ? a.counters + 2 * (size_t)b : nullptr;
  job.node = p;
  search_query<BITS, G, V, true>(a.ix, job, carve(a.L), a.hash_slots, a.probes, 1, threadIdx.x);
  for (int r = threadIdx.x; r < a.ix.R; r += 64)
    gpw(job.ids)[a.L + r] = gp(a.ix.adj)[(size_t)p * (size_t)a.ix.R + r];
  if (a.stats && job.counters && threadIdx.x == 0) {  // the lane that wrote the counters
    atomicAdd(&a.stats[0], 1ull);
    atomicAdd(&a.stats[1], (unsigned long long)job.counters[0]);
    atomicAdd(&a.stats[2], (unsigned long long)job.counters[1]);
  }
}

__global__ void reset_counter_kernel(unsigned int *counter) { *counter = 0u; }

template <int BITS, int G, int V>
int launch_plain_t(const PlainArgs &a, bool team, size_t lds, hipStream_t s) {
  if (team)
    hipLaunchKernelGGL((team_kernel<BITS, G, V>), dim3((unsigned)a.m), dim3(64 * kTeamWaves),
                       lds + kTeamLdsBytes, s, a);
  else if (a.expand > 1)
    hipLaunchKernelGGL((beam_kernel<BITS, G, V, true>), dim3((unsigned)a.m), dim3(64), lds, s,
                       a);
  else
    hipLaunchKernelGGL((beam_kernel<BITS, G, V, false>), dim3((unsigned)a.m), dim3(64), lds, s,
                       a);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

template <int BITS, int G, int V>
int launch_batched_t(const StepHeader *hdr, const IndexView *subs, unsigned int *counter,
                        int Lmax, VisitedCfg vc, size_t lds, int grid, hipStream_t s) {
  if (counter) hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  if (vc.expand > 1)
    hipLaunchKernelGGL((batched_kernel<BITS, G, V, true>), dim3(grid), dim3(64), lds, s, hdr,
                       subs, counter, Lmax, vc.slots, vc.probes, vc.expand);
  else
    hipLaunchKernelGGL((batched_kernel<BITS, G, V, false>), dim3(grid), dim3(64), lds, s, hdr,
                       subs, counter, Lmax, vc.slots, vc.probes, vc.expand);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

template <int BITS, int G, int V>
int occupancy_t(size_t lds, bool multi, int *blocks) {
  const void *k = multi ? reinterpret_cast<const void *>(batched_kernel<BITS, G, V, true>)
                        : reinterpret_cast<const void *>(batched_kernel<BITS, G, V, false>);
  LV_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, 64, lds));
  return LV_OK;
}

// Dispatch on (bits, group, vbytes) to the matching template instance.
template <class F>
int dispatch(int bits, int group, int vbytes, F &&f) {
  const int key = group * 100 + vbytes;
#define LV_CASE(B, GG, VV) \
  if (bits == B && key == GG * 100 + VV) return f.template operator()<B, GG, VV>();
  LV_CASE(8, 16, 4) LV_CASE(8, 8, 12) LV_CASE(8, 16, 8) LV_CASE(8, 16, 12) LV_CASE(8, 16, 16)
  LV_CASE(8, 64, 8) LV_CASE(8, 64, 12) LV_CASE(8, 64, 16)
  LV_CASE(4, 16, 4) LV_CASE(4, 8, 12) LV_CASE(4, 16, 8) LV_CASE(4, 16, 12) LV_CASE(4, 16, 16)
  LV_CASE(4, 64, 8) LV_CASE(4, 64, 12) LV_CASE(4, 64, 16)
#undef LV_CASE
  LV_FAIL(LV_EUNSUPPORTED, "no search kernel for %d-bit records of group %d x %d bytes", bits,
          group, vbytes);
}

struct PlainLaunch {
  const PlainArgs &a;
  bool team;
  size_t lds;
  hipStream_t s;
  template <int B, int GG, int VV>
  int operator()() { return launch_plain_t<B, GG, VV>(a, team, lds, s); }
};

struct BatchedLaunch {
  const StepHeader *hdr;
  const IndexView *subs;
  unsigned int *counter;
  int Lmax;
  VisitedCfg vc;
  size_t lds;
  int grid;
  hipStream_t s;
  template <int B, int GG, int VV>
  int operator()() {
    return launch_batched_t<B, GG, VV>(hdr, subs, counter, Lmax, vc, lds, grid, s);
  }
};

struct BuildLaunch {
  const BuildSearchArgs &a;
  size_t lds;
  hipStream_t s;
  template <int B, int GG, int VV>
  int operator()() {
    hipLaunchKernelGGL((build_search_kernel<B, GG, VV>), dim3((unsigned)a.B), dim3(64), lds, s,
                       a);
    LV_CHECK_LAUNCH();
    return LV_OK;
  }
};

struct Occupancy {
  size_t lds;
  bool multi;
  int *blocks;
  template <int B, int GG, int VV>
  int operator()() { return occupancy_t<B, GG, VV>(lds, multi, blocks); }
};

}  // namespace

IndexView make_view(const lv_index *ix) {
  const lv_index_desc &d = ix->desc;
  IndexView v;
  v.records = static_cast<const unsigned char *>(d.records);
  v.stride = d.record_stride;
  v.d = d.d;
  v.code_bytes = ix->code_bytes;
  v.mu = d.mu;
  v.sec = static_cast<const unsigned char *>(d.secondaries);
  v.D = d.D;
  v.sec_row_bytes = lv_secondary_row_bytes(secondary_dims(d), d.sec_dtype);
  v.sec_packets = ix->sec_packets;
  v.sec_kind = d.sec_dtype;
  v.sec_mu = d.sec_mu;
  v.adj = d.adjacency;
  v.R = d.R;
  v.entry = d.entry;
  v.N = (uint32_t)d.N;
  v.A = d.A;
  return v;
}

int visited_config(const lv_search_params *params, VisitedCfg *cfg) {
  const int hs = params && params->hash_slots ? params->hash_slots : kDefaultHashSlots;
  if (hs < 256 || hs > 65536 || hs % 256)
    LV_FAIL(LV_EINVAL, "hash_slots must be a multiple of 256 in [256, 65536] (got %d)", hs);
  const int pr = params ? params->probes : 0;
  if (pr < 0 || pr > 16) LV_FAIL(LV_EINVAL, "probes must be in [0, 16] (got %d)", pr);
  const int ex = params ? params->expand : 0;
  if (ex < 0 || ex > kMaxExpand)
    LV_FAIL(LV_EINVAL, "expand must be in [0, %d] (got %d)", kMaxExpand, ex);
  cfg->expand = ex > 1 ? ex : 1;
  const int la = params ? params->launch : LV_LAUNCH_PER_QUERY;
  if (la != LV_LAUNCH_PER_QUERY && la != LV_LAUNCH_PERSISTENT && la != LV_LAUNCH_TEAM)
    LV_FAIL(LV_EINVAL, "launch must be LV_LAUNCH_PER_QUERY, LV_LAUNCH_PERSISTENT or "
                       "LV_LAUNCH_TEAM (got %d)", la);
  cfg->team = la == LV_LAUNCH_TEAM;
  cfg->slots = hs;
  // small sets (occupancy matters): few probes; large sets: nearly exact
  cfg->probes = pr ? pr : (hs >= 4096 ? 8 : 2);
  return LV_OK;
}

size_t beam_lds_bytes(int L, int slots) {
  return (size_t)L * 12 + 64 * 12 + 4 * kMaxExpand + (size_t)4 * (size_t)slots;
}

int check_lds(size_t lds, int L, int slots) {
  int dev = 0, lds_max = 0;
  LV_CHECK_HIP(hipGetDevice(&dev));
  LV_CHECK_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (lds > (size_t)lds_max)
    LV_FAIL(LV_EINVAL, "window %d with %d hash slots needs %zu bytes of LDS (limit %d)", L,
            slots, lds, lds_max);
  return LV_OK;
}

int launch_beam(const lv_index *ix, const float *Q, const float *Qp, int64_t m, int32_t k,
                int32_t L, uint32_t *ids, float *scores, uint32_t *counters,
                const lv_search_params *params, hipStream_t stream) {
  VisitedCfg vc;
  int rc = visited_config(params, &vc);
  if (rc != LV_OK) return rc;
  if (m == 0) return LV_OK;
  if (m > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "at most 2^31-1 queries per call");
  const size_t lds = beam_lds_bytes(L, vc.slots);
  rc = check_lds(lds + (vc.team ? kTeamLdsBytes : 0), L, vc.slots);
  if (rc != LV_OK) return rc;
  PlainArgs a;
  a.ix = make_view(ix);
  a.Q = Q;
  a.Qp = Qp;
  a.m = m;
  a.k = k;
  a.L = L;
  a.ids = ids;
  a.scores = scores;
  a.counters = counters;
  a.hash_slots = vc.slots;
  a.probes = vc.probes;
  a.expand = vc.expand;
  a.qp_stride = ix->qp_width;
  PlainLaunch f{a, vc.team, lds, stream};
  return dispatch(ix->desc.bits, ix->group, ix->vbytes, f);
}

int launch_batched(int bits, int group, int vbytes, const StepHeader *hdr,
                      const IndexView *subs, unsigned int *counter, int Lmax, VisitedCfg vc,
                      int grid, hipStream_t stream) {
  const size_t lds = beam_lds_bytes(Lmax, vc.slots);
  BatchedLaunch f{hdr, subs, counter, Lmax, vc, lds, grid, stream};
  return dispatch(bits, group, vbytes, f);
}

int launch_build_search(int bits, int group, int vbytes, const BuildSearchArgs &a,
                        hipStream_t stream) {
  if (a.B <= 0) return LV_OK;
  const size_t lds = beam_lds_bytes(a.L, a.hash_slots);
  BuildLaunch f{a, lds, stream};
  return dispatch(bits, group, vbytes, f);
}

int batched_occupancy(int bits, int group, int vbytes, int Lmax, VisitedCfg vc, int *blocks) {
  const size_t lds = beam_lds_bytes(Lmax, vc.slots);
  int rc = check_lds(lds, Lmax, vc.slots);
  if (rc != LV_OK) return rc;
  Occupancy f{lds, vc.expand > 1, blocks};
  return dispatch(bits, group, vbytes, f);
}

}  // namespace lv
