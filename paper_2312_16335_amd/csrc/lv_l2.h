// Squared Euclidean distance between the LVQ reconstructions of two primary
// records, as graph construction uses it (Section 2 "Graph construction":
// only the primary vectors take part; Appendix A: search and pruning).
//
// With y^ = mu + lo + delta * c, mu cancels; for records a and b with
// e = lo_a - lo_b and integer code sums S_a = sum c_a, S_aa = sum c_a^2,
// S_ab = sum c_a c_b over the d components,
//   ||y^_a - y^_b||^2 = d e^2 + delta_a^2 S_aa + delta_b^2 S_bb
//                       - 2 delta_a delta_b S_ab + 2 e (delta_a S_a - delta_b S_b).
// The integer sums are exact; the float64 operations below run in one fixed
// order and grouping with contraction off, so every kernel that calls this
// (the construction search and the pruning) takes the same decisions.
#pragma once

namespace lv {

__device__ __forceinline__ double lvq_l2(double d, double da, double loa, double sa, double saa,
                                         double db, double lob, double sb, double sbb,
                                         double sab) {
#pragma clang fp contract(off)
  const double e = loa - lob;
  double t = d * (e * e);
  t = t + (da * da) * saa;
  t = t + (db * db) * sbb;
  t = t - 2.0 * ((da * db) * sab);
  t = t + 2.0 * (e * (da * sa - db * sb));
  return t;
}

}  // namespace lv
