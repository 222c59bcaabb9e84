// Row (a1): host packer of one hopping list (the lattice-gauge Bloch sum of
// Sec. II-A needs each amplitude with its orbital pair and lattice vector).
// Plain C++ with no HIP types or calls, so that it is also built on its own
// and run under the address and undefined-behaviour sanitizers on a CPU.
//
// Packing: duplicate (i, j, R) keys are merged (amplitudes added), the list
// is checked to be Hermitian ((i, j, R, t) needs (j, i, -R, conj t) within
// 1e-12 of the largest amplitude), and the upper triangle (i <= j) is kept,
// grouped into (row, col) pairs sorted by column, then row, then R; each pair
// lists its entries (R, t). The output arrays have the memory layout of
// HIP's int2, int32, int4 and double2 vectors, which the library uploads as
// they are.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <string>
#include <tuple>
#include <vector>

namespace be {
namespace hkpack {

struct PairRC {  // layout of int2: (row, col), row <= col
  int32_t r, c;
};
struct EntR {  // layout of int4: lattice vector (x, y, z), w = 0
  int32_t x, y, z, w;
};
struct EntT {  // layout of double2: amplitude (re, im)
  double re, im;
};

// Packed systems, appended one after another: pair p of all systems has
// entries start[p] .. start[p + 1] - 1 of R and t (the caller appends the
// final sentinel after the last system).
struct Packed {
  std::vector<PairRC> rc;
  std::vector<int32_t> start;
  std::vector<EntR> R;
  std::vector<EntT> t;
};

struct Ent {
  int32_t i, j, R[3];
  double tr, ti;
};

inline bool key_less(const Ent &a, const Ent &b) {
  // column-major grouping: by j, then i, then R
  return std::tie(a.j, a.i, a.R[0], a.R[1], a.R[2]) < std::tie(b.j, b.i, b.R[0], b.R[1], b.R[2]);
}
inline bool key_eq(const Ent &a, const Ent &b) {
  return a.i == b.i && a.j == b.j && a.R[0] == b.R[0] && a.R[1] == b.R[1] && a.R[2] == b.R[2];
}

// Appends one system's pairs and entries to out and sets *n_pairs. Entry e
// has orbitals i[e], j[e], lattice vector R[e*dim .. e*dim+dim-1] and
// amplitude (t[2e], t[2e+1]). Returns an empty string, or the reason the
// list is rejected (out is then left as it was).
inline std::string pack_system(int32_t N, int32_t dim, int64_t nnz, const int32_t *i, const int32_t *j,
                               const int32_t *R, const double *t, Packed &out, int32_t *n_pairs) {
  if (N <= 0 || dim < 1 || dim > 3 || nnz < 0 || (nnz > 0 && (!i || !j || !R || !t)))
    return "bad N/dim/nnz or null arrays";
  std::vector<Ent> ents(static_cast<size_t>(nnz));
  double tmax = 0.0;
  for (int64_t e = 0; e < nnz; ++e) {
    Ent x;
    x.i = i[e];
    x.j = j[e];
    if (x.i < 0 || x.i >= N || x.j < 0 || x.j >= N) return "orbital index out of range";
    for (int d = 0; d < 3; ++d) {
      x.R[d] = d < dim ? R[e * dim + d] : 0;
      // -R must exist for the partner entry
      if (x.R[d] == std::numeric_limits<int32_t>::min()) return "lattice vector component out of range";
    }
    x.tr = t[2 * e];
    x.ti = t[2 * e + 1];
    if (!std::isfinite(x.tr) || !std::isfinite(x.ti)) return "non-finite amplitude";
    tmax = std::max(tmax, std::hypot(x.tr, x.ti));
    ents[static_cast<size_t>(e)] = x;
  }
  std::sort(ents.begin(), ents.end(), key_less);
  std::vector<Ent> merged;
  for (const Ent &x : ents) {
    if (!merged.empty() && key_eq(merged.back(), x)) {
      merged.back().tr += x.tr;
      merged.back().ti += x.ti;
    } else {
      merged.push_back(x);
    }
  }
  const double tol = 1e-12 * std::max(tmax, 1e-300);
  for (const Ent &x : merged) {
    Ent key = x;
    key.i = x.j;
    key.j = x.i;
    for (int d = 0; d < 3; ++d) key.R[d] = -x.R[d];
    auto it = std::lower_bound(merged.begin(), merged.end(), key, key_less);
    double pr = 0.0, pi = 0.0;
    if (it != merged.end() && key_eq(*it, key)) {
      pr = it->tr;
      pi = it->ti;
    }
    if (!(std::hypot(pr - x.tr, pi + x.ti) <= tol))  // also rejects a sum that overflowed
      return "not Hermitian (entry (" + std::to_string(x.i) + "," + std::to_string(x.j) + ") lacks its partner)";
  }
  size_t kept = 0;
  for (const Ent &x : merged) kept += x.i <= x.j;
  if (out.R.size() + kept > size_t(std::numeric_limits<int32_t>::max())) return "too many entries";
  int32_t np = 0;
  for (size_t a = 0; a < merged.size();) {
    const Ent &x = merged[a];
    if (x.i > x.j) {
      ++a;
      continue;
    }
    out.rc.push_back({x.i, x.j});
    out.start.push_back(static_cast<int32_t>(out.R.size()));
    size_t b = a;
    while (b < merged.size() && merged[b].i == x.i && merged[b].j == x.j) {
      out.R.push_back({merged[b].R[0], merged[b].R[1], merged[b].R[2], 0});
      out.t.push_back({merged[b].tr, merged[b].ti});
      ++b;
    }
    ++np;
    a = b;
  }
  *n_pairs = np;
  return std::string();
}

}  // namespace hkpack
}  // namespace be
