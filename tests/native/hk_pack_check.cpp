// Checks of the host hop-list packer (row (a1)), built with the address and
// undefined-behaviour sanitizers and run on a CPU by test_native_sanitizers.py.
// Prints "hk_pack: <n> checks passed" and exits 0, or names the failed check.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>

#include "hk_pack.hpp"

using be::hkpack::pack_system;
using be::hkpack::Packed;
using cd = std::complex<double>;

static int n_checks = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    ++n_checks;                                                            \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      std::exit(1);                                                        \
    }                                                                      \
  } while (0)

struct List {
  int32_t N = 0, dim = 0;
  std::vector<int32_t> i, j, R;
  std::vector<double> t;
  void add(int32_t a, int32_t b, std::vector<int32_t> r, cd v) {
    i.push_back(a);
    j.push_back(b);
    for (int d = 0; d < dim; ++d) R.push_back(r[d]);
    t.push_back(v.real());
    t.push_back(v.imag());
  }
  void add_h(int32_t a, int32_t b, std::vector<int32_t> r, cd v) {  // entry and its Hermitian partner
    add(a, b, r, v);
    std::vector<int32_t> m(r.size());
    for (size_t d = 0; d < r.size(); ++d) m[d] = -r[d];
    add(b, a, m, std::conj(v));
  }
  int64_t nnz() const { return int64_t(i.size()); }
  std::string pack(Packed &pk, int32_t *np) const {
    return pack_system(N, dim, nnz(), i.data(), j.data(), R.data(), t.data(), pk, np);
  }
};

// Dense H(k) (row-major N x N) from the raw entries, and from the packed
// pairs of the system that starts at pair p0.
static std::vector<cd> dense_raw(const List &L, const double *k) {
  std::vector<cd> H(size_t(L.N) * L.N);
  for (int64_t e = 0; e < L.nnz(); ++e) {
    double x = 0;
    for (int d = 0; d < L.dim; ++d) x += k[d] * L.R[e * L.dim + d];
    H[size_t(L.i[e]) * L.N + L.j[e]] += cd(L.t[2 * e], L.t[2 * e + 1]) * std::polar(1.0, 2 * M_PI * x);
  }
  return H;
}
static std::vector<cd> dense_packed(const Packed &pk, size_t p0, int32_t np, int32_t N, const double *k) {
  std::vector<cd> H(size_t(N) * N);
  for (size_t p = p0; p < p0 + size_t(np); ++p) {
    const int32_t e1 = p + 1 < pk.start.size() ? pk.start[p + 1] : int32_t(pk.R.size());
    cd v = 0;
    for (int32_t e = pk.start[p]; e < e1; ++e) {
      const double x = k[0] * pk.R[e].x + k[1] * pk.R[e].y + k[2] * pk.R[e].z;
      v += cd(pk.t[e].re, pk.t[e].im) * std::polar(1.0, 2 * M_PI * x);
    }
    H[size_t(pk.rc[p].r) * N + pk.rc[p].c] = v;
    if (pk.rc[p].r != pk.rc[p].c) H[size_t(pk.rc[p].c) * N + pk.rc[p].r] = std::conj(v);
  }
  return H;
}

static void check_layout(const Packed &pk, size_t p0, int32_t np) {
  for (size_t p = p0; p < p0 + size_t(np); ++p) {
    CHECK(pk.rc[p].r <= pk.rc[p].c);
    if (p > p0) {
      const auto &a = pk.rc[p - 1], &b = pk.rc[p];
      CHECK(a.c < b.c || (a.c == b.c && a.r < b.r));  // by column, then row, no repeats
    }
    const int32_t e1 = p + 1 < pk.start.size() ? pk.start[p + 1] : int32_t(pk.R.size());
    CHECK(pk.start[p] < e1);
    for (int32_t e = pk.start[p] + 1; e < e1; ++e) {
      const auto &a = pk.R[e - 1], &b = pk.R[e];
      CHECK(std::tie(a.x, a.y, a.z) < std::tie(b.x, b.y, b.z));  // merged: distinct R
      CHECK(b.w == 0);
    }
  }
}

int main() {
  // ---- two-band list (QWZ-like): packs, merges, reproduces H(k)
  {
    List L;
    L.N = 2;
    L.dim = 2;
    L.add(0, 0, {0, 0}, 1.5);
    L.add(1, 1, {0, 0}, -1.5);
    L.add_h(0, 0, {1, 0}, 0.5);
    L.add_h(1, 1, {1, 0}, -0.5);
    L.add_h(0, 1, {1, 0}, cd(0, -0.5));
    L.add_h(0, 1, {0, 1}, -0.5);
    L.add_h(0, 1, {0, 1}, -0.25);  // duplicate key: merged to -0.75
    Packed pk;
    int32_t np = -1;
    CHECK(L.pack(pk, &np).empty());
    CHECK(np == 3);  // pairs (0,0), (0,1), (1,1)
    check_layout(pk, 0, np);
    CHECK(pk.rc[0].r == 0 && pk.rc[0].c == 0 && pk.rc[1].r == 0 && pk.rc[1].c == 1 && pk.rc[2].r == 1);
    const double k[3] = {0.3, -0.15, 0.0};
    auto A = dense_raw(L, k), B = dense_packed(pk, 0, np, 2, k);
    for (size_t e = 0; e < A.size(); ++e) CHECK(std::abs(A[e] - B[e]) < 1e-13);
  }
  // ---- rejections leave the packed arrays unchanged
  {
    List good;
    good.N = 3;
    good.dim = 1;
    good.add_h(0, 2, {1}, cd(0.2, 0.1));
    Packed pk;
    int32_t np = 0;
    CHECK(good.pack(pk, &np).empty());
    const size_t n_rc = pk.rc.size(), n_R = pk.R.size();
    auto rejected = [&](const List &L, const char *what) {
      int32_t np2 = -7;
      const std::string why = L.pack(pk, &np2);
      CHECK(why.find(what) != std::string::npos);
      CHECK(np2 == -7 && pk.rc.size() == n_rc && pk.R.size() == n_R && pk.start.size() == n_rc);
    };
    List a = good;
    a.add(0, 1, {0}, 1.0);  // no partner
    rejected(a, "not Hermitian");
    List b = good;
    b.add_h(0, 3, {0}, 1.0);  // orbital index N
    rejected(b, "out of range");
    List c = good;
    c.add_h(-1, 0, {0}, 1.0);
    rejected(c, "out of range");
    List d = good;
    d.add_h(0, 1, {0}, cd(NAN, 0));
    rejected(d, "non-finite");
    List e = good;
    e.add_h(0, 1, {0}, cd(0, INFINITY));
    rejected(e, "non-finite");
    List f = good;  // -R of INT32_MIN does not exist
    f.add(0, 1, {std::numeric_limits<int32_t>::min()}, 1.0);
    rejected(f, "lattice vector");
    List g = good;  // duplicates whose sum overflows
    g.add_h(1, 2, {0}, 1e308);
    g.add_h(1, 2, {0}, 1e308);
    rejected(g, "not Hermitian");
    List h = good;
    h.dim = 0;
    rejected(h, "bad N/dim");
    List h4 = good;
    h4.dim = 4;
    rejected(h4, "bad N/dim");
    List n0 = good;
    n0.N = 0;
    rejected(n0, "bad N/dim");
    int32_t np3 = 0;
    CHECK(!pack_system(3, 1, 2, nullptr, nullptr, nullptr, nullptr, pk, &np3).empty());
  }
  // ---- extreme lattice vectors with their partners, an empty list
  {
    List L;
    L.N = 1;
    L.dim = 3;
    L.add_h(0, 0, {std::numeric_limits<int32_t>::max(), -5, 7}, cd(0.1, 0.2));
    Packed pk;
    int32_t np = 0;
    CHECK(L.pack(pk, &np).empty() && np == 1 && pk.R.size() == 2);
    check_layout(pk, 0, np);
    List E;
    E.N = 4;
    E.dim = 2;
    CHECK(E.pack(pk, &np).empty() && np == 0);
  }
  // ---- random Hermitian lists with duplicates: layout and H(k) agree with the raw sum
  std::mt19937_64 rng(20231);
  for (int trial = 0; trial < 300; ++trial) {
    List L;
    L.N = 1 + int32_t(rng() % 20);
    L.dim = 1 + int32_t(rng() % 3);
    const int n = int(rng() % 150);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    for (int e = 0; e < n; ++e) {
      std::vector<int32_t> r(L.dim);
      for (auto &x : r) x = int32_t(rng() % 5) - 2;
      const int32_t a = int32_t(rng() % L.N), b = int32_t(rng() % L.N);
      const cd v(U(rng), U(rng));
      if (a == b && std::all_of(r.begin(), r.end(), [](int32_t x) { return x == 0; }))
        L.add(a, a, r, v.real());  // on-site: real
      else
        L.add_h(a, b, r, v);
      if (rng() % 4 == 0) L.add_h(a, b, r, v * 0.5);  // a duplicate key now and then
    }
    Packed pk;
    pk.rc.push_back({0, 0});  // something already packed before this system
    pk.start.push_back(0);
    pk.R.push_back({0, 0, 0, 0});
    pk.t.push_back({0.0, 0.0});
    int32_t np = 0;
    CHECK(L.pack(pk, &np).empty());
    CHECK(pk.rc.size() == size_t(1 + np) && pk.start.size() == pk.rc.size());
    check_layout(pk, 1, np);
    double k[3] = {U(rng), U(rng), U(rng)};
    for (int d = L.dim; d < 3; ++d) k[d] = 0.0;
    auto A = dense_raw(L, k), B = dense_packed(pk, 1, np, L.N, k);
    for (size_t e = 0; e < A.size(); ++e) CHECK(std::abs(A[e] - B[e]) < 1e-12);
  }
  std::printf("hk_pack: %d checks passed\n", n_checks);
  return 0;
}
