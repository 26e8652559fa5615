// Code constructions: rotated surface code and bivariate-bicycle codes.
//
// Rotated surface code [[d^2,1,d]] (Supplementary Note 2).  Plaquette (i, j),
// i, j in -1..d-1, covers data (i,j) NW, (i,j+1) NE, (i+1,j) SW, (i+1,j+1) SE
// where they exist; type X when i+j is even, else Z.  Bulk plaquettes are kept,
// the top and bottom boundaries keep X plaquettes and the left and right
// boundaries keep Z plaquettes, giving (d^2-1)/2 checks of each type.  The CX
// schedule avoids hook errors along the logicals (X checks NW, NE, SW, SE; Z
// checks NW, SW, NE, SE; both types share the 4 layers).  Z_L = Z on data row 0.
//
// Bivariate-bicycle codes (Supplementary Note 3, Table IV): x = S_l (x) I_m,
// y = I_l (x) S_m with S the cyclic shift S[r][(r+1) mod j] = 1, so the
// monomial x^a y^b maps index (i, j) = (r / m, r % m) to ((i+a) mod l, (j+b) mod m).
// A = a(x,y), B = b(x,y), H_X = [A|B], H_Z = [B^T|A^T].  Every monomial is a
// permutation, so every term is one collision-free CX layer.  The round uses
// the interleaved depth-7 cycle of the bivariate-bicycle memory experiments the
// paper builds on (Methods, "Simulation"): at each step every X check applies
// one term (an A term on left data or a B term on right data) and every Z check
// one term on the other half of the data (a B^T term on left data or an A^T
// term on right data); X checks idle at the first step, Z checks at the last.
//
// Logical Z basis of a BB code: the rows of the reduced row echelon form of
// ker(H_X), taken in order and kept when independent of rowspace(H_Z) and of
// the rows already kept.  The RREF of a subspace is unique, so the basis is
// fixed by that definition.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace tmcs {

static inline bool getbit(const BitRow& r, int j) { return (r[j >> 6] >> (j & 63)) & 1ull; }
static inline void flipbit(BitRow& r, int j) { r[j >> 6] ^= 1ull << (j & 63); }
static inline void xor_into(BitRow& a, const BitRow& b) {
  for (size_t w = 0; w < a.size(); ++w) a[w] ^= b[w];
}

int gf2_rank_rows(std::vector<BitRow> rows, int ncols) {
  int r = 0;
  const int n = (int)rows.size();
  for (int c = 0; c < ncols && r < n; ++c) {
    int piv = -1;
    for (int i = r; i < n; ++i)
      if (getbit(rows[i], c)) { piv = i; break; }
    if (piv < 0) continue;
    std::swap(rows[r], rows[piv]);
    for (int i = r + 1; i < n; ++i)
      if (getbit(rows[i], c)) xor_into(rows[i], rows[r]);
    ++r;
  }
  return r;
}

// Reduced row echelon form (pivot = lowest column index of each row).
static std::vector<BitRow> rref_rows(std::vector<BitRow> rows, int ncols, std::vector<int>* pivots) {
  int r = 0;
  const int n = (int)rows.size();
  std::vector<int> piv;
  for (int c = 0; c < ncols && r < n; ++c) {
    int p = -1;
    for (int i = r; i < n; ++i)
      if (getbit(rows[i], c)) { p = i; break; }
    if (p < 0) continue;
    std::swap(rows[r], rows[p]);
    for (int i = 0; i < n; ++i)
      if (i != r && getbit(rows[i], c)) xor_into(rows[i], rows[r]);
    piv.push_back(c);
    ++r;
  }
  rows.resize(r);
  if (pivots) *pivots = piv;
  return rows;
}

static BitRow row_from_support(const std::vector<int>& supp, int n) {
  BitRow r((n + 63) / 64, 0ull);
  for (int j : supp) flipbit(r, j);
  return r;
}

static std::vector<BitRow> kernel_rref(const std::vector<std::vector<int>>& h, int n) {
  std::vector<BitRow> rows;
  for (auto& s : h) rows.push_back(row_from_support(s, n));
  std::vector<int> piv;
  std::vector<BitRow> R = rref_rows(rows, n, &piv);
  std::vector<char> is_piv(n, 0);
  for (int c : piv) is_piv[c] = 1;
  std::vector<BitRow> ker;
  for (int f = 0; f < n; ++f) {
    if (is_piv[f]) continue;
    BitRow v((n + 63) / 64, 0ull);
    flipbit(v, f);
    for (size_t i = 0; i < R.size(); ++i)
      if (getbit(R[i], f)) flipbit(v, piv[i]);
    ker.push_back(v);
  }
  return rref_rows(ker, n, nullptr);
}

static void surface_code(int d, CodeBlock* c) {
  c->kind = TMCS_SC;
  c->n = d * d;
  c->k = 1;
  std::vector<std::array<int, 4>> xs, zs;
  for (int i = -1; i < d; ++i) {
    for (int j = -1; j < d; ++j) {
      const bool bulk = i >= 0 && i <= d - 2 && j >= 0 && j <= d - 2;
      const bool is_x = (((i + j) % 2) + 2) % 2 == 0;
      const bool tb = (i == -1 || i == d - 1) && j >= 0 && j <= d - 2;
      const bool lr = (j == -1 || j == d - 1) && i >= 0 && i <= d - 2;
      if (!(bulk || (tb && is_x) || (lr && !is_x))) continue;
      std::array<int, 4> cs;
      const int ci[4][2] = {{i, j}, {i, j + 1}, {i + 1, j}, {i + 1, j + 1}};
      for (int k = 0; k < 4; ++k) {
        const int a = ci[k][0], b = ci[k][1];
        cs[k] = (a >= 0 && a < d && b >= 0 && b < d) ? a * d + b : -1;
      }
      (is_x ? xs : zs).push_back(cs);
    }
  }
  c->nx = (int)xs.size();
  c->nz = (int)zs.size();
  auto supports = [](const std::vector<std::array<int, 4>>& ps) {
    std::vector<std::vector<int>> h;
    for (auto& cs : ps) {
      std::vector<int> s;
      for (int q : cs)
        if (q >= 0) s.push_back(q);
      std::sort(s.begin(), s.end());
      h.push_back(s);
    }
    return h;
  };
  c->hx = supports(xs);
  c->hz = supports(zs);
  const int xo[4] = {0, 1, 2, 3};  // NW NE SW SE
  const int zo[4] = {0, 2, 1, 3};  // NW SW NE SE
  c->layers = 4;
  c->xs.assign(4, {});
  c->zs.assign(4, {});
  for (int t = 0; t < 4; ++t) {
    for (int r = 0; r < c->nx; ++r)
      if (xs[r][xo[t]] >= 0) c->xs[t].push_back({r, xs[r][xo[t]]});
    for (int r = 0; r < c->nz; ++r)
      if (zs[r][zo[t]] >= 0) c->zs[t].push_back({r, zs[r][zo[t]]});
  }
  std::vector<int> row0;
  for (int j = 0; j < d; ++j) row0.push_back(j);
  c->lz = {row0};
}

static tmcs_status bb_code(const tmcs_circuit_spec& s, CodeBlock* c) {
  const int l = s.bb_l, m = s.bb_m;
  if (l < 1 || m < 1 || l * m > (1 << 20))
    return fail(TMCS_EINVAL, "bb_l and bb_m must be positive (l*m <= 2^20)");
  const int h = l * m;
  c->kind = TMCS_BB;
  c->n = 2 * h;
  c->nx = c->nz = h;
  auto perm = [&](int a, int b) {
    std::vector<int> p(h);
    for (int r = 0; r < h; ++r) {
      const int i = r / m, j = r % m;
      const int aa = ((a % l) + l) % l, bbm = ((b % m) + m) % m;
      p[r] = ((i + aa) % l) * m + (j + bbm) % m;
    }
    return p;
  };
  std::vector<std::vector<int>> pa, pb;
  for (int k = 0; k < 3; ++k) {
    pa.push_back(perm(s.bb_a[k][0], s.bb_a[k][1]));
    pb.push_back(perm(s.bb_b[k][0], s.bb_b[k][1]));
  }
  // H_X row r: left data pa_k[r], right data h + pb_k[r] (mod-2 sum of terms)
  std::vector<std::vector<int>> hx(h), hz(h);
  for (int r = 0; r < h; ++r) {
    std::vector<int> cnt;
    auto toggle = [](std::vector<int>& v, int q) {
      auto it = std::find(v.begin(), v.end(), q);
      if (it == v.end()) v.push_back(q); else v.erase(it);
    };
    for (int k = 0; k < 3; ++k) toggle(hx[r], pa[k][r]);
    for (int k = 0; k < 3; ++k) toggle(hx[r], h + pb[k][r]);
    std::sort(hx[r].begin(), hx[r].end());
  }
  // H_Z = [B^T | A^T]: Z check r touches left data c with B[c][r] = 1, i.e.
  // c = pb_k^{-1}(r), and right data c with A[c][r] = 1.
  std::vector<std::vector<int>> ia(3, std::vector<int>(h)), ib(3, std::vector<int>(h));
  for (int k = 0; k < 3; ++k)
    for (int r = 0; r < h; ++r) { ia[k][pa[k][r]] = r; ib[k][pb[k][r]] = r; }
  for (int r = 0; r < h; ++r) {
    auto toggle = [](std::vector<int>& v, int q) {
      auto it = std::find(v.begin(), v.end(), q);
      if (it == v.end()) v.push_back(q); else v.erase(it);
    };
    for (int k = 0; k < 3; ++k) toggle(hz[r], ib[k][r]);
    for (int k = 0; k < 3; ++k) toggle(hz[r], h + ia[k][r]);
    std::sort(hz[r].begin(), hz[r].end());
  }
  c->hx = hx;
  c->hz = hz;
  // interleaved depth-7 cycle: step t applies X term X_STEPS[t] (0-2: A_k on left
  // data, 3-5: B_k on right data) and Z term Z_STEPS[t] (0-2: B_k^T on left data,
  // 3-5: A_k^T on right data) to every check; -1 leaves that check type idle
  static const int X_STEPS[7] = {-1, 1, 4, 3, 5, 0, 2};
  static const int Z_STEPS[7] = {3, 5, 0, 1, 2, 4, -1};
  c->layers = 7;
  c->xs.assign(7, {});
  c->zs.assign(7, {});
  for (int t = 0; t < 7; ++t)
    for (int r = 0; r < h; ++r) {
      const int xt = X_STEPS[t], zt = Z_STEPS[t];
      if (xt >= 0) c->xs[t].push_back({r, xt < 3 ? pa[xt][r] : h + pb[xt - 3][r]});
      if (zt >= 0) c->zs[t].push_back({r, zt < 3 ? ib[zt][r] : h + ia[zt - 3][r]});
    }
  const int n = c->n;
  std::vector<BitRow> X, Z;
  for (auto& sp : hx) X.push_back(row_from_support(sp, n));
  for (auto& sp : hz) Z.push_back(row_from_support(sp, n));
  const int rx = gf2_rank_rows(X, n), rz = gf2_rank_rows(Z, n);
  c->k = n - rx - rz;
  std::vector<BitRow> ker = kernel_rref(hx, n);
  std::vector<BitRow> acc = Z;
  int have = rz;
  for (auto& v : ker) {
    if ((int)c->lz.size() == c->k) break;
    acc.push_back(v);
    const int rr = gf2_rank_rows(acc, n);
    if (rr > have) {
      have = rr;
      std::vector<int> supp;
      for (int j = 0; j < n; ++j)
        if (getbit(v, j)) supp.push_back(j);
      c->lz.push_back(supp);
    } else {
      acc.pop_back();
    }
  }
  return TMCS_OK;
}

tmcs_status make_code(const tmcs_circuit_spec& s, CodeBlock* out) {
  if (s.code == TMCS_SC) {
    if (s.d < 3 || (s.d % 2) == 0 || s.d > 201)
      return fail(TMCS_EINVAL, "surface-code distance must be odd, 3 <= d <= 201");
    surface_code(s.d, out);
    return TMCS_OK;
  }
  if (s.code == TMCS_BB) return bb_code(s, out);
  return fail(TMCS_EINVAL, "unknown code family");
}

}  // namespace tmcs
