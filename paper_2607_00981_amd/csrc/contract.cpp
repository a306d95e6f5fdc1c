// Contraction planner: label bookkeeping on the host, all arithmetic in the
// strided GEMM and permute kernels.
#include "contract.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace cct {

DT dense(double* p, std::initializer_list<long long> dims) {
  DT t;
  t.p = p;
  t.nd = (int)dims.size();
  int i = 0;
  for (long long d : dims) t.dim[i++] = d;
  long long s = 1;
  for (int k = t.nd - 1; k >= 0; --k) {
    t.st[k] = s;
    s *= t.dim[k];
  }
  return t;
}

DT strided(double* p, std::initializer_list<long long> dims, std::initializer_list<long long> strides) {
  DT t;
  t.p = p;
  t.nd = (int)dims.size();
  int i = 0;
  for (long long d : dims) t.dim[i++] = d;
  i = 0;
  for (long long s : strides) t.st[i++] = s;
  return t;
}

double* Arena::alloc(size_t n) {
  const size_t bytes = ((n * sizeof(double) + 255) / 256) * 256;
  if (top_ + bytes > cap_) return nullptr;
  double* p = (double*)(base_ + top_);
  top_ += bytes;
  peak_ = std::max(peak_, top_);
  return p;
}

namespace {

struct Lab {
  char c;
  long long dim;
  long long sa, sb, sc;  // stride in A, B, C (0 if absent)
};

int find(const char* l, char c) {
  const char* p = std::strchr(l, c);
  return p ? (int)(p - l) : -1;
}

// Collapse an ordered label group (outermost first) for one tensor into at
// most two levels.  which: 0 = A, 1 = B, 2 = C.
bool collapse(const std::vector<Lab>& g, int which, Idx2& out, long long& total) {
  struct Comp { long long size, stride; };
  std::vector<Comp> comps;
  total = 1;
  for (int i = (int)g.size() - 1; i >= 0; --i) {
    const long long d = g[i].dim;
    const long long s = which == 0 ? g[i].sa : (which == 1 ? g[i].sb : g[i].sc);
    total *= d;
    if (d == 1) continue;
    if (!comps.empty() && comps.back().stride * comps.back().size == s) {
      comps.back().size *= d;
    } else {
      comps.push_back({d, s});
    }
  }
  if (comps.empty()) { out = idx1(0); return true; }
  if (comps.size() == 1) { out = idx1(comps[0].stride); return true; }
  if (comps.size() == 2) {
    if (comps[0].size > 0x7fffffffLL) return false;
    out = idx2((int)comps[0].size, comps[1].stride, comps[0].stride);
    return true;
  }
  return false;
}

// Find an order of group g valid for the tensors in `need` (bitmask of
// which), trying all permutations (groups have at most 6 labels).
bool choose_order(std::vector<Lab>& g, int need) {
  std::vector<int> idx(g.size());
  for (size_t i = 0; i < g.size(); ++i) idx[i] = (int)i;
  std::vector<Lab> orig = g;
  // start from the order of decreasing stride in the first needed tensor
  do {
    std::vector<Lab> cand(g.size());
    for (size_t i = 0; i < g.size(); ++i) cand[i] = orig[idx[i]];
    bool ok = true;
    for (int w = 0; w < 3 && ok; ++w) {
      if (!(need & (1 << w))) continue;
      Idx2 d;
      long long t;
      ok = collapse(cand, w, d, t);
    }
    if (ok) { g = cand; return true; }
  } while (std::next_permutation(idx.begin(), idx.end()));
  return false;
}

void set_contiguous_strides(std::vector<Lab>& outer, std::vector<Lab>& inner, int which) {
  long long s = 1;
  for (int i = (int)inner.size() - 1; i >= 0; --i) {
    (which == 0 ? inner[i].sa : which == 1 ? inner[i].sb : inner[i].sc) = s;
    s *= inner[i].dim;
  }
  for (int i = (int)outer.size() - 1; i >= 0; --i) {
    (which == 0 ? outer[i].sa : which == 1 ? outer[i].sb : outer[i].sc) = s;
    s *= outer[i].dim;
  }
}

}  // namespace

Status accumulate(hipStream_t s, double alpha, const DT& X, const char* lx, double beta, const DT& Y, const char* ly) {
  Status st;
  const int nd = Y.nd;
  if ((int)std::strlen(lx) != X.nd || (int)std::strlen(ly) != nd || X.nd != nd || nd > 6) {
    st.msg = std::string("accumulate: label/rank mismatch ") + lx + " -> " + ly;
    return st;
  }
  PermArgs p{};
  p.nd = nd;
  p.alpha = alpha;
  p.beta = beta;
  for (int d = 0; d < nd; ++d) {
    const int k = find(lx, ly[d]);
    if (k < 0 || X.dim[k] != Y.dim[d]) {
      st.msg = std::string("accumulate: labels ") + lx + " vs " + ly;
      return st;
    }
    p.dim[d] = Y.dim[d];
    p.sy[d] = Y.st[d];
    p.sx[d] = X.st[k];
  }
  st.err = permute_add(X.p, Y.p, p, s);
  return st;
}

Status contract(Arena& ws, hipStream_t s, Prec prec, double alpha, const DT& A, const char* la, const DT& B,
                const char* lb, double beta, const DT& C, const char* lc) {
  Status st;
  if ((int)std::strlen(la) != A.nd || (int)std::strlen(lb) != B.nd || (int)std::strlen(lc) != C.nd) {
    st.msg = std::string("contract: rank mismatch ") + la + "," + lb + "->" + lc;
    return st;
  }
  std::vector<Lab> M, N, K;
  auto dim_of = [&](char c) -> long long {
    int k;
    if ((k = find(la, c)) >= 0) return A.dim[k];
    if ((k = find(lb, c)) >= 0) return B.dim[k];
    return C.dim[find(lc, c)];
  };
  std::string all = std::string(la) + lb + lc;
  std::string seen;
  for (char c : all) {
    if (seen.find(c) != std::string::npos) continue;
    seen.push_back(c);
    const int ia = find(la, c), ib = find(lb, c), ic = find(lc, c);
    Lab L{c, dim_of(c), ia >= 0 ? A.st[ia] : 0, ib >= 0 ? B.st[ib] : 0, ic >= 0 ? C.st[ic] : 0};
    if ((ia >= 0 && A.dim[ia] != L.dim) || (ib >= 0 && B.dim[ib] != L.dim) || (ic >= 0 && C.dim[ic] != L.dim)) {
      st.msg = std::string("contract: dimension mismatch for label ") + c;
      return st;
    }
    const int cnt = (ia >= 0) + (ib >= 0) + (ic >= 0);
    if (cnt != 2) {
      st.msg = std::string("contract: unsupported label ") + c + " in " + la + "," + lb + "->" + lc;
      return st;
    }
    if (ia >= 0 && ic >= 0) M.push_back(L);
    else if (ib >= 0 && ic >= 0) N.push_back(L);
    else K.push_back(L);
  }
  // group orders in the output's order for M and N, A's order for K
  auto by = [](const char* l) {
    return [l](const Lab& x, const Lab& y) { return find(l, x.c) < find(l, y.c); };
  };
  std::sort(M.begin(), M.end(), by(lc));
  std::sort(N.begin(), N.end(), by(lc));
  std::sort(K.begin(), K.end(), by(la));

  bool copyA = false, copyB = false, tempC = false;
  if (!choose_order(M, 1 | 4)) {
    if (choose_order(M, 4)) copyA = true;
    else if (choose_order(M, 1)) tempC = true;
    else { copyA = true; tempC = true; }
  }
  if (!choose_order(N, 2 | 4)) {
    if (choose_order(N, 4)) copyB = true;
    else if (choose_order(N, 2)) tempC = true;
    else { copyB = true; tempC = true; }
  }
  if (!choose_order(K, 1 | 2)) {
    if (!copyB && choose_order(K, 2)) copyA = true;
    else if (!copyA && choose_order(K, 1)) copyB = true;
    else { copyA = true; copyB = true; }
  }
  // still-invalid single-tensor groups force copies
  {
    Idx2 d;
    long long t;
    if (!copyA && (!collapse(M, 0, d, t) || !collapse(K, 0, d, t))) copyA = true;
    if (!copyB && (!collapse(K, 1, d, t) || !collapse(N, 1, d, t))) copyB = true;
    if (!tempC && (!collapse(M, 2, d, t) || !collapse(N, 2, d, t))) tempC = true;
  }
  long long m_tot = 1, n_tot = 1, k_tot = 1;
  for (auto& l : M) m_tot *= l.dim;
  for (auto& l : N) n_tot *= l.dim;
  for (auto& l : K) k_tot *= l.dim;
  if (m_tot > 0x7fffffffLL || n_tot > 0x7fffffffLL || k_tot > 0x7fffffffLL) {
    st.msg = "contract: dimension exceeds 2^31";
    return st;
  }
  const size_t mark = ws.mark();
  const double* Ap = A.p;
  const double* Bp = B.p;
  double* Cp = C.p;
  // copies into contiguous scratch: A as [M][K], B as [K][N], C as [M][N]
  if (copyA) {
    double* t = ws.alloc((size_t)(m_tot * k_tot));
    if (!t) { st.msg = "contract: scratch exhausted (A copy)"; return st; }
    std::vector<Lab> m2 = M, k2 = K;
    set_contiguous_strides(m2, k2, 0);
    PermArgs p{};
    p.nd = 0;
    p.alpha = 1.0;
    p.beta = 0.0;
    auto add = [&](const Lab& orig, const Lab& now) {
      p.dim[p.nd] = orig.dim;
      p.sx[p.nd] = orig.sa;
      p.sy[p.nd] = now.sa;
      ++p.nd;
    };
    for (size_t i = 0; i < M.size(); ++i) add(M[i], m2[i]);
    for (size_t i = 0; i < K.size(); ++i) add(K[i], k2[i]);
    if (p.nd > 6) { st.msg = "contract: rank > 6"; ws.reset(mark); return st; }
    st.err = permute_add(A.p, t, p, s);
    if (st.err != hipSuccess) { ws.reset(mark); return st; }
    M = m2; K = k2;
    Ap = t;
  }
  if (copyB) {
    double* t = ws.alloc((size_t)(k_tot * n_tot));
    if (!t) { st.msg = "contract: scratch exhausted (B copy)"; ws.reset(mark); return st; }
    std::vector<Lab> k2 = K, n2 = N;
    set_contiguous_strides(k2, n2, 1);
    PermArgs p{};
    p.alpha = 1.0;
    p.beta = 0.0;
    auto add = [&](const Lab& orig, const Lab& now) {
      p.dim[p.nd] = orig.dim;
      p.sx[p.nd] = orig.sb;
      p.sy[p.nd] = now.sb;
      ++p.nd;
    };
    for (size_t i = 0; i < K.size(); ++i) add(K[i], k2[i]);
    for (size_t i = 0; i < N.size(); ++i) add(N[i], n2[i]);
    if (p.nd > 6) { st.msg = "contract: rank > 6"; ws.reset(mark); return st; }
    st.err = permute_add(B.p, t, p, s);
    if (st.err != hipSuccess) { ws.reset(mark); return st; }
    K = k2; N = n2;
    Bp = t;
  }
  std::vector<Lab> Corig_m = M, Corig_n = N;
  if (tempC) {
    double* t = ws.alloc((size_t)(m_tot * n_tot));
    if (!t) { st.msg = "contract: scratch exhausted (C temp)"; ws.reset(mark); return st; }
    set_contiguous_strides(M, N, 2);
    Cp = t;
  }
  GemmArgs g{};
  g.M = (int)m_tot;
  g.N = (int)n_tot;
  g.K = (int)k_tot;
  g.batch = 1;
  g.A = Ap;
  g.B = Bp;
  g.C = Cp;
  long long t;
  bool ok = collapse(M, 0, g.am, t) && collapse(K, 0, g.ak, t) && collapse(K, 1, g.bk, t) &&
            collapse(N, 1, g.bn, t) && collapse(M, 2, g.cm, t) && collapse(N, 2, g.cn, t);
  if (!ok) { st.msg = "contract: planner failed to map index groups"; ws.reset(mark); return st; }
  auto extent = [](const DT& t) {
    long long e = 1;
    for (int i = 0; i < t.nd; ++i) e += (t.dim[i] - 1) * t.st[i];
    return e;
  };
  g.a_len = copyA ? m_tot * k_tot : extent(A);
  g.b_len = copyB ? k_tot * n_tot : extent(B);
  g.c_len = tempC ? m_tot * n_tot : extent(C);
  g.alpha = alpha;
  g.beta = tempC ? 0.0 : beta;
  if (k_tot == 0) {
    g.K = 0;
  }
  // scratch for a split-K launch: what is left of the arena, up to 64 M doubles
  const size_t split_mark = ws.mark();
  const size_t avail = ws.available() / sizeof(double);
  const long long cap = (long long)std::min<size_t>(avail > 4096 ? avail - 4096 : 0, (size_t)1 << 26);
  if (cap > 0) {
    g.split_ws = ws.alloc((size_t)cap);
    g.split_cap = g.split_ws ? cap : 0;
  }
  st.err = gemm(g, prec, s);
  ws.reset(split_mark);
  if (st.err != hipSuccess) { ws.reset(mark); return st; }
  if (tempC) {
    PermArgs p{};
    p.alpha = 1.0;
    p.beta = beta;
    auto add = [&](const Lab& tmp, const Lab& orig) {
      p.dim[p.nd] = orig.dim;
      p.sx[p.nd] = tmp.sc;
      p.sy[p.nd] = orig.sc;
      ++p.nd;
    };
    for (size_t i = 0; i < M.size(); ++i) add(M[i], Corig_m[i]);
    for (size_t i = 0; i < N.size(); ++i) add(N[i], Corig_n[i]);
    if (p.nd > 6) { st.msg = "contract: rank > 6"; ws.reset(mark); return st; }
    st.err = permute_add(Cp, C.p, p, s);
  }
  ws.reset(mark);
  return st;
}

}  // namespace cct
