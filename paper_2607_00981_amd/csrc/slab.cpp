// libcct slab runtime: the triples residual terms that need only the locally
// stored T3 blocks, for a contiguous range of packed triples.
//
// In a run sharded by packed triples (paper, Sec. "Parallel implementation":
// each process owns a range of i<=j<=k blocks, with T1, T2 and the
// intermediates replicated) these terms need no communication: the
// particle-particle ladder, the F_vv part of the Fock term and the two T2*W
// drivers (Eq. resi-rccsdt).  The ladder's W^{ab}_{de} is never stored whole
// (v^4 doubles is 205 GB at v = 400): it is rebuilt panel by panel from the
// T1-dressed density-fitting factors,
//   W^{ab}_{de} = sum_P B~^P_{ad} B~^P_{be} + sum_lm v~^{lm}_{de} t_lm^ab,
// for a range of rows a at a time, and every panel is contracted with all
// stored blocks of the slab before the next one is built.
#include "../../include/cct.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

using namespace cct;

struct cct_slab {
  cct_alloc_fn alloc_fn = nullptr;  // the caller's device allocator (both null: hipMalloc / hipFree)
  cct_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  int o = 0, v = 0, n = 0, naux = 0, first = 0, count = 0, ntri_all = 0;
  Prec prec = Prec::F64;
  hipStream_t s = nullptr;
  int panel = 0;  // rows a per W panel
  bool have_ims = false, have_t3 = false, timers = false;
  long long v3 = 0;
  // device buffers
  double* BvvT = nullptr;  // [a][d][P] = B~^P_{v_a v_d}
  double* t2T = nullptr;   // [a][b][(l,m)] = t_lm^ab
  double* VoT = nullptr;   // [(d,e)][(l,m)] = v~^{lm}_{de}
  double* t2 = nullptr;    // [i][j][a][b]
  double* Fvv = nullptr;   // [a][d]
  double* Wt = nullptr;    // [j][a][b][d] = W^{ab}_{dj}
  double* Wvooo = nullptr; // [a][l][i][j] = W^{al}_{ij}
  double* t3 = nullptr;    // [count][v^3]
  double* r3 = nullptr;    // [count][v^3]
  void* views = nullptr;   // relabelled copies of the slab's T3 (see slab_pp)
  void* BvvL = nullptr;    // mixed modes: BvvT, t2T, VoT in the working precision with
  void* t2L = nullptr;     // their K (naux, o^2) padded with zeros to the vector width
  void* VoL = nullptr;     // (ka, ko elements per row), the operands of the panel rebuild
  long long ka = 0, ko = 0;
  double* Wp = nullptr;    // FP64 panel [panel][v][v][v]
  void* Wl = nullptr;      // low-precision panel
  double* eps0 = nullptr;  // zeros (no Jacobi step here)
  int4* tri = nullptr;     // the slab's (i,j,k,multiplicity)
  double* red = nullptr;
  long long red_n = 0;
  std::vector<int4> tri_h;
  std::vector<void*> owned;
  hipEvent_t ev[7] = {};
  double macs[5] = {0, 0, 0, 0, 0};  // ladder, W rebuild, F_vv, drivers (W^{ab}_{dj}), drivers (W^{al}_{ij})
  double ms[6] = {0, 0, 0, 0, 0, 0}; // views, rebuild, ladder, F_vv, drivers, post
  std::string err;
};

namespace {

#define SHIP(expr)                                                         \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      sl->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return e_ == hipErrorInvalidValue ? CCT_EINVAL : CCT_EDEVICE;        \
    }                                                                      \
  } while (0)

#define RCK_(expr)                 \
  do {                             \
    const int r_ = (expr);         \
    if (r_ != CCT_OK) return r_;   \
  } while (0)

// Device memory from the caller's allocator when one was given, else hipMalloc.
int sdev_alloc(cct_slab* sl, void** p, size_t bytes) {
  void* q = nullptr;
  bytes = std::max<size_t>(bytes, 8);
  if (sl->alloc_fn) {
    q = sl->alloc_fn(bytes, sl->alloc_user);
    if (!q || ((uintptr_t)q & 255)) {
      if (q) sl->free_fn(q, sl->alloc_user);
      sl->err = "caller allocator: " + std::string(q ? "pointer not 256-byte aligned" : "NULL") + " for " +
                std::to_string(bytes) + " bytes";
      return CCT_ENOMEM;
    }
  } else if (hipMalloc(&q, bytes) != hipSuccess) {
    sl->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    return CCT_ENOMEM;
  }
  *p = q;
  return CCT_OK;
}
void sdev_free(cct_slab* sl, void* p) {
  if (!p) return;
  if (sl->free_fn) sl->free_fn(p, sl->alloc_user);
  else (void)hipFree(p);
}

int salloc(cct_slab* sl, void** p, size_t bytes) {
  void* q = nullptr;
  const int rc = sdev_alloc(sl, &q, bytes);
  if (rc != CCT_OK) return rc;
  sl->owned.push_back(q);
  *p = q;
  return CCT_OK;
}

template <typename T>
int sallocd(cct_slab* sl, T** p, long long n) {
  void* q = nullptr;
  const int rc = salloc(sl, &q, (size_t)n * sizeof(T));
  *p = (T*)q;
  return rc;
}

bool opt_find(const std::string& js, const std::string& key, std::string& val) {
  const std::string pat = "\"" + key + "\"";
  size_t p = js.find(pat);
  if (p == std::string::npos) return false;
  p = js.find(':', p + pat.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < js.size() && (js[p] == ' ' || js[p] == '\t' || js[p] == '"')) ++p;
  size_t q = p;
  while (q < js.size() && js[q] != ',' && js[q] != '}' && js[q] != ' ' && js[q] != '"') ++q;
  val = js.substr(p, q - p);
  return true;
}

void mark(cct_slab* sl, int i) {
  if (sl->timers) (void)hipEventRecord(sl->ev[i], sl->s);
}

bool lp_ok(const cct_slab* sl) { return sl->prec != Prec::F64; }
bool nt_ok(const cct_slab* sl) { return sl->prec == Prec::F64 && ((long long)sl->v * sl->v) % 2 == 0; }

// The ladder's three relabelled terms, each a GEMM C[(t,x)][(y,z)] with K = (d,e):
//   term 2 reads T[t][x][(d,e)] (stored order) and writes R[t][x][y][z]  (W^{bc}_{de} t^{ade});
//   term 1 reads T[t][d][x][e] swapped to [t][x][(d,e)], writes R[t][y][x][z]  (W^{ac}_{de} t^{dbe});
//   term 0 reads T[t][(d,e)][x] rotated to [t][x][(d,e)], writes R[t][y][z][x]  (W^{ab}_{de} t^{dec}).
void ladder_maps(int v, Idx2 cm[3], Idx2 cn[3]) {
  const long long v2 = (long long)v * v, v3 = v2 * v;
  cm[0] = idx2(v, v3, 1);
  cm[1] = idx2(v, v3, v);
  cm[2] = idx2(v, v3, v2);
  cn[0] = idx1(v);
  cn[1] = idx2(v, v2, 1);
  cn[2] = idx1(1);
}

// Format of the ladder operands (views and W panel) in the mixed modes: FP32,
// or split BF16 interleaved by blocks of 32 when the rows (v^2 values) hold
// whole blocks, else as two planes.
int ladder_fmt(const cct_slab* sl) {
  const long long v2 = (long long)sl->v * sl->v;
  return sl->prec == Prec::F32 ? OUT_F32 : (v2 % 32 == 0 ? OUT_BF16X2I : OUT_BF16X2);
}

// Relabelled copies of the slab's T3: views[term] = [t][x][(d,e)] with x the
// free axis of that term, in the working precision (FP64 terms 0 and 1 only;
// term 2 reads T3 itself in FP64).
int build_views(cct_slab* sl) {
  const int v = sl->v;
  const long long v2 = (long long)v * v, v3 = sl->v3, nb = sl->count;
  if (lp_ok(sl)) {
    const int fmt = ladder_fmt(sl);
    char* base = (char*)sl->views;
    for (int term = 0; term < 3; ++term) {
      void* dst = base + (size_t)term * nb * v3 * 4;
      const OutSpec os{dst, fmt, nb * v3};
      if (term == 2) SHIP(convert(sl->t3, os, nb * v3, sl->s));
      else if (term == 1) SHIP(swap01_batched(sl->t3, os, nb, v, v, v, sl->s));
      else SHIP(transpose_batched(sl->t3, os, nb, (int)v2, v, sl->s));
    }
  } else if (nt_ok(sl)) {
    double* base = (double*)sl->views;
    SHIP(transpose_batched(sl->t3, OutSpec{base, OUT_F64, 0}, nb, (int)v2, v, sl->s));
    SHIP(swap01_batched(sl->t3, OutSpec{base + nb * v3, OUT_F64, 0}, nb, v, v, v, sl->s));
  }
  return CCT_OK;
}

// W panel for rows a in [a0, a0 + na): Wp[a - a0][b][d][e] (FP64).
int build_panel(cct_slab* sl, int a0, int na) {
  const int o = sl->o, v = sl->v, naux = sl->naux;
  const long long v2 = (long long)v * v, v3 = sl->v3, o2 = (long long)o * o;
  if (lp_ok(sl)) {
    // mixed modes: the panel is an operand of the low-precision ladder, so it
    // is rebuilt from operands in the same precision (FP64 output, converted
    // with the panel afterwards)
    const size_t esz = sl->prec == Prec::F32 ? 4 : 2;  // bytes per element of one operand plane
    const long long ka = sl->ka, ko = sl->ko;
    NtLpArgs g{};
    g.M = v; g.N = (int)v2; g.K = (int)ka; g.batch = na;
    g.A = (const char*)sl->BvvL + (size_t)((long long)a0 * v * ka) * esz; g.lda = ka; g.a_batch = (long long)v * ka;
    g.a_plane = v2 * ka;
    g.B = sl->BvvL; g.ldb = ka; g.b_batch = 0; g.b_plane = v2 * ka;
    g.C = sl->Wp; g.cm = idx1(v); g.cn = idx2(v, v2, 1); g.c_batch = v3;
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = (v2 - (long long)a0 * v) * ka; g.b_len = v2 * ka; g.c_len = (long long)na * v3;
    SHIP(gemm_nt_lp(g, sl->prec, sl->s));
    NtLpArgs h{};
    h.M = (int)((long long)na * v); h.N = (int)v2; h.K = (int)ko; h.batch = 1;
    h.A = (const char*)sl->t2L + (size_t)((long long)a0 * v * ko) * esz; h.lda = ko; h.a_plane = v2 * ko;
    h.B = sl->VoL; h.ldb = ko; h.b_plane = v2 * ko;
    h.C = sl->Wp; h.cm = idx1(v2); h.cn = idx1(1);
    h.alpha = 1.0; h.beta = 1.0;
    h.a_len = (v2 - (long long)a0 * v) * ko; h.b_len = v2 * ko; h.c_len = (long long)na * v3;
    SHIP(gemm_nt_lp(h, sl->prec, sl->s));
    return CCT_OK;
  }
  // sum_P B~_{ad} B~_{be}: per a, C[d][(b,e)] = sum_P BvvT[a][d][P] BvvT[(b,e)][P]
  if (naux % 2 == 0) {
    NtArgs g{};
    g.M = v; g.N = (int)v2; g.K = naux; g.batch = na;
    g.A = sl->BvvT + (long long)a0 * v * naux; g.lda = naux; g.a_batch = (long long)v * naux;
    g.B = sl->BvvT; g.ldb = naux; g.b_batch = 0;
    g.C = sl->Wp; g.cm = idx1(v); g.cn = idx2(v, v2, 1); g.c_batch = v3;
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = v2 * naux - (long long)a0 * v * naux; g.b_len = v2 * naux; g.c_len = (long long)na * v3;
    SHIP(gemm_nt(g, Prec::F64, sl->s));
  } else {
    GemmArgs g{};
    g.M = v; g.N = (int)v2; g.K = naux; g.batch = na;
    g.A = sl->BvvT + (long long)a0 * v * naux; g.am = idx1(naux); g.ak = idx1(1); g.a_batch = (long long)v * naux;
    g.B = sl->BvvT; g.bk = idx1(1); g.bn = idx1(naux); g.b_batch = 0;
    g.C = sl->Wp; g.cm = idx1(v); g.cn = idx2(v, v2, 1); g.c_batch = v3;
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = v2 * naux - (long long)a0 * v * naux; g.b_len = v2 * naux; g.c_len = (long long)na * v3;
    SHIP(gemm(g, Prec::F64, sl->s));
  }
  // + sum_lm t_lm^ab v~^{lm}_{de}: C[(a,b)][(d,e)] = sum_(l,m) t2T[(a,b)][(l,m)] VoT[(d,e)][(l,m)]
  if (o2 % 2 == 0) {
    NtArgs g{};
    g.M = (int)((long long)na * v); g.N = (int)v2; g.K = (int)o2; g.batch = 1;
    g.A = sl->t2T + (long long)a0 * v * o2; g.lda = o2;
    g.B = sl->VoT; g.ldb = o2;
    g.C = sl->Wp; g.cm = idx1(v2); g.cn = idx1(1);
    g.alpha = 1.0; g.beta = 1.0;
    g.a_len = v2 * o2 - (long long)a0 * v * o2; g.b_len = v2 * o2; g.c_len = (long long)na * v3;
    SHIP(gemm_nt(g, Prec::F64, sl->s));
  } else {
    GemmArgs g{};
    g.M = (int)((long long)na * v); g.N = (int)v2; g.K = (int)o2; g.batch = 1;
    g.A = sl->t2T + (long long)a0 * v * o2; g.am = idx1(o2); g.ak = idx1(1);
    g.B = sl->VoT; g.bk = idx1(1); g.bn = idx1(o2);
    g.C = sl->Wp; g.cm = idx1(v2); g.cn = idx1(1);
    g.alpha = 1.0; g.beta = 1.0;
    g.a_len = v2 * o2 - (long long)a0 * v * o2; g.b_len = v2 * o2; g.c_len = (long long)na * v3;
    SHIP(gemm(g, Prec::F64, sl->s));
  }
  return CCT_OK;
}

// Ladder over all panels: R[t] += sum_de W^{..}_{de} t^{..} (three relabelled terms).
int slab_pp(cct_slab* sl) {
  const int v = sl->v;
  const long long v2 = (long long)v * v, v3 = sl->v3, nb = sl->count;
  Idx2 cm[3], cn[3];
  ladder_maps(v, cm, cn);
  const bool lp = lp_ok(sl), nt = nt_ok(sl);
  mark(sl, 0);
  RCK_(build_views(sl));
  mark(sl, 1);
  float t_rebuild = 0.f, t_ladder = 0.f;
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  if (sl->timers) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventCreate(&e2);
  }
  for (int a0 = 0; a0 < v; a0 += sl->panel) {
    const int na = std::min(sl->panel, v - a0);
    const long long prow = (long long)na * v;  // W rows (a, b) of this panel
    if (sl->timers) (void)hipEventRecord(e0, sl->s);
    RCK_(build_panel(sl, a0, na));
    if (lp) SHIP(convert(sl->Wp, OutSpec{sl->Wl, ladder_fmt(sl), prow * v2}, prow * v2, sl->s));
    if (sl->timers) (void)hipEventRecord(e1, sl->s);
    for (int term = 0; term < 3; ++term) {
      // panel rows (y,z) = (a0 + r / v, r % v): offset of the output by a0 along y
      const long long coff = (cn[term].inner == 0 ? (long long)a0 * v * cn[term].s_lo : (long long)a0 * cn[term].s_hi);
      if (lp) {
        NtLpArgs g{};
        g.M = (int)(nb * v); g.N = (int)prow; g.K = (int)v2; g.batch = 1;
        g.A = (const char*)sl->views + (size_t)term * nb * v3 * 4; g.lda = v2; g.a_plane = nb * v3;
        g.B = sl->Wl; g.ldb = v2; g.b_plane = prow * v2;
        g.C = sl->r3 + coff; g.cm = cm[term]; g.cn = cn[term];
        g.alpha = 1.0; g.beta = 1.0;
        g.a_len = nb * v3; g.b_len = prow * v2; g.c_len = nb * v3 - coff;
        g.il = ladder_fmt(sl) == OUT_BF16X2I;
        SHIP(gemm_nt_lp(g, sl->prec, sl->s));
      } else if (nt) {
        NtArgs g{};
        g.M = (int)(nb * v); g.N = (int)prow; g.K = (int)v2; g.batch = 1;
        g.A = term == 2 ? sl->t3 : (const double*)sl->views + (term == 0 ? 0 : nb * v3); g.lda = v2;
        g.B = sl->Wp; g.ldb = v2;
        g.C = sl->r3 + coff; g.cm = cm[term]; g.cn = cn[term];
        g.alpha = 1.0; g.beta = 1.0;
        g.a_len = nb * v3; g.b_len = prow * v2; g.c_len = nb * v3 - coff;
        SHIP(gemm_nt(g, Prec::F64, sl->s));
      } else {
        // generic strided kernel reading the stored blocks in place
        const Idx2 am[3] = {idx2(v, v3, 1), idx2(v, v3, v), idx2(v, v3, v2)};
        const Idx2 ak[3] = {idx1(v), idx2(v, v2, 1), idx1(1)};
        GemmArgs g{};
        g.M = (int)(nb * v); g.N = (int)prow; g.K = (int)v2; g.batch = 1;
        g.A = sl->t3; g.am = am[term]; g.ak = ak[term];
        g.B = sl->Wp; g.bk = idx1(1); g.bn = idx1(v2);
        g.C = sl->r3 + coff; g.cm = cm[term]; g.cn = cn[term];
        g.alpha = 1.0; g.beta = 1.0;
        g.a_len = nb * v3; g.b_len = prow * v2; g.c_len = nb * v3 - coff;
        SHIP(gemm(g, Prec::F64, sl->s));
      }
    }
    if (sl->timers) {
      (void)hipEventRecord(e2, sl->s);
      (void)hipEventSynchronize(e2);
      float a = 0.f, b = 0.f;
      (void)hipEventElapsedTime(&a, e0, e1);
      (void)hipEventElapsedTime(&b, e1, e2);
      t_rebuild += a;
      t_ladder += b;
    }
  }
  if (sl->timers) {
    sl->ms[1] = t_rebuild;
    sl->ms[2] = t_ladder;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
  }
  return CCT_OK;
}

// F_vv part of the Fock term: sum_d F^a_d t^{dbc} + F^b_d t^{adc} + F^c_d t^{abd} per block.
int slab_f1(cct_slab* sl) {
  const int v = sl->v;
  const long long v2 = (long long)v * v, v3 = sl->v3;
  for (int start = 0; start < sl->count; start += 65535) {
    const int nb = std::min(65535, sl->count - start);
    const long long off = (long long)start * v3;
    for (int axis = 0; axis < 3; ++axis) {
      GemmArgs g{};
      g.M = v; g.K = v; g.N = (int)v2; g.batch = nb;
      g.A = sl->Fvv; g.am = idx1(v); g.ak = idx1(1); g.a_batch = 0;
      g.B = sl->t3 + off; g.b_batch = v3;
      g.C = sl->r3 + off; g.c_batch = v3;
      if (axis == 0) { g.bk = idx1(v2); g.bn = idx1(1); g.cm = idx1(v2); g.cn = idx1(1); }
      if (axis == 1) { g.bk = idx1(v); g.bn = idx2(v, v2, 1); g.cm = idx1(v); g.cn = idx2(v, v2, 1); }
      if (axis == 2) { g.bk = idx1(1); g.bn = idx1(v); g.cm = idx1(1); g.cn = idx1(v); }
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = v2; g.b_len = (long long)sl->count * v3 - off; g.c_len = (long long)sl->count * v3 - off;
      SHIP(gemm(g, Prec::F64, sl->s));
    }
  }
  return CCT_OK;
}

const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// T2 drivers for every stored block and every simultaneous column permutation
// sigma: with (p,q,r) = sigma(i,j,k) and (x,y,z) = sigma(a,b,c),
//   R[abc] += sum_d W^{xy}_{dq} t_{pr}^{dz} - sum_l W^{xl}_{pq} t_{lr}^{yz}.
int slab_drivers(cct_slab* sl, bool d1, bool d2) {
  const int o = sl->o, v = sl->v;
  const long long v2 = (long long)v * v, v3 = sl->v3, o2v2 = (long long)o * o * v2;
  const long long ax_stride[3] = {v2, (long long)v, 1};
  for (int t = 0; t < sl->count; ++t) {
    const int4 tr = sl->tri_h[t];
    const int occ[3] = {tr.x, tr.y, tr.z};
    double* R = sl->r3 + (long long)t * v3;
    for (int s = 0; s < 6; ++s) {
      const int* pi = PERM3[s];
      const int p = occ[pi[0]], q = occ[pi[1]], r = occ[pi[2]];
      // output axes: x lives on R's axis pi[0], y on pi[1], z on pi[2]
      const long long sx = ax_stride[pi[0]], sy = ax_stride[pi[1]], sz = ax_stride[pi[2]];
      if (d1) {
        // C[(x,y)][z] = sum_d Wt[q][x][y][d] t2[r][p][z][d]  (t_{pr}^{dz} = t_{rp}^{zd})
        const double* Bm = sl->t2 + ((long long)r * o + p) * v2;
        if (v % 2 == 0) {
          NtArgs g{};
          g.M = (int)v2; g.N = v; g.K = v; g.batch = 1;
          g.A = sl->Wt + (long long)q * v3; g.lda = v;
          g.B = Bm; g.ldb = v;
          g.C = R; g.cm = idx2(v, sx, sy); g.cn = idx1(sz);
          g.alpha = 1.0; g.beta = 1.0;
          g.a_len = v3; g.b_len = v2; g.c_len = v3;
          SHIP(gemm_nt(g, Prec::F64, sl->s));
        } else {
          GemmArgs g{};
          g.M = (int)v2; g.N = v; g.K = v; g.batch = 1;
          g.A = sl->Wt + (long long)q * v3; g.am = idx1(v); g.ak = idx1(1);
          g.B = Bm; g.bk = idx1(1); g.bn = idx1(v);
          g.C = R; g.cm = idx2(v, sx, sy); g.cn = idx1(sz);
          g.alpha = 1.0; g.beta = 1.0;
          g.a_len = v3; g.b_len = v2; g.c_len = v3;
          SHIP(gemm(g, Prec::F64, sl->s));
        }
      }
      if (d2) {
        // C[x][(y,z)] = -sum_l Wvooo[x][l][p][q] t2[l][r][y][z]
        GemmArgs g{};
        g.M = v; g.N = (int)v2; g.K = o; g.batch = 1;
        g.A = sl->Wvooo + ((long long)p * o + q); g.am = idx1((long long)o * o * o); g.ak = idx1((long long)o * o);
        g.B = sl->t2 + (long long)r * v2; g.bk = idx1((long long)o * v2); g.bn = idx1(1);
        g.C = R; g.cm = idx1(sx); g.cn = idx2(v, sy, sz);
        g.alpha = -1.0; g.beta = 1.0;
        g.a_len = (long long)v * o * o * o - ((long long)p * o + q); g.b_len = o2v2 - (long long)r * v2; g.c_len = v3;
        SHIP(gemm(g, Prec::F64, sl->s));
      }
    }
  }
  return CCT_OK;
}

}  // namespace

extern "C" {

void cct_slab_destroy(cct_slab* sl) {
  if (!sl) return;
  if (sl->s) (void)hipStreamSynchronize(sl->s);
  for (void* p : sl->owned) sdev_free(sl, p);
  for (hipEvent_t e : sl->ev)
    if (e) (void)hipEventDestroy(e);
  delete sl;
}

int cct_slab_create(int nocc, int nvir, int naux, int first, int count, cct_precision prec, const char* opts_json,
                    cct_alloc_fn alloc, cct_free_fn free_fn, void* alloc_user, void* hip_stream, cct_slab** out) {
  if (!out) return CCT_EINVAL;
  *out = nullptr;
  if (nocc < 1 || nvir < 1 || naux < 1 || nocc > 200 || nvir > 1200 || (int)prec < 0 || (int)prec > 2)
    return CCT_EINVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) return CCT_EINVAL;
  const long long ntri = (long long)nocc * (nocc + 1) * (nocc + 2) / 6;
  if (first < 0 || count < 1 || first + (long long)count > ntri || count > 65535) return CCT_EINVAL;
  cct_slab* sl = new cct_slab();
  sl->alloc_fn = alloc;
  sl->free_fn = free_fn;
  sl->alloc_user = alloc_user;
  sl->o = nocc; sl->v = nvir; sl->n = nocc + nvir; sl->naux = naux;
  sl->first = first; sl->count = count; sl->ntri_all = (int)ntri;
  sl->prec = (Prec)prec;
  sl->s = (hipStream_t)hip_stream;
  sl->v3 = (long long)nvir * nvir * nvir;
  sl->panel = std::max(1, std::min(nvir, 8));
  if (opts_json) {
    std::string js(opts_json), val;
    if (opt_find(js, "panel", val)) sl->panel = std::atoi(val.c_str());
    if (opt_find(js, "timers", val)) sl->timers = (val == "true" || val == "1");
  }
  if (sl->panel < 1 || sl->panel > nvir) { delete sl; return CCT_EINVAL; }
  const int o = nocc, v = nvir, n = sl->n;
  const long long v2 = (long long)v * v, v3 = sl->v3, o2 = (long long)o * o, nb = count;
  // packed triples of the slab, in the lexicographic i<=j<=k order
  {
    long long idx = 0;
    for (int i = 0; i < o; ++i)
      for (int j = i; j < o; ++j)
        for (int k = j; k < o; ++k, ++idx)
          if (idx >= first && idx < first + count) {
            const int mult = (i == j && j == k) ? 1 : ((i == j || j == k) ? 3 : 6);
            sl->tri_h.push_back(int4{i, j, k, mult});
          }
  }
  int rc = CCT_OK;
  const bool lp = lp_ok(sl), nt = nt_ok(sl);
  const size_t view_bytes = lp ? (size_t)3 * nb * v3 * 4 : (nt ? (size_t)2 * nb * v3 * 8 : 8);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->BvvT, v2 * naux);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->t2T, v2 * o2);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->VoT, v2 * o2);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->t2, o2 * v2);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->Fvv, v2);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->Wt, (long long)o * v3);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->Wvooo, (long long)v * o * o2);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->t3, nb * v3);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->r3, nb * v3);
  if (rc == CCT_OK) rc = salloc(sl, &sl->views, view_bytes);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->Wp, (long long)sl->panel * v3);
  if (lp) {
    const int w = sl->prec == Prec::F32 ? 4 : 8;
    sl->ka = ((long long)naux + w - 1) / w * w;
    sl->ko = (o2 + w - 1) / w * w;
    if (rc == CCT_OK) rc = salloc(sl, &sl->BvvL, (size_t)(v2 * sl->ka) * 4);
    if (rc == CCT_OK) rc = salloc(sl, &sl->t2L, (size_t)(v2 * sl->ko) * 4);
    if (rc == CCT_OK) rc = salloc(sl, &sl->VoL, (size_t)(v2 * sl->ko) * 4);
  }
  if (rc == CCT_OK && lp) rc = salloc(sl, &sl->Wl, (size_t)sl->panel * v3 * 4);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->eps0, n);
  if (rc == CCT_OK) rc = sallocd(sl, &sl->tri, nb);
  sl->red_n = 2048 + 64LL * nb;
  if (rc == CCT_OK) rc = sallocd(sl, &sl->red, sl->red_n);
  if (rc == CCT_OK && hipMemcpy(sl->tri, sl->tri_h.data(), sizeof(int4) * nb, hipMemcpyHostToDevice) != hipSuccess)
    rc = CCT_EDEVICE;
  if (rc == CCT_OK && fill(sl->eps0, 0.0, n, sl->s) != hipSuccess) rc = CCT_EDEVICE;
  if (rc == CCT_OK && sl->timers)
    for (int i = 0; i < 7 && rc == CCT_OK; ++i)
      if (hipEventCreate(&sl->ev[i]) != hipSuccess) rc = CCT_EDEVICE;
  if (rc == CCT_OK && hipStreamSynchronize(sl->s) != hipSuccess) rc = CCT_EDEVICE;
  if (rc != CCT_OK) {
    cct_slab_destroy(sl);
    return rc;
  }
  *out = sl;
  return CCT_OK;
}

int cct_slab_set_intermediates(cct_slab* sl, const double* Bt, const double* t2, const double* Fvv,
                               const double* Wt, const double* Wvooo) {
  if (!sl || !Bt || !t2 || !Fvv || !Wt || !Wvooo) return CCT_EINVAL;
  const int o = sl->o, v = sl->v, n = sl->n, naux = sl->naux;
  const long long v2 = (long long)v * v, o2 = (long long)o * o, n2 = (long long)n * n;
  // host-side relayouts of the small replicated inputs
  std::vector<double> bvv((size_t)(v2 * naux)), tt((size_t)(v2 * o2));
  for (int a = 0; a < v; ++a)
    for (int d = 0; d < v; ++d)
      for (int P = 0; P < naux; ++P)
        bvv[((size_t)a * v + d) * naux + P] = Bt[(size_t)P * n2 + (size_t)(o + a) * n + (o + d)];
  for (int l = 0; l < o; ++l)
    for (int m = 0; m < o; ++m)
      for (int a = 0; a < v; ++a)
        for (int b = 0; b < v; ++b)
          tt[((size_t)a * v + b) * o2 + (size_t)l * o + m] = t2[(((size_t)l * o + m) * v + a) * v + b];
  SHIP(hipMemcpy(sl->BvvT, bvv.data(), bvv.size() * 8, hipMemcpyHostToDevice));
  SHIP(hipMemcpy(sl->t2T, tt.data(), tt.size() * 8, hipMemcpyHostToDevice));
  SHIP(hipMemcpy(sl->t2, t2, (size_t)(o2 * v2) * 8, hipMemcpyHostToDevice));
  SHIP(hipMemcpy(sl->Fvv, Fvv, (size_t)v2 * 8, hipMemcpyHostToDevice));
  SHIP(hipMemcpy(sl->Wt, Wt, (size_t)o * v2 * v * 8, hipMemcpyHostToDevice));
  SHIP(hipMemcpy(sl->Wvooo, Wvooo, (size_t)v * o * o2 * 8, hipMemcpyHostToDevice));
  // v~^{lm}_{de} = sum_P B~^P_{ld} B~^P_{me} as VoT[(d,e)][(l,m)]: host copy of the
  // occupied-virtual factors, one GEMM on the device
  std::vector<double> bov((size_t)naux * o * v);
  for (int P = 0; P < naux; ++P)
    for (int l = 0; l < o; ++l)
      for (int d = 0; d < v; ++d) bov[((size_t)P * o + l) * v + d] = Bt[(size_t)P * n2 + (size_t)l * n + (o + d)];
  double* dbov = nullptr;
  RCK_(sdev_alloc(sl, (void**)&dbov, bov.size() * 8));
  hipError_t e = hipMemcpy(dbov, bov.data(), bov.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    // C[(d,e)][(l,m)] = sum_P bov[P][l][d] bov[P][m][e]: batch over d, M = e... written as
    // M = (d), N = (l, m, e) would need a 3-level map; instead batch over l:
    // C_l[d][(m,e)] = sum_P bov[P][l][d] bov[P][(m,e)], stored at VoT[d][e][l][m].
    GemmArgs g{};
    g.M = v; g.N = (int)((long long)o * v); g.K = naux; g.batch = o;
    g.A = dbov; g.am = idx1(1); g.ak = idx1((long long)o * v); g.a_batch = v;
    g.B = dbov; g.bk = idx1((long long)o * v); g.bn = idx2(v, v, 1); g.b_batch = 0;
    g.C = sl->VoT; g.cm = idx1((long long)v * o2); g.cn = idx2(v, 1, o2); g.c_batch = o;
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = (long long)naux * o * v; g.b_len = (long long)naux * o * v; g.c_len = v2 * o2;
    e = gemm(g, Prec::F64, sl->s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sl->s);
  sdev_free(sl, dbov);
  if (e != hipSuccess) {
    sl->err = std::string("v~^{lm}_{de} build: ") + hipGetErrorString(e);
    return CCT_EDEVICE;
  }
  if (lp_ok(sl)) {
    const int fmt = sl->prec == Prec::F32 ? OUT_F32 : OUT_BF16X2;
    SHIP(copy_pad_rows(sl->BvvT, v2, naux, OutSpec{sl->BvvL, fmt, v2 * sl->ka}, sl->ka, sl->s));
    SHIP(copy_pad_rows(sl->t2T, v2, o2, OutSpec{sl->t2L, fmt, v2 * sl->ko}, sl->ko, sl->s));
    SHIP(copy_pad_rows(sl->VoT, v2, o2, OutSpec{sl->VoL, fmt, v2 * sl->ko}, sl->ko, sl->s));
    SHIP(hipStreamSynchronize(sl->s));
  }
  sl->have_ims = true;
  return CCT_OK;
}

int cct_slab_set_t3(cct_slab* sl, const double* t3slab) {
  if (!sl || !t3slab) return CCT_EINVAL;
  SHIP(hipMemcpy(sl->t3, t3slab, (size_t)sl->count * sl->v3 * 8, hipMemcpyHostToDevice));
  sl->have_t3 = true;
  return CCT_OK;
}

int cct_slab_residual(cct_slab* sl, unsigned term_mask, double* r3slab, double* norm2) {
  if (!sl) return CCT_EINVAL;
  const unsigned allowed = CCT_TERM_PP | CCT_TERM_F1 | CCT_TERM_D1 | CCT_TERM_D2;
  if (term_mask & ~allowed) {
    sl->err = "slab terms are PP, F1, D1, D2 (the others need blocks of other ranges)";
    return CCT_EINVAL;
  }
  if (!sl->have_ims || !sl->have_t3) {
    sl->err = "intermediates and T3 slab must be set first";
    return CCT_ESTATE;
  }
  const long long v3 = sl->v3, nb = sl->count;
  for (double& m : sl->ms) m = 0.0;
  SHIP(fill(sl->r3, 0.0, nb * v3, sl->s));
  if (term_mask & CCT_TERM_PP) RCK_(slab_pp(sl));
  mark(sl, 2);
  if (term_mask & CCT_TERM_F1) RCK_(slab_f1(sl));
  mark(sl, 3);
  if (term_mask & (CCT_TERM_D1 | CCT_TERM_D2))
    RCK_(slab_drivers(sl, term_mask & CCT_TERM_D1, term_mask & CCT_TERM_D2));
  mark(sl, 4);
  PostArgs pa{sl->o, sl->v, (int)nb, v3, 0, 1};
  int np = 0;
  if (64LL * nb > sl->red_n - 1024) { sl->err = "reduction scratch too small"; return CCT_EDEVICE; }
  SHIP(post_update(sl->r3, sl->t3, sl->tri, sl->eps0, sl->red + 1024, &np, pa, sl->s));
  SHIP(reduce_sum(sl->red + 1024, np, sl->red + 1000, sl->red, sl->s));
  mark(sl, 5);
  double h = 0.0;
  SHIP(hipMemcpyAsync(&h, sl->red + 1000, sizeof(double), hipMemcpyDeviceToHost, sl->s));
  SHIP(hipStreamSynchronize(sl->s));
  if (sl->timers) {
    float x = 0.f;
    if ((term_mask & CCT_TERM_PP) && hipEventElapsedTime(&x, sl->ev[0], sl->ev[1]) == hipSuccess) sl->ms[0] = x;
    if (hipEventElapsedTime(&x, sl->ev[2], sl->ev[3]) == hipSuccess) sl->ms[3] = x;
    if (hipEventElapsedTime(&x, sl->ev[3], sl->ev[4]) == hipSuccess) sl->ms[4] = x;
    if (hipEventElapsedTime(&x, sl->ev[4], sl->ev[5]) == hipSuccess) sl->ms[5] = x;
  }
  const double v_ = sl->v, o_ = sl->o, nb_ = (double)nb;
  sl->macs[0] = (term_mask & CCT_TERM_PP) ? 3.0 * nb_ * std::pow(v_, 5) : 0.0;
  sl->macs[1] = (term_mask & CCT_TERM_PP) ? ((double)sl->naux + o_ * o_) * std::pow(v_, 4) : 0.0;
  sl->macs[2] = (term_mask & CCT_TERM_F1) ? 3.0 * nb_ * std::pow(v_, 4) : 0.0;
  sl->macs[3] = (term_mask & CCT_TERM_D1) ? 6.0 * nb_ * std::pow(v_, 4) : 0.0;
  sl->macs[4] = (term_mask & CCT_TERM_D2) ? 6.0 * nb_ * o_ * std::pow(v_, 3) : 0.0;
  if (!std::isfinite(h)) { sl->err = "non-finite residual norm"; return CCT_ENUMERIC; }
  if (norm2) *norm2 = h;
  if (r3slab) SHIP(hipMemcpy(r3slab, sl->r3, (size_t)(nb * v3) * 8, hipMemcpyDeviceToHost));
  return CCT_OK;
}

int cct_slab_copy_r3(cct_slab* sl, int64_t first, int64_t count, double* out) {
  if (!sl || !out || first < 0 || count < 0 || first + count > (int64_t)sl->count * sl->v3) return CCT_EINVAL;
  SHIP(hipMemcpy(out, sl->r3 + first, (size_t)count * 8, hipMemcpyDeviceToHost));
  return CCT_OK;
}

int cct_slab_get_counters(cct_slab* sl, double* macs, double* ms, int cap) {
  if (!sl || cap < 0) return CCT_EINVAL;
  for (int i = 0; i < std::min(cap, 6); ++i) {
    if (macs) macs[i] = i < 5 ? sl->macs[i] : 0.0;
    if (ms) ms[i] = sl->ms[i];
  }
  return CCT_OK;
}

const char* cct_slab_last_error(const cct_slab* sl) { return sl ? sl->err.c_str() : "null slab"; }

}  // extern "C"
