// libcct quadruples ladder: the particle-particle ladder of the RCCSDTQ
// quadruples residual on compactly stored T4.
//
// T4 is kept only for occupied quadruples i <= j <= k <= l (lexicographic
// order), each with its full v^4 virtual block [a][b][c][d].  The ladder term
// of Eq. resi-rccsdtq, P_(ia)(jb)(kc)(ld) [1/4 sum_ef W^{ab}_{ef} t_ijkl^efcd],
// restricted to a stored block is the sum of six terms (Sec. "RCCSDTQ
// contractions"), one per pair of virtual positions (p, q):
//   R[.. x at p .. y at q ..] += sum_ef W^{xy}_{ef} T[.. e at p .. f at q ..],
// every operand taken from the same stored block (the column symmetry carries
// the virtual labels with the occupied ones), exact also for repeated
// occupied indices.  Each term is one GEMM batched over the stored blocks with
// K = (e, f) = v^2: a relabelled copy of T4 puts the contracted pair last
// (K-contiguous rows), and the product is computed as C or as its transpose
// so that the writes into R4 run along R4's unit-stride axis.
#include "../../include/cct.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

using namespace cct;

struct cct_quad {
  cct_alloc_fn alloc_fn = nullptr;
  cct_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  int o = 0, v = 0;
  long long nq = 0, v4 = 0;
  Prec prec = Prec::F64;
  hipStream_t s = nullptr;
  bool timers = false, have_w = false, have_t4 = false, have_r = false;
  double* W = nullptr;   // [a][b][e][f] = W^{ab}_{ef}
  double* t4 = nullptr;  // [nq][v^4]
  double* r4 = nullptr;  // [nq][v^4]
  double* tc = nullptr;  // FP64 relabelled copy of T4 [nq][r1][r2][e][f]
  void* tl = nullptr;    // the same in the working precision (mixed modes)
  void* wl = nullptr;    // W in the working precision (mixed modes)
  int4* blk = nullptr;   // (i, j, k) and the multiplicity of each stored block (l is implied by order)
  double* red = nullptr;
  double* scal = nullptr;
  std::vector<void*> owned;
  hipEvent_t ev[3] = {};
  double macs = 0.0, ms[2] = {0.0, 0.0};  // relabelling, GEMMs
  std::string err;
};

namespace {

#define QHIP(expr)                                                         \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      q->err = std::string(#expr) + ": " + hipGetErrorString(e_);          \
      return e_ == hipErrorInvalidValue ? CCT_EINVAL : CCT_EDEVICE;        \
    }                                                                      \
  } while (0)

int qalloc(cct_quad* q, void** p, size_t bytes) {
  void* x = nullptr;
  bytes = std::max<size_t>(bytes, 8);
  if (q->alloc_fn) {
    x = q->alloc_fn(bytes, q->alloc_user);
    if (!x || ((uintptr_t)x & 255)) {
      if (x) q->free_fn(x, q->alloc_user);
      q->err = "caller allocator: " + std::string(x ? "pointer not 256-byte aligned" : "NULL");
      return CCT_ENOMEM;
    }
  } else if (hipMalloc(&x, bytes) != hipSuccess) {
    q->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    return CCT_ENOMEM;
  }
  q->owned.push_back(x);
  *p = x;
  return CCT_OK;
}

template <typename T>
int qallocd(cct_quad* q, T** p, long long n) {
  void* x = nullptr;
  const int rc = qalloc(q, &x, (size_t)n * sizeof(T));
  *p = (T*)x;
  return rc;
}

long long quad_count(int o) { return (long long)o * (o + 1) * (o + 2) * (o + 3) / 24; }

int multiplicity4(int i, int j, int k, int l) {
  // distinct orderings of (i, j, k, l): 4! / prod(run lengths!)
  const int a[4] = {i, j, k, l};
  int den = 1, run = 1;
  for (int x = 1; x <= 4; ++x) {
    if (x < 4 && a[x] == a[x - 1]) {
      ++run;
    } else {
      for (int y = 2; y <= run; ++y) den *= y;
      run = 1;
    }
  }
  return 24 / den;
}

// One term: contract virtual axes (p, q) of every stored block with W.
int ladder_term(cct_quad* q, int p, int qq) {
  const int v = q->v;
  const long long v2 = (long long)v * v, v4 = q->v4, nq = q->nq;
  const long long S[4] = {v2 * v, v2, v, 1};
  int r[2], nr = 0;
  for (int a = 0; a < 4; ++a)
    if (a != p && a != qq) r[nr++] = a;
  const bool lp = q->prec != Prec::F64;
  const bool f64_nt = !lp && (v2 % 2 == 0);
  const bool identity = (p == 2 && qq == 3);  // T4 already has the pair last
  // relabelled copy Tc[t][r1][r2][e][f] = T[t][e at p, f at q, r1, r2]
  const double* A64 = q->t4;
  if (!identity && (lp || f64_nt)) {
    PermArgs pa{};
    pa.nd = 5;
    const long long dim[5] = {nq, v, v, v, v};
    const long long sx[5] = {v4, S[r[0]], S[r[1]], S[p], S[qq]};
    const long long sy[5] = {v4, v2 * v, v2, v, 1};
    for (int d = 0; d < 5; ++d) {
      pa.dim[d] = dim[d];
      pa.sx[d] = sx[d];
      pa.sy[d] = sy[d];
    }
    pa.alpha = 1.0;
    pa.beta = 0.0;
    QHIP(permute_add(q->t4, q->tc, pa, q->s));
    A64 = q->tc;
  }
  if (lp) QHIP(convert(A64, OutSpec{q->tl, q->prec == Prec::F32 ? OUT_F32 : OUT_BF16X2, nq * v4}, nq * v4, q->s));
  if (q->timers) (void)hipEventRecord(q->ev[1], q->s);
  // writes along R4's unit-stride axis: with axis 3 in the contracted pair the
  // product is C[(r1,r2)][(x,y)] (y along axis 3), otherwise its transpose
  // C'[(x,y)][(r1,r2)] (r2 = axis 3)
  const bool plain = (qq == 3);
  const Idx2 m_rr = idx2(v, S[r[0]], S[r[1]]), m_pq = idx2(v, S[p], S[qq]);
  if (lp) {
    NtLpArgs g{};
    g.M = (int)v2; g.N = (int)v2; g.K = (int)v2; g.batch = (int)nq;
    if (plain) {
      g.A = q->tl; g.lda = v2; g.a_batch = v4; g.a_plane = nq * v4;
      g.B = q->wl; g.ldb = v2; g.b_batch = 0; g.b_plane = v4;
      g.cm = m_rr; g.cn = m_pq;
      g.a_len = nq * v4; g.b_len = v4;
    } else {
      g.A = q->wl; g.lda = v2; g.a_batch = 0; g.a_plane = v4;
      g.B = q->tl; g.ldb = v2; g.b_batch = v4; g.b_plane = nq * v4;
      g.cm = m_pq; g.cn = m_rr;
      g.a_len = v4; g.b_len = nq * v4;
    }
    g.C = q->r4; g.c_batch = v4; g.c_len = nq * v4;
    g.alpha = 1.0; g.beta = 1.0;
    QHIP(gemm_nt_lp(g, q->prec, q->s));
  } else if (f64_nt) {
    NtArgs g{};
    g.M = (int)v2; g.N = (int)v2; g.K = (int)v2; g.batch = (int)nq;
    if (plain) {
      g.A = A64; g.lda = v2; g.a_batch = v4;
      g.B = q->W; g.ldb = v2; g.b_batch = 0;
      g.cm = m_rr; g.cn = m_pq;
      g.a_len = nq * v4; g.b_len = v4;
    } else {
      g.A = q->W; g.lda = v2; g.a_batch = 0;
      g.B = A64; g.ldb = v2; g.b_batch = v4;
      g.cm = m_pq; g.cn = m_rr;
      g.a_len = v4; g.b_len = nq * v4;
    }
    g.C = q->r4; g.c_batch = v4; g.c_len = nq * v4;
    g.alpha = 1.0; g.beta = 1.0;
    QHIP(gemm_nt(g, Prec::F64, q->s));
  } else {
    // odd v^2 in FP64: the strided kernel reads the stored blocks in place
    GemmArgs g{};
    g.M = (int)v2; g.N = (int)v2; g.K = (int)v2; g.batch = (int)nq;
    g.A = q->t4; g.am = m_rr; g.ak = m_pq; g.a_batch = v4;
    g.B = q->W; g.bk = idx1(1); g.bn = idx1(v2); g.b_batch = 0;
    g.C = q->r4; g.cm = m_rr; g.cn = m_pq; g.c_batch = v4;
    g.alpha = 1.0; g.beta = 1.0;
    g.a_len = nq * v4; g.b_len = v4; g.c_len = nq * v4;
    QHIP(gemm(g, Prec::F64, q->s));
  }
  return CCT_OK;
}

}  // namespace

extern "C" {

int64_t cct_quad_count(int nocc) { return nocc < 0 ? -1 : (int64_t)quad_count(nocc); }

int64_t cct_quad_packed_index(int nocc, int i, int j, int k, int l) {
  if (nocc < 1 || i < 0 || i > j || j > k || k > l || l >= nocc) return -1;
  int64_t idx = 0;
  for (int a = 0; a < nocc; ++a)
    for (int b = a; b < nocc; ++b)
      for (int c = b; c < nocc; ++c)
        for (int d = c; d < nocc; ++d) {
          if (a == i && b == j && c == k && d == l) return idx;
          ++idx;
        }
  return -1;
}

void cct_quad_destroy(cct_quad* q) {
  if (!q) return;
  (void)hipStreamSynchronize(q->s);
  for (void* p : q->owned) {
    if (q->free_fn) q->free_fn(p, q->alloc_user);
    else (void)hipFree(p);
  }
  for (hipEvent_t e : q->ev)
    if (e) (void)hipEventDestroy(e);
  delete q;
}

int cct_quad_create(int nocc, int nvir, cct_precision prec, const char* opts_json, cct_alloc_fn alloc,
                    cct_free_fn free_fn, void* alloc_user, void* hip_stream, cct_quad** out) {
  if (!out) return CCT_EINVAL;
  *out = nullptr;
  if (nocc < 1 || nvir < 1 || (int)prec < 0 || (int)prec > 2) return CCT_EINVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) return CCT_EINVAL;
  const long long nq = quad_count(nocc), v2 = (long long)nvir * nvir;
  if (nq > 65535 || v2 > 46340 || v2 * v2 * nq > (1LL << 40)) return CCT_EINVAL;
  cct_quad* q = new cct_quad();
  q->alloc_fn = alloc;
  q->free_fn = free_fn;
  q->alloc_user = alloc_user;
  q->o = nocc;
  q->v = nvir;
  q->nq = nq;
  q->v4 = v2 * v2;
  q->prec = (Prec)prec;
  q->s = (hipStream_t)hip_stream;
  if (opts_json) {
    const std::string js(opts_json);
    q->timers = js.find("\"timers\": true") != std::string::npos || js.find("\"timers\":true") != std::string::npos;
  }
  const long long n4 = nq * q->v4;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete q;
    return CCT_EDEVICE;
  }
  const bool lp = q->prec != Prec::F64;
  const double need = 8.0 * (double)(q->v4 + 3 * n4) + (lp ? 4.0 * (double)(n4 + q->v4) : 0.0) + 64e6;
  if (!alloc && need > (double)free_b) {
    delete q;
    return CCT_ENOMEM;
  }
  int rc = CCT_OK;
  if (rc == CCT_OK) rc = qallocd(q, &q->W, q->v4);
  if (rc == CCT_OK) rc = qallocd(q, &q->t4, n4);
  if (rc == CCT_OK) rc = qallocd(q, &q->r4, n4);
  if (rc == CCT_OK) rc = qallocd(q, &q->tc, n4);
  if (rc == CCT_OK && lp) rc = qalloc(q, &q->tl, (size_t)n4 * 4);
  if (rc == CCT_OK && lp) rc = qalloc(q, &q->wl, (size_t)q->v4 * 4);
  if (rc == CCT_OK) rc = qallocd(q, &q->blk, nq);
  // reduction partials: at most 16 per stored block (weighted_dot_t3), then a fixed-order sum
  if (rc == CCT_OK) rc = qallocd(q, &q->red, 16 * nq + 1024);
  if (rc == CCT_OK) rc = qallocd(q, &q->scal, 8);
  if (rc == CCT_OK) {
    std::vector<int4> b;
    for (int i = 0; i < nocc; ++i)
      for (int j = i; j < nocc; ++j)
        for (int k = j; k < nocc; ++k)
          for (int l = k; l < nocc; ++l) b.push_back(int4{i, j, k, multiplicity4(i, j, k, l)});
    if (hipMemcpy(q->blk, b.data(), sizeof(int4) * b.size(), hipMemcpyHostToDevice) != hipSuccess) rc = CCT_EDEVICE;
  }
  for (int i = 0; i < 3 && rc == CCT_OK && q->timers; ++i)
    if (hipEventCreate(&q->ev[i]) != hipSuccess) rc = CCT_EDEVICE;
  if (rc != CCT_OK) {
    cct_quad_destroy(q);
    return rc;
  }
  *out = q;
  return CCT_OK;
}

int cct_quad_set(cct_quad* q, const double* W, const double* t4p) {
  if (!q || (!W && !t4p)) return CCT_EINVAL;
  if (W) {
    QHIP(hipMemcpyAsync(q->W, W, (size_t)q->v4 * 8, hipMemcpyHostToDevice, q->s));
    if (q->prec != Prec::F64)
      QHIP(convert(q->W, OutSpec{q->wl, q->prec == Prec::F32 ? OUT_F32 : OUT_BF16X2, q->v4}, q->v4, q->s));
    q->have_w = true;
  }
  if (t4p) {
    QHIP(hipMemcpyAsync(q->t4, t4p, (size_t)(q->nq * q->v4) * 8, hipMemcpyHostToDevice, q->s));
    q->have_t4 = true;
  }
  QHIP(hipStreamSynchronize(q->s));
  return CCT_OK;
}

int cct_quad_ladder(cct_quad* q, double* r4p, double* norm2) {
  if (!q) return CCT_EINVAL;
  if (!q->have_w || !q->have_t4) {
    q->err = "W and T4 not set (cct_quad_set)";
    return CCT_ESTATE;
  }
  QHIP(fill(q->r4, 0.0, q->nq * q->v4, q->s));
  float t_rel = 0.f, t_gemm = 0.f;
  const int pairs[6][2] = {{2, 3}, {0, 3}, {1, 3}, {0, 1}, {0, 2}, {1, 2}};
  for (const auto& pq : pairs) {
    if (q->timers) (void)hipEventRecord(q->ev[0], q->s);
    const int rc = ladder_term(q, pq[0], pq[1]);
    if (rc != CCT_OK) return rc;
    if (q->timers) {
      (void)hipEventRecord(q->ev[2], q->s);
      (void)hipEventSynchronize(q->ev[2]);
      float a = 0.f, b = 0.f;
      (void)hipEventElapsedTime(&a, q->ev[0], q->ev[1]);
      (void)hipEventElapsedTime(&b, q->ev[1], q->ev[2]);
      t_rel += a;
      t_gemm += b;
    }
  }
  q->macs = 6.0 * (double)q->nq * (double)q->v4 * (double)q->v * (double)q->v;  // 6 nq v^4 outputs x v^2
  q->ms[0] = t_rel;
  q->ms[1] = t_gemm;
  double h = 0.0;
  QHIP(weighted_dot_t3(q->r4, q->r4, q->blk, (int)q->nq, q->v4, q->v4, q->scal, q->red, q->s));
  QHIP(hipMemcpyAsync(&h, q->scal, sizeof(double), hipMemcpyDeviceToHost, q->s));
  if (r4p) QHIP(hipMemcpyAsync(r4p, q->r4, (size_t)(q->nq * q->v4) * 8, hipMemcpyDeviceToHost, q->s));
  QHIP(hipStreamSynchronize(q->s));
  q->have_r = true;
  if (norm2) *norm2 = h;
  if (!std::isfinite(h)) {
    q->err = "non-finite residual norm";
    return CCT_ENUMERIC;
  }
  return CCT_OK;
}

int cct_quad_copy_r4(cct_quad* q, int64_t first, int64_t count, double* out) {
  if (!q || !out || first < 0 || count < 0 || first + count > q->nq * q->v4) return CCT_EINVAL;
  if (!q->have_r) {
    q->err = "no residual yet (cct_quad_ladder)";
    return CCT_ESTATE;
  }
  QHIP(hipMemcpyAsync(out, q->r4 + first, (size_t)count * 8, hipMemcpyDeviceToHost, q->s));
  QHIP(hipStreamSynchronize(q->s));
  return CCT_OK;
}

int cct_quad_get_counters(cct_quad* q, double* macs, double* ms, int cap) {
  if (!q || cap < 0) return CCT_EINVAL;
  const double m[2] = {q->macs, 0.0};
  for (int i = 0; i < std::min(cap, 2); ++i) {
    if (macs) macs[i] = m[i];
    if (ms) ms[i] = q->ms[i];
  }
  return CCT_OK;
}

const char* cct_quad_last_error(const cct_quad* q) { return q ? q->err.c_str() : "null quad"; }

}  // extern "C"
