// libcct host runtime: context, memory plan, the RCCSDT iteration and the C ABI.
//
// One residual evaluation (paper, Appendix A; compact contractions of Sec.
// "Tensor contractions for compact amplitudes"):
//   1. T1 dressing of the density-fitting factors and the Fock matrix, and the
//      dressed integrals v~^{pq}_{rs} = sum_P B~^P_{pr} B~^P_{qs} (one GEMM).
//   2. RCCSD intermediates, R1 and the RCCSD part of R2.
//   3. RCCSDT intermediates W^{ab}_{dj}, W^{al}_{ij}, Wbar, W^{ab}_{de}.
//   4. T3 feedback into R1, R2, W^{ab}_{dj}, W^{al}_{ij} from unpacked,
//      spin-summed T3 slabs.
//   5. R3 on packed i<=j<=k blocks: particle-particle ladder by direct
//      traversal (each of the three relabelled terms split into symmetric
//      and antisymmetric halves over the virtual pairs, two GEMMs over all
//      stored blocks), Fock terms, hole ladder (+F_oo), the three ring types
//      and the two T2*W drivers by tile unpacking -> GEMM -> output-stationary
//      fold.
//   6. R3 post-processing fused with the norm and the Jacobi update.
#include "../../include/cct.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "contract.h"
#include "internal.h"

using namespace cct;

namespace {

struct Batch {
  int slot0 = 0, nslots = 0;
  int2* d_slots = nullptr;
  FoldTask* d_tasks = nullptr;
  int ntasks = 0;
  FoldContrib* d_contribs = nullptr;
};

struct Job {
  int nslot_total = 0;
  int per_batch = 1;
  std::vector<int2> slots;  // fixed occupied indices per slot
  std::vector<Batch> batches;
};

enum Phase { PH_CCSD = 0, PH_FEED, PH_PP, PH_RING, PH_HH, PH_DRV, PH_F1, PH_POST, PH_DIIS, PH_N };

const char* kErr[] = {"ok", "invalid argument", "out of device memory", "device error", "call out of order",
                      "non-finite residual or energy", "not converged"};

}  // namespace

struct cct_ctx {
  cct_alloc_fn alloc_fn = nullptr;  // the caller's device allocator (both null: hipMalloc / hipFree)
  cct_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  int o = 0, v = 0, n = 0, naux = 0;
  long long ntri = 0, v3 = 0;
  Prec prec = Prec::F64;
  hipStream_t s = nullptr;
  int dev = 0;  // the HIP device current at cct_create (the stream's device)
  int diis_space = 8, diis_start = 2;
  bool diis_on = true, diis_t3 = true;
  int diis_sv = 0;  // T3 in DIIS: the sub-cube a, b, c < diis_sv of every block (0: all of T3)
  double tol = 1e-8;  // default convergence threshold of cct_solve
  double ws_gb = 0.0;  // 0: size the workspace from free device memory
  int tune_ladder = 0, tune_rings = 0;  // GEMM tile variants chosen by cct_autotune (0 = size-based default)
  std::string err;
  bool have_f = false, have_B = false, have_res = false;

  std::vector<void*> owned;
  // inputs
  double *f = nullptr, *B = nullptr, *eps = nullptr, *fov = nullptr;
  double *vbare_c = nullptr;  // 2 v^{ij}_{ab} - v^{ij}_{ba} (bare), [i][j][a][b]
  double *vbare = nullptr;    // v^{ij}_{ab} (bare), [i][j][a][b]
  // dressed quantities
  double *Bt = nullptr, *ft = nullptr, *V = nullptr, *fG = nullptr, *G = nullptr, *cP = nullptr, *Dt = nullptr;
  // amplitudes and residuals
  double *t1 = nullptr, *t2 = nullptr, *t3 = nullptr, *r1 = nullptr, *r2 = nullptr, *r3 = nullptr, *X2 = nullptr;
  double *zero_r1 = nullptr;
  // intermediates
  double *tau2 = nullptr, *VCoovv = nullptr, *VCovvo = nullptr, *VCovvv = nullptr, *VCoovo = nullptr;
  double *Fvv = nullptr, *Foo = nullptr, *Woooo = nullptr, *Wh = nullptr, *Wovvo = nullptr, *Wovov = nullptr;
  double *Wt = nullptr, *Wvooo = nullptr, *Wb1 = nullptr, *Wb2 = nullptr, *Wvvvv = nullptr;
  double *tau_e = nullptr;
  // tables
  BlockRef* tbl = nullptr;
  int4* tri = nullptr;
  int* pair_rows = nullptr;  // p*o + q for the ordered pairs p <= q (hole ladder rows)
  long long* vpair_src = nullptr;  // (y*v + z)*v^2 for the virtual pairs y <= z (ladder W rows)
  int2* vpair_yz = nullptr;        // (y, z) of the virtual pairs y <= z
  bool ladder_split = true;        // symmetric / antisymmetric split of the ladder
  long long lp_block_k = 1024;     // split-BF16 ladder/ring operands with K >= this are stored by blocks of 32
  double* red = nullptr;  // reduction scratch
  long long red_n = 0;
  double* scal = nullptr;  // device scalars
  // workspace
  char* wsbuf = nullptr;
  Arena ws;
  // plans
  Job ring[3], hh, d1, d2, feed1;
  // DIIS
  // history in device memory: M slots of diis_len doubles, overlap matrix,
  // bookkeeping (see DiisArgs); diis_new: the Jacobi / extrapolated vector
  double *dvecs = nullptr, *derrs = nullptr, *diis_new = nullptr, *diis_part = nullptr;
  double *diis_d = nullptr, *diis_B = nullptr, *diis_coef = nullptr;
  int* diis_st = nullptr;
  double* diis_old = nullptr;
  long long diis_len = 0;
  // counters
  double macs[9] = {0};
  double ms[PH_N] = {0};
  hipEvent_t ev[PH_N + 1] = {};
  bool events = false;
  // device time of the ladder GEMM launches alone (event pairs around each
  // group of launches, created on first use), their multiply-adds and count
  std::vector<hipEvent_t> lad_ev;
  int lad_nev = 0;
  double lad_macs = 0.0, lad_launches = 0.0, lad_ms = 0.0;
  long long lad_chunks = 0;  // chunks of packed blocks the last ladder took
};

namespace {

#define HIPCK(expr)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                     \
      return CCT_EDEVICE;                                                               \
    }                                                                                   \
  } while (0)

#define STCK(expr)                                                                      \
  do {                                                                                  \
    Status st_ = (expr);                                                                \
    if (!st_.ok()) {                                                                    \
      ctx->err = st_.msg.empty() ? std::string(hipGetErrorString(st_.err)) : st_.msg;   \
      ctx->err += std::string(" [") + #expr + "]";                                      \
      return st_.msg.empty() ? CCT_EDEVICE : CCT_EINVAL;                                \
    }                                                                                   \
  } while (0)

#define RCK(expr)              \
  do {                         \
    int r_ = (expr);           \
    if (r_ != CCT_OK) return r_; \
  } while (0)

long long tri_count(int o) { return (long long)o * (o + 1) * (o + 2) / 6; }

// Device memory from the caller's allocator when one was given, else hipMalloc.
int dev_alloc(cct_ctx* ctx, void** p, size_t bytes) {
  void* q = nullptr;
  bytes = std::max<size_t>(bytes, 8);
  if (ctx->alloc_fn) {
    q = ctx->alloc_fn(bytes, ctx->alloc_user);
    if (!q || ((uintptr_t)q & 255)) {
      if (q) ctx->free_fn(q, ctx->alloc_user);
      ctx->err = "caller allocator: " + std::string(q ? "pointer not 256-byte aligned" : "NULL") + " for " +
                 std::to_string(bytes) + " bytes";
      return CCT_ENOMEM;
    }
  } else {
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
      ctx->err = std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e);
      return CCT_ENOMEM;
    }
  }
  *p = q;
  return CCT_OK;
}
void dev_free(cct_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx->free_fn) ctx->free_fn(p, ctx->alloc_user);
  else (void)hipFree(p);
}

int dalloc(cct_ctx* ctx, double** p, long long n) {
  void* q = nullptr;
  RCK(dev_alloc(ctx, &q, (size_t)std::max<long long>(n, 1) * sizeof(double)));
  ctx->owned.push_back(q);
  *p = (double*)q;
  return CCT_OK;
}

template <typename T>
int dalloc_t(cct_ctx* ctx, T** p, long long n) {
  void* q = nullptr;
  RCK(dev_alloc(ctx, &q, (size_t)std::max<long long>(n, 1) * sizeof(T)));
  ctx->owned.push_back(q);
  *p = (T*)q;
  return CCT_OK;
}

// --- options: a tiny reader for flat JSON objects ----------------------------
bool json_find(const std::string& js, const std::string& key, std::string& val) {
  const std::string pat = "\"" + key + "\"";
  size_t p = js.find(pat);
  if (p == std::string::npos) return false;
  p = js.find(':', p + pat.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < js.size() && (js[p] == ' ' || js[p] == '\t')) ++p;
  if (p < js.size() && js[p] == '"') {
    size_t q = js.find('"', p + 1);
    if (q == std::string::npos) return false;
    val = js.substr(p + 1, q - p - 1);
    return true;
  }
  size_t q = p;
  while (q < js.size() && js[q] != ',' && js[q] != '}' && js[q] != ' ') ++q;
  val = js.substr(p, q - p);
  return true;
}

// --- views of the dressed integrals -----------------------------------------
// v~^{pq}_{rs} is stored as V[p][r][q][s] (the GEMM over the fitting index).
DT Vv(cct_ctx* c, const char* blk) {
  const long long n = c->n;
  long long off[4], dim[4];
  for (int i = 0; i < 4; ++i) {
    off[i] = blk[i] == 'o' ? 0 : c->o;
    dim[i] = blk[i] == 'o' ? c->o : c->v;
  }
  DT t;
  t.p = c->V + off[0] * n * n * n + off[2] * n * n + off[1] * n + off[3];
  t.nd = 4;
  for (int i = 0; i < 4; ++i) t.dim[i] = dim[i];
  t.st[0] = n * n * n;
  t.st[1] = n;
  t.st[2] = n * n;
  t.st[3] = 1;
  return t;
}

DT fview(cct_ctx* c, double* base, char a, char b) {
  const long long n = c->n;
  const long long oa = a == 'o' ? 0 : c->o, ob = b == 'o' ? 0 : c->o;
  return strided(base + oa * n + ob, {a == 'o' ? c->o : c->v, b == 'o' ? c->o : c->v}, {n, 1});
}

// Table of unpacked blocks: for every ordered (p,q,r) the stored block
// sort(p,q,r) and the strides of the three virtual axes in the order of
// (p,q,r) (the column symmetry carries the virtual labels along).
void build_tables(int o, int v, std::vector<BlockRef>& tbl, std::vector<int4>& tri) {
  std::map<std::array<int, 3>, int> index;
  tri.clear();
  for (int i = 0; i < o; ++i)
    for (int j = i; j < o; ++j)
      for (int k = j; k < o; ++k) {
        index[{i, j, k}] = (int)tri.size();
        const int mult = (i == j && j == k) ? 1 : ((i == j || j == k) ? 3 : 6);
        tri.push_back(int4{i, j, k, mult});
      }
  const long long v3 = (long long)v * v * v;
  const int axis_stride[3] = {v * v, v, 1};
  tbl.assign((size_t)o * o * o, BlockRef{});
  for (int p = 0; p < o; ++p)
    for (int q = 0; q < o; ++q)
      for (int r = 0; r < o; ++r) {
        const int occ[3] = {p, q, r};
        int order[3] = {0, 1, 2};
        std::stable_sort(order, order + 3, [&](int x, int y) { return occ[x] < occ[y]; });
        BlockRef b{};
        b.off = (long long)index[{occ[order[0]], occ[order[1]], occ[order[2]]}] * v3;
        for (int nax = 0; nax < 3; ++nax) b.s[order[nax]] = axis_stride[nax];
        tbl[((size_t)p * o + q) * o + r] = b;
      }
}

// ---------------------------------------------------------------------------
// Fold plans
// ---------------------------------------------------------------------------
struct Contrib {
  int slot;
  long long base;
  long long sa, sb, sc;
  double coef;
};

// Build the batches of a job: per batch, fold tasks grouping contributions by
// output block.  contribs_of(t) lists the contributions of packed triple t.
template <typename F>
int build_job(cct_ctx* ctx, Job& job, long long slot_doubles, F contribs_of) {
  const int S = job.per_batch;
  const int nb = (job.nslot_total + S - 1) / S;
  std::vector<std::vector<std::pair<int, FoldContrib>>> per_batch(nb);
  for (long long t = 0; t < ctx->ntri; ++t) {
    std::vector<Contrib> cs = contribs_of((int)t);
    for (const Contrib& c : cs) {
      if (c.slot < 0 || c.slot >= job.nslot_total) {
        ctx->err = "fold plan: slot out of range";
        return CCT_EINVAL;
      }
      const int b = c.slot / S;
      const int ls = c.slot - b * S;
      // every element read by this contribution must lie inside its slot
      const long long vm = ctx->v - 1;
      if (c.base < 0 || c.base + vm * (c.sa + c.sb + c.sc) >= slot_doubles) {
        ctx->err = "fold plan: contribution exceeds its slot";
        return CCT_EINVAL;
      }
      FoldContrib fc{(long long)ls * slot_doubles + c.base, c.sa, c.sb, c.sc, c.coef};
      per_batch[b].push_back({(int)t, fc});
    }
  }
  job.batches.clear();
  for (int b = 0; b < nb; ++b) {
    Batch B;
    B.slot0 = b * S;
    B.nslots = std::min(S, job.nslot_total - b * S);
    auto& lst = per_batch[b];
    std::stable_sort(lst.begin(), lst.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    std::vector<FoldTask> tasks;
    std::vector<FoldContrib> cons;
    for (size_t i = 0; i < lst.size();) {
      size_t j = i;
      FoldTask tk{lst[i].first, 0, (int)cons.size(), 0};
      while (j < lst.size() && lst[j].first == lst[i].first) {
        cons.push_back(lst[j].second);
        ++j;
      }
      tk.nc = (int)(j - i);
      tasks.push_back(tk);
      i = j;
    }
    B.ntasks = (int)tasks.size();
    RCK(dalloc_t(ctx, &B.d_slots, B.nslots));
    RCK(dalloc_t(ctx, &B.d_tasks, std::max<size_t>(tasks.size(), 1)));
    RCK(dalloc_t(ctx, &B.d_contribs, std::max<size_t>(cons.size(), 1)));
    HIPCK(hipMemcpy(B.d_slots, job.slots.data() + B.slot0, sizeof(int2) * B.nslots, hipMemcpyHostToDevice));
    if (!tasks.empty()) {
      HIPCK(hipMemcpy(B.d_tasks, tasks.data(), sizeof(FoldTask) * tasks.size(), hipMemcpyHostToDevice));
      HIPCK(hipMemcpy(B.d_contribs, cons.data(), sizeof(FoldContrib) * cons.size(), hipMemcpyHostToDevice));
    }
    job.batches.push_back(B);
  }
  return CCT_OK;
}

const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

int slots_per_batch(long long budget_doubles, long long per_slot, int nslots) {
  long long s = budget_doubles / std::max<long long>(per_slot, 1);
  if (s < 1) s = 1;
  if (s > nslots) s = nslots;
  if (s > 4096) s = 4096;
  return (int)s;
}

int build_plans(cct_ctx* ctx) {
  const int o = ctx->o, v = ctx->v;
  const long long v2 = (long long)v * v, v3 = v2 * v;
  const long long ov3 = o * v3, o2v3 = (long long)o * o * v3;
  std::vector<int4> tri;
  std::vector<BlockRef> tbl;
  build_tables(o, v, tbl, tri);
  // scratch left after the planner's operand copies (at most a few o*v^3 blocks)
  const long long budget = (long long)(ctx->ws.capacity() / sizeof(double)) - 6 * ov3 - (1 << 22);
  if (budget < 2 * o2v3) {
    ctx->err = "workspace too small for one unpacked slab";
    return CCT_ENOMEM;
  }
  // ---- rings: slots are occupied pairs; A and B over q <= r, C over all (q, r)
  std::map<std::pair<int, int>, int> pair_ab, pair_c;
  for (int q = 0; q < o; ++q)
    for (int r = q; r < o; ++r) {
      pair_ab[{q, r}] = (int)ctx->ring[0].slots.size();
      ctx->ring[0].slots.push_back(int2{q, r});
    }
  ctx->ring[1].slots = ctx->ring[0].slots;
  for (int q = 0; q < o; ++q)
    for (int r = 0; r < o; ++r) {
      pair_c[{q, r}] = (int)ctx->ring[2].slots.size();
      ctx->ring[2].slots.push_back(int2{q, r});
    }
  const double ring_coef[3] = {0.5, -0.5, -1.0};
  for (int kind = 0; kind < 3; ++kind) {
    Job& J = ctx->ring[kind];
    J.nslot_total = (int)J.slots.size();
    // per slot: the unpacked operand U (rows padded by < 32) and the products Z,
    // each in its working format (FP64; FP32 U and FP64 Z; split-BF16 U and FP32 Z)
    const long long ring_slot = ctx->prec == Prec::F64 ? 2 * ov3 : (ctx->prec == Prec::F32 ? ov3 + ov3 / 2 : ov3);
    J.per_batch = slots_per_batch(budget, ring_slot + 16 * v2, J.nslot_total);
    const double cf = ring_coef[kind];
    RCK(build_job(ctx, J, ov3, [&](int t) {
      std::vector<Contrib> cs;
      const int occ[3] = {tri[t].x, tri[t].y, tri[t].z};
      if (kind < 2) {
        // Y(p; q, r)[x; y, z] stored as Z[slot(q,r)][p][x][y][z]
        // sigma1: (i; j,k)[a; b,c]   sigma2: (j; i,k)[b; a,c]   sigma3: (k; i,j)[c; a,b]
        cs.push_back({pair_ab[{occ[1], occ[2]}], (long long)occ[0] * v3, v2, v, 1, cf});
        cs.push_back({pair_ab[{occ[0], occ[2]}], (long long)occ[1] * v3, v, v2, 1, cf});
        cs.push_back({pair_ab[{occ[0], occ[1]}], (long long)occ[2] * v3, v, 1, v2, cf});
      } else {
        // Y(p,q,r)[x,y,z] stored as Z[slot(q,r)][p][y][x][z]; six column permutations
        for (int s = 0; s < 6; ++s) {
          const int* pi = PERM3[s];
          long long st[3];
          st[pi[0]] = v;
          st[pi[1]] = v2;
          st[pi[2]] = 1;
          cs.push_back({pair_c[{occ[pi[1]], occ[pi[2]]}], (long long)occ[pi[0]] * v3, st[0], st[1], st[2], cf});
        }
      }
      return cs;
    }));
  }
  // ---- hole ladder (+ F_oo): slots are r; Z[slot(r)][pair(p<=q)][x][y][z]
  //      (every contribution of a packed triple has its first two occupied
  //      indices in order, so only the o(o+1)/2 ordered pairs are formed)
  {
    Job& J = ctx->hh;
    const long long npair = (long long)o * (o + 1) / 2;
    auto pidx = [o](int p, int q) { return (long long)p * o - (long long)p * (p - 1) / 2 + (q - p); };
    for (int r = 0; r < o; ++r) J.slots.push_back(int2{r, 0});
    J.nslot_total = o;
    J.per_batch = slots_per_batch(budget, o2v3 + npair * v3, o);
    RCK(build_job(ctx, J, npair * v3, [&](int t) {
      const int i = tri[t].x, j = tri[t].y, k = tri[t].z;
      std::vector<Contrib> cs;
      cs.push_back({k, pidx(i, j) * v3, v2, v, 1, 1.0});  // (i,j;k)[a,b;c]
      cs.push_back({j, pidx(i, k) * v3, v2, 1, v, 1.0});  // (i,k;j)[a,c;b]
      cs.push_back({i, pidx(j, k) * v3, 1, v2, v, 1.0});  // (j,k;i)[b,c;a]
      return cs;
    }));
    std::vector<int> rows;
    for (int p_ = 0; p_ < o; ++p_)
      for (int q = p_; q < o; ++q) rows.push_back(p_ * o + q);
    RCK(dalloc_t(ctx, &ctx->pair_rows, (long long)rows.size()));
    HIPCK(hipMemcpy(ctx->pair_rows, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice));
  }
  // ---- ladder split: the virtual pairs y <= z in the order p(y,z)
  {
    std::vector<long long> src;
    std::vector<int2> yz;
    for (int y = 0; y < v; ++y)
      for (int z = y; z < v; ++z) {
        src.push_back(((long long)y * v + z) * v2);
        yz.push_back(int2{y, z});
      }
    RCK(dalloc_t(ctx, &ctx->vpair_src, (long long)src.size()));
    RCK(dalloc_t(ctx, &ctx->vpair_yz, (long long)yz.size()));
    HIPCK(hipMemcpy(ctx->vpair_src, src.data(), sizeof(long long) * src.size(), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(ctx->vpair_yz, yz.data(), sizeof(int2) * yz.size(), hipMemcpyHostToDevice));
  }
  // ---- drivers
  {
    Job& J = ctx->d1;  // slots q; Z[slot(q)][(x,y)][(p,r,z)]
    for (int q = 0; q < o; ++q) J.slots.push_back(int2{q, 0});
    J.nslot_total = o;
    J.per_batch = slots_per_batch(budget, o2v3, o);
    const long long sx = (long long)o * o * v2, sy = (long long)o * o * v;
    RCK(build_job(ctx, J, o2v3, [&](int t) {
      const int occ[3] = {tri[t].x, tri[t].y, tri[t].z};
      std::vector<Contrib> cs;
      for (int s = 0; s < 6; ++s) {
        const int* pi = PERM3[s];
        long long st[3];
        st[pi[0]] = sx;
        st[pi[1]] = sy;
        st[pi[2]] = 1;
        const int p = occ[pi[0]], q = occ[pi[1]], r = occ[pi[2]];
        cs.push_back({q, ((long long)p * o + r) * v, st[0], st[1], st[2], 1.0});
      }
      return cs;
    }));
  }
  {
    Job& J = ctx->d2;  // slots r; Z[slot(r)][(x,p,q)][(y,z)]
    for (int r = 0; r < o; ++r) J.slots.push_back(int2{r, 0});
    J.nslot_total = o;
    J.per_batch = slots_per_batch(budget, o2v3, o);
    const long long sx = (long long)o * o * v2;
    RCK(build_job(ctx, J, o2v3, [&](int t) {
      const int occ[3] = {tri[t].x, tri[t].y, tri[t].z};
      std::vector<Contrib> cs;
      for (int s = 0; s < 6; ++s) {
        const int* pi = PERM3[s];
        long long st[3];
        st[pi[0]] = sx;
        st[pi[1]] = v;
        st[pi[2]] = 1;
        const int p = occ[pi[0]], q = occ[pi[1]], r = occ[pi[2]];
        cs.push_back({r, ((long long)p * o + q) * v2, st[0], st[1], st[2], -1.0});
      }
      return cs;
    }));
  }
  // ---- feedback unpack batches (no fold)
  for (Job* J : {&ctx->feed1}) {
    for (int f = 0; f < o; ++f) J->slots.push_back(int2{f, 0});
    J->nslot_total = o;
    J->per_batch = slots_per_batch(budget, 2 * o2v3 + (long long)o * o * v2, o);  // UA, UB, one X2 partial
    const int S = J->per_batch;
    for (int b = 0; b * S < o; ++b) {
      Batch B;
      B.slot0 = b * S;
      B.nslots = std::min(S, o - b * S);
      RCK(dalloc_t(ctx, &B.d_slots, B.nslots));
      HIPCK(hipMemcpy(B.d_slots, J->slots.data() + B.slot0, sizeof(int2) * B.nslots, hipMemcpyHostToDevice));
      J->batches.push_back(B);
    }
  }
  RCK(dalloc_t(ctx, &ctx->tbl, (long long)tbl.size()));
  RCK(dalloc_t(ctx, &ctx->tri, (long long)tri.size()));
  HIPCK(hipMemcpy(ctx->tbl, tbl.data(), sizeof(BlockRef) * tbl.size(), hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(ctx->tri, tri.data(), sizeof(int4) * tri.size(), hipMemcpyHostToDevice));
  return CCT_OK;
}

// Unpack terms: spin-summation combinations on the first column (S1) and on
// the first two columns (S12), as linear combinations of virtual orders.
void set_s1(UnpackArgs& a, const int occ[3]) {
  const UnpackTerm t[3] = {{2.0, {occ[0], occ[1], occ[2]}, {0, 1, 2}},
                           {-1.0, {occ[0], occ[1], occ[2]}, {1, 0, 2}},
                           {-1.0, {occ[0], occ[1], occ[2]}, {2, 1, 0}}};
  a.nterms = 3;
  for (int i = 0; i < 3; ++i) a.terms[i] = t[i];
}

void set_s12(UnpackArgs& a, const int occ[3]) {
  const double c[6] = {4.0, -2.0, -2.0, -2.0, 1.0, 1.0};
  const int vp[6][3] = {{0, 1, 2}, {1, 0, 2}, {2, 1, 0}, {0, 2, 1}, {2, 0, 1}, {1, 2, 0}};
  a.nterms = 6;
  for (int i = 0; i < 6; ++i) {
    a.terms[i].coef = c[i];
    for (int m = 0; m < 3; ++m) {
      a.terms[i].occ[m] = occ[m];
      a.terms[i].virt[m] = vp[i][m];
    }
  }
}

void set_ident(UnpackArgs& a, const int occ[3]) {
  a.nterms = 1;
  a.terms[0].coef = 1.0;
  for (int m = 0; m < 3; ++m) {
    a.terms[0].occ[m] = occ[m];
    a.terms[0].virt[m] = m;
  }
}

// ---------------------------------------------------------------------------
// timing helpers
// ---------------------------------------------------------------------------
void mark(cct_ctx* ctx, int ph) {
  if (ctx->events) (void)hipEventRecord(ctx->ev[ph], ctx->s);
}

// Bracket a group of ladder GEMM launches (macs: their multiply-adds,
// n: launches).  Timing stops quietly past 256 groups per residual.
void lad_begin(cct_ctx* ctx) {
  if (!ctx->events || ctx->lad_nev >= 512) return;
  while ((int)ctx->lad_ev.size() < ctx->lad_nev + 2) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    ctx->lad_ev.push_back(e);
  }
  (void)hipEventRecord(ctx->lad_ev[ctx->lad_nev], ctx->s);
}
void lad_end(cct_ctx* ctx, double macs, int n) {
  ctx->lad_macs += macs;
  ctx->lad_launches += n;
  if (!ctx->events || ctx->lad_nev >= 512 || (int)ctx->lad_ev.size() < ctx->lad_nev + 2) return;
  (void)hipEventRecord(ctx->lad_ev[ctx->lad_nev + 1], ctx->s);
  ctx->lad_nev += 2;
}

// ---------------------------------------------------------------------------
// the residual
// ---------------------------------------------------------------------------
int dress(cct_ctx* ctx) {
  const int o = ctx->o, v = ctx->v, n = ctx->n;
  const long long naux = ctx->naux;
  const long long n2 = (long long)n * n;
  hipStream_t s = ctx->s;
  // Bt = x B y^T per fitting index P; x = 1 - t1 (rows of virtuals), y^T = 1 + t1 (columns of occupied)
  HIPCK(axpby(1.0, ctx->B, 0.0, ctx->Bt, (long long)naux * n2, s));
  {
    GemmArgs g{};  // Bt[P][o+a][q] -= sum_i t1[i][a] B[P][i][q]
    g.M = v; g.N = n; g.K = o; g.batch = (int)naux;
    g.A = ctx->t1; g.am = idx1(1); g.ak = idx1(v); g.a_batch = 0;
    g.B = ctx->B; g.bk = idx1(n); g.bn = idx1(1); g.b_batch = n2;
    g.C = ctx->Bt + (long long)o * n; g.cm = idx1(n); g.cn = idx1(1); g.c_batch = n2;
    g.alpha = -1.0; g.beta = 1.0;
    g.a_len = (long long)o * v; g.b_len = naux * n2; g.c_len = naux * n2 - (long long)o * n;
    HIPCK(gemm(g, Prec::F64, s));
  }
  {
    GemmArgs g{};  // Bt[P][p][i] += sum_a Bt[P][p][o+a] t1[i][a]
    g.M = n; g.N = o; g.K = v; g.batch = (int)naux;
    g.A = ctx->Bt + o; g.am = idx1(n); g.ak = idx1(1); g.a_batch = n2;
    g.B = ctx->t1; g.bk = idx1(1); g.bn = idx1(v); g.b_batch = 0;
    g.C = ctx->Bt; g.cm = idx1(n); g.cn = idx1(1); g.c_batch = n2;
    g.alpha = 1.0; g.beta = 1.0;
    g.a_len = naux * n2 - o; g.b_len = (long long)o * v; g.c_len = naux * n2;
    HIPCK(gemm(g, Prec::F64, s));
  }
  // G_rs = 2 sum_P c_P B[P][r][s] - sum_{P,i} D[P][r][i] B[P][i][s],
  // c_P = sum_ia B[P][i][o+a] t_ia, D[P][r][i] = sum_a B[P][r][o+a] t_ia
  {
    GemmArgs g{};
    g.M = (int)naux; g.N = 1; g.K = o * v; g.batch = 1;
    g.A = ctx->B + o; g.am = idx1(n2); g.ak = idx2(v, n, 1);
    g.B = ctx->t1; g.bk = idx1(1); g.bn = idx1(0);
    g.C = ctx->cP; g.cm = idx1(1); g.cn = idx1(0);
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = naux * n2 - o; g.b_len = (long long)o * v; g.c_len = naux;
    HIPCK(gemm(g, Prec::F64, s));
  }
  {
    GemmArgs g{};
    g.M = 1; g.N = (int)n2; g.K = (int)naux; g.batch = 1;
    g.A = ctx->cP; g.am = idx1(0); g.ak = idx1(1);
    g.B = ctx->B; g.bk = idx1(n2); g.bn = idx1(1);
    g.C = ctx->G; g.cm = idx1(0); g.cn = idx1(1);
    g.alpha = 2.0; g.beta = 0.0;
    g.a_len = naux; g.b_len = naux * n2; g.c_len = n2;
    HIPCK(gemm(g, Prec::F64, s));
  }
  {
    GemmArgs g{};
    g.M = n; g.N = o; g.K = v; g.batch = (int)naux;
    g.A = ctx->B + o; g.am = idx1(n); g.ak = idx1(1); g.a_batch = n2;
    g.B = ctx->t1; g.bk = idx1(1); g.bn = idx1(v); g.b_batch = 0;
    g.C = ctx->Dt; g.cm = idx1(o); g.cn = idx1(1); g.c_batch = (long long)n * o;
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = naux * n2 - o; g.b_len = (long long)o * v; g.c_len = (long long)naux * n * o;
    HIPCK(gemm(g, Prec::F64, s));
  }
  {
    GemmArgs g{};
    g.M = n; g.N = n; g.K = (int)naux * o; g.batch = 1;
    g.A = ctx->Dt; g.am = idx1(o); g.ak = idx2(o, (long long)n * o, 1);
    g.B = ctx->B; g.bk = idx2(o, n2, n); g.bn = idx1(1);
    g.C = ctx->G; g.cm = idx1(n); g.cn = idx1(1);
    g.alpha = -1.0; g.beta = 1.0;
    g.a_len = (long long)naux * n * o; g.b_len = naux * n2; g.c_len = n2;
    HIPCK(gemm(g, Prec::F64, s));
  }
  HIPCK(axpby(1.0, ctx->f, 0.0, ctx->fG, n2, s));
  HIPCK(axpby(1.0, ctx->G, 1.0, ctx->fG, n2, s));
  HIPCK(axpby(1.0, ctx->fG, 0.0, ctx->ft, n2, s));
  {
    GemmArgs g{};
    g.M = v; g.N = n; g.K = o; g.batch = 1;
    g.A = ctx->t1; g.am = idx1(1); g.ak = idx1(v);
    g.B = ctx->fG; g.bk = idx1(n); g.bn = idx1(1);
    g.C = ctx->ft + (long long)o * n; g.cm = idx1(n); g.cn = idx1(1);
    g.alpha = -1.0; g.beta = 1.0;
    g.a_len = (long long)o * v; g.b_len = n2; g.c_len = n2 - (long long)o * n;
    HIPCK(gemm(g, Prec::F64, s));
  }
  {
    GemmArgs g{};
    g.M = n; g.N = o; g.K = v; g.batch = 1;
    g.A = ctx->ft + o; g.am = idx1(n); g.ak = idx1(1);
    g.B = ctx->t1; g.bk = idx1(1); g.bn = idx1(v);
    g.C = ctx->ft; g.cm = idx1(n); g.cn = idx1(1);
    g.alpha = 1.0; g.beta = 1.0;
    g.a_len = n2 - o; g.b_len = (long long)o * v; g.c_len = n2;
    HIPCK(gemm(g, Prec::F64, s));
  }
  // V[(p,r)][(q,s)] = sum_P Bt[P][p][r] Bt[P][q][s]
  {
    GemmArgs g{};
    g.M = (int)n2; g.N = (int)n2; g.K = (int)naux; g.batch = 1;
    g.A = ctx->Bt; g.am = idx1(1); g.ak = idx1(n2);
    g.B = ctx->Bt; g.bk = idx1(n2); g.bn = idx1(1);
    g.C = ctx->V; g.cm = idx1(n2); g.cn = idx1(1);
    g.alpha = 1.0; g.beta = 0.0;
    g.a_len = naux * n2; g.b_len = naux * n2; g.c_len = n2 * n2;
    HIPCK(gemm(g, Prec::F64, s));
  }
  return CCT_OK;
}

int ccsd_part(cct_ctx* ctx) {
  const int o = ctx->o, v = ctx->v;
  hipStream_t s = ctx->s;
  Arena& ws = ctx->ws;
  const Prec F = Prec::F64;
  DT t2 = dense(ctx->t2, {o, o, v, v});
  DT tau = dense(ctx->tau2, {o, o, v, v});
  STCK(accumulate(s, 2.0, t2, "ijab", 0.0, tau, "ijab"));
  STCK(accumulate(s, -1.0, t2, "ijba", 1.0, tau, "ijab"));
  // spin-summed integral blocks  2 v~^{pq}_{rs} - v~^{pq}_{sr}
  struct VC { double* p; const char* blk; const char* sw; } vcs[4] = {
      {ctx->VCoovv, "oovv", "oovv"}, {ctx->VCovvo, "ovvo", "ovov"}, {ctx->VCovvv, "ovvv", "ovvv"},
      {ctx->VCoovo, "oovo", "ooov"}};
  for (auto& c : vcs) {
    DT src = Vv(ctx, c.blk), sw = Vv(ctx, c.sw);
    DT d = dense(c.p, {src.dim[0], src.dim[1], src.dim[2], src.dim[3]});
    STCK(accumulate(s, 2.0, src, "pqrs", 0.0, d, "pqrs"));
    STCK(accumulate(s, -1.0, sw, "pqsr", 1.0, d, "pqrs"));
  }
  DT VCoovv = dense(ctx->VCoovv, {o, o, v, v}), VCovvo = dense(ctx->VCovvo, {o, v, v, o});
  DT VCovvv = dense(ctx->VCovvv, {o, v, v, v}), VCoovo = dense(ctx->VCoovo, {o, o, v, o});
  DT Fvv = dense(ctx->Fvv, {v, v}), Foo = dense(ctx->Foo, {o, o});
  DT Woooo = dense(ctx->Woooo, {o, o, o, o}), Wovvo = dense(ctx->Wovvo, {o, v, v, o});
  DT Wovov = dense(ctx->Wovov, {o, v, o, v});
  // RCCSD intermediates
  STCK(accumulate(s, 1.0, fview(ctx, ctx->ft, 'v', 'v'), "bc", 0.0, Fvv, "bc"));
  STCK(contract(ws, s, F, -1.0, VCoovv, "kldc", t2, "kldb", 1.0, Fvv, "bc"));
  STCK(accumulate(s, 1.0, fview(ctx, ctx->ft, 'o', 'o'), "kj", 0.0, Foo, "kj"));
  STCK(contract(ws, s, F, 1.0, VCoovv, "lkcd", t2, "ljcd", 1.0, Foo, "kj"));
  STCK(accumulate(s, 1.0, Vv(ctx, "oooo"), "klij", 0.0, Woooo, "klij"));
  STCK(contract(ws, s, F, 1.0, Vv(ctx, "oovv"), "klcd", t2, "ijcd", 1.0, Woooo, "klij"));
  STCK(accumulate(s, 1.0, VCovvo, "kaci", 0.0, Wovvo, "kaci"));
  STCK(contract(ws, s, F, 0.5, VCoovv, "lkdc", tau, "lida", 1.0, Wovvo, "kaci"));
  STCK(accumulate(s, 1.0, Vv(ctx, "ovov"), "kaic", 0.0, Wovov, "kaic"));
  STCK(contract(ws, s, F, -0.5, Vv(ctx, "oovv"), "lkcd", t2, "ilda", 1.0, Wovov, "kaic"));
  // R1 (RCCSD part)
  DT r1 = dense(ctx->r1, {o, v});
  STCK(accumulate(s, 1.0, fview(ctx, ctx->ft, 'v', 'o'), "ai", 0.0, r1, "ia"));
  STCK(contract(ws, s, F, 1.0, fview(ctx, ctx->ft, 'o', 'v'), "kc", tau, "ikac", 1.0, r1, "ia"));
  STCK(contract(ws, s, F, 1.0, Vv(ctx, "vovv"), "akcd", tau, "ikcd", 1.0, r1, "ia"));
  STCK(contract(ws, s, F, -1.0, Vv(ctx, "ooov"), "klic", tau, "klac", 1.0, r1, "ia"));
  // R2 (RCCSD part) before P_(ia)(jb)
  DT X2 = dense(ctx->X2, {o, o, v, v});
  DT Wvvvv = dense(ctx->Wvvvv, {v, v, v, v});
  STCK(accumulate(s, 0.5, Vv(ctx, "vvoo"), "abij", 0.0, X2, "ijab"));
  STCK(contract(ws, s, F, 1.0, Fvv, "bc", t2, "ijac", 1.0, X2, "ijab"));
  STCK(contract(ws, s, F, -1.0, Foo, "kj", t2, "ikab", 1.0, X2, "ijab"));
  STCK(accumulate(s, 1.0, Vv(ctx, "vvvv"), "abcd", 0.0, Wvvvv, "abcd"));
  STCK(contract(ws, s, F, 0.5, Wvvvv, "abcd", t2, "ijcd", 1.0, X2, "ijab"));
  STCK(contract(ws, s, F, 0.5, Woooo, "klij", t2, "klab", 1.0, X2, "ijab"));
  STCK(contract(ws, s, F, 0.5, Wovvo, "kaci", tau, "kjcb", 1.0, X2, "ijab"));
  STCK(contract(ws, s, F, -0.5, Wovov, "kaic", t2, "jkcb", 1.0, X2, "ijab"));
  STCK(contract(ws, s, F, -1.0, Wovov, "kbic", t2, "jkca", 1.0, X2, "ijab"));
  // RCCSDT intermediates (T2 parts)
  DT Wt = dense(ctx->Wt, {v, o, v, v});  // [d][j][b][a] = W^{ab}_{dj}
  STCK(accumulate(s, 1.0, Vv(ctx, "vvvo"), "abdj", 0.0, Wt, "djba"));
  STCK(contract(ws, s, F, 0.5, VCovvv, "laed", tau, "ljeb", 1.0, Wt, "djba"));
  STCK(contract(ws, s, F, -0.5, Vv(ctx, "ovvv"), "lade", t2, "jleb", 1.0, Wt, "djba"));
  STCK(contract(ws, s, F, -1.0, Vv(ctx, "ovvv"), "lbde", t2, "jlea", 1.0, Wt, "djba"));
  STCK(contract(ws, s, F, 1.0, Vv(ctx, "oovo"), "lmdj", t2, "lmab", 1.0, Wt, "djba"));
  DT Wvooo = dense(ctx->Wvooo, {v, o, o, o});  // [a][l][i][j] = W^{al}_{ij}
  STCK(accumulate(s, 1.0, Vv(ctx, "vooo"), "alij", 0.0, Wvooo, "alij"));
  STCK(contract(ws, s, F, 1.0, fview(ctx, ctx->ft, 'o', 'v'), "ld", t2, "ijad", 1.0, Wvooo, "alij"));
  STCK(contract(ws, s, F, 0.5, VCoovo, "mldj", tau, "mida", 1.0, Wvooo, "alij"));
  STCK(contract(ws, s, F, -0.5, Vv(ctx, "ooov"), "mljd", t2, "imda", 1.0, Wvooo, "alij"));
  STCK(contract(ws, s, F, -1.0, Vv(ctx, "ooov"), "mlid", t2, "jmda", 1.0, Wvooo, "alij"));
  STCK(contract(ws, s, F, 1.0, Vv(ctx, "vovv"), "alde", t2, "ijde", 1.0, Wvooo, "alij"));
  // Wbar^{la}_{di} and Wbar^{la}_{id}, both stored [i][a][l][d]: the ring
  // contractions read them as (i,a) x (l,d) row-major matrices
  DT Wb1 = dense(ctx->Wb1, {o, v, o, v});
  STCK(accumulate(s, 1.0, Wovvo, "ladi", 0.0, Wb1, "iald"));
  STCK(contract(ws, s, F, 0.5, VCoovv, "mled", tau, "miea", 1.0, Wb1, "iald"));
  DT Wb2 = dense(ctx->Wb2, {o, v, o, v});
  STCK(accumulate(s, 1.0, Wovov, "laid", 0.0, Wb2, "iald"));
  STCK(contract(ws, s, F, -0.5, Vv(ctx, "oovv"), "mlde", t2, "imea", 1.0, Wb2, "iald"));
  STCK(contract(ws, s, F, 1.0, Vv(ctx, "oovv"), "lmde", t2, "lmab", 1.0, Wvvvv, "abde"));
  return CCT_OK;
}

// T3 contributions to R1, R2 and to W^{ab}_{dj}, W^{al}_{ij} (RCCSDT
// appendix).  For each batch of first-column indices f the spin-summed slab
// U_f[o1][o2][x][y][z] = t~_{f o1 o2}^{xyz} (single check on column 1) is
// unpacked once and contracted five ways; R1's double check is rebuilt from
// the same slab: t~_{j'k'i}^{b'c'a} = 2 U_j[k][i][b][c][a] - U_j[k][i][b][a][c].
// K-contiguous product C = alpha A B^T + beta C (A: M x K rows of lda, B: N x K
// rows of ldb): the matrix-core NT kernel when its alignment rules hold, the
// generic strided kernel otherwise.
int nt_or_generic(cct_ctx* ctx, int M, int N, long long K, const double* A, long long lda, long long a_len,
                  const double* B, long long ldb, long long b_len, double* C, Idx2 cm, Idx2 cn, long long c_len,
                  double alpha, double beta) {
  const bool even = !(K & 1) && !(lda & 1) && !(ldb & 1) && !((uintptr_t)A & 15) && !((uintptr_t)B & 15);
  if (K > INT_MAX) { ctx->err = "contraction length exceeds int"; return CCT_EINVAL; }
  if (even) {
    NtArgs g{};
    g.M = M; g.N = N; g.K = (int)K; g.batch = 1;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb;
    g.C = C; g.cm = cm; g.cn = cn;
    g.alpha = alpha; g.beta = beta;
    g.a_len = a_len; g.b_len = b_len; g.c_len = c_len;
    HIPCK(gemm_nt(g, Prec::F64, ctx->s));
  } else {
    GemmArgs g{};
    g.M = M; g.N = N; g.K = (int)K; g.batch = 1;
    g.A = A; g.am = idx1(lda); g.ak = idx1(1);
    g.B = B; g.bk = idx1(1); g.bn = idx1(ldb);
    g.C = C; g.cm = cm; g.cn = cn;
    g.alpha = alpha; g.beta = beta;
    g.a_len = a_len; g.b_len = b_len; g.c_len = c_len;
    HIPCK(gemm(g, Prec::F64, ctx->s));
  }
  return CCT_OK;
}

// T3 -> R1, R2, W^{ab}_{dj}, W^{al}_{ij} (Eq. resi-rccsdt feedback terms and
// the T3 parts of the two RCCSDT intermediates).  For a batch of S slots f,
// the single-check spin-summed amplitudes t~_{f..}^{...} are unpacked twice,
// in the two layouts that make every contraction one K-contiguous GEMM with
// the slot index folded into K:
//   UA[(i,j,a)][f][(p,q)] = t~_{fij}^{q a p}   (K = f, two virtuals)
//   UB[(i,a,b)][f][(k,c)] = t~_{fik}^{c a b}   (K = f, occupied, virtual)
// and
//   X2[ij][ab] +=  sum_{fcd} v~^{bf}_{cd} t~_{fij}^{dac} + 1/2 sum_{fc} f~^f_c t~_{fij}^{cab}   (UA, one GEMM:
//                  the Fock term rides on the diagonal p = b of the integral rows)
//   X2[ij][ab] -=  sum_{fkc} v~^{kf}_{jc} t~_{fik}^{cab}                                         (UB)
//   W^{ab}_{dj} -= sum_{fle} v~^{lf}_{de} t~_{fjl}^{eba}                                         (UB)
//   W^{al}_{ij} += sum_{fde} v~^{lf}_{de} t~_{fij}^{ead}                                         (UA)
//   R1[ia]      += 1/2 sum v~^{jk}_{bc} (2 t~_{jki}^{bca} - t~_{jki}^{bac})                        (UA, reduction kernel)
int feedback(cct_ctx* ctx) {
  const int o = ctx->o, v = ctx->v, n = ctx->n;
  const long long v2 = (long long)v * v, v3 = ctx->v3, o2v3 = (long long)o * o * v3;
  const long long ov = (long long)o * v, o2v2 = ov * ov;
  hipStream_t s = ctx->s;
  Arena& ws = ctx->ws;
  const size_t mk0 = ws.mark();
  // integral slices with the summed slot index next to the contracted pair
  double* VbT = ws.alloc((size_t)(o * v3));            // [b][f][c][d] = v~^{bf}_{cd} (+ 1/2 f~ on c = b)
  double* VcT = ws.alloc((size_t)o * o * o * v);       // [j][f][k][c] = v~^{kf}_{jc}
  double* VdT = ws.alloc((size_t)o2v2);                // [d][f][l][e] = v~^{lf}_{de}
  double* VeT = ws.alloc((size_t)o2v2);                // [l][f][d][e] = v~^{lf}_{de}
  double* vvT = ws.alloc((size_t)o2v2);                // [j][k][c][b] = v~^{jk}_{bc}
  if (!VbT || !VcT || !VdT || !VeT || !vvT) { ctx->err = "workspace exhausted (feedback slices)"; return CCT_ENOMEM; }
  STCK(accumulate(s, 1.0, Vv(ctx, "vovv"), "bfcd", 0.0, dense(VbT, {v, o, v, v}), "bfcd"));
  STCK(accumulate(s, 1.0, Vv(ctx, "ooov"), "kfjc", 0.0, dense(VcT, {o, o, o, v}), "jfkc"));
  STCK(accumulate(s, 1.0, Vv(ctx, "oovv"), "lfde", 0.0, dense(VdT, {v, o, o, v}), "dfle"));
  STCK(accumulate(s, 1.0, Vv(ctx, "oovv"), "lfde", 0.0, dense(VeT, {o, o, v, v}), "lfde"));
  STCK(accumulate(s, 1.0, Vv(ctx, "oovv"), "jkbc", 0.0, dense(vvT, {o, o, v, v}), "jkcb"));
  // VbT[b][f][b][q] += 1/2 f~^f_{v_q}
  HIPCK(add_diag_rows(VbT, ctx->ft + o, v, o, v, (long long)o * v2, v2, v, 1, n, 0.5, s));
  for (const Batch& b : ctx->feed1.batches) {
    const size_t mk = ws.mark();
    const int S = b.nslots, f0 = b.slot0;
    const long long slab = (long long)S * o2v3;
    double* UA = ws.alloc((size_t)slab);
    double* UB = ws.alloc((size_t)slab);
    if (!UA || !UB) { ctx->err = "workspace exhausted (feedback)"; return CCT_ENOMEM; }
    const int occ[3] = {0, 2, 3};  // t~_{f, free0, free1}, gathered once, written in two layouts
    {
      UnpackArgs ua{};
      ua.o = o; ua.v = v; ua.nslots = S; ua.nfree = 2;
      set_s1(ua, occ);
      const long long row = (long long)S * v2;  // UA: one (i,j,a) row
      ua.s_slot = v2; ua.s_free[0] = (long long)o * v * row; ua.s_free[1] = v * row;
      ua.s_x = 1; ua.s_y = row; ua.s_z = v; ua.fast = 2;  // (x,y,z) = (q,a,p)
      const long long rowb = (long long)S * ov;  // UB: one (i,a,b) row
      ua.s2_slot = ov; ua.s2_free[0] = v2 * rowb; ua.s2_free[1] = v;
      ua.s2_x = 1; ua.s2_y = v * rowb; ua.s2_z = rowb; ua.fast2 = 2;  // (x,y,z) = (c,a,b)
      HIPCK(unpack_t3_dual(ctx->t3, ctx->tbl, b.d_slots, OutSpec{UA, OUT_F64, 0}, OutSpec{UB, OUT_F64, 0}, ua, s));
    }
    const long long KA = (long long)S * v2, KB = (long long)S * ov;
    // X2[(i,j,a)][b] += UA[(i,j,a)][K] VbT[b][f0.. K].  With v^2 a multiple of
    // 16 the product is batched over the S slots (K = v^2 each, one partial
    // per slot, then summed into X2): N = v is a single tile column, so one
    // product over the whole K would give too few tiles to fill the chip.
    double* Xp = (v2 % 16 == 0 && S > 1) ? ws.alloc((size_t)(S * o2v2)) : nullptr;
    if (Xp) {
      NtArgs g{};
      g.M = (int)((long long)o * o * v); g.N = v; g.K = (int)v2; g.batch = S;
      g.A = UA; g.lda = KA; g.a_batch = v2;
      g.B = VbT + (long long)f0 * v2; g.ldb = (long long)o * v2; g.b_batch = v2;
      g.C = Xp; g.cm = idx1(v); g.cn = idx1(1); g.c_batch = o2v2;
      g.alpha = 1.0; g.beta = 0.0;
      g.a_len = slab; g.b_len = (long long)o * v3 - (long long)f0 * v2; g.c_len = S * o2v2;
      HIPCK(gemm_nt(g, Prec::F64, s));
      for (int k = 0; k < S; ++k) HIPCK(axpby(1.0, Xp + (long long)k * o2v2, 1.0, ctx->X2, o2v2, s));
    } else {
      RCK(nt_or_generic(ctx, (int)((long long)o * o * v), v, KA, UA, KA, slab, VbT + (long long)f0 * v2,
                        (long long)o * v2, (long long)o * v3 - (long long)f0 * v2, ctx->X2, idx1(v), idx1(1), o2v2,
                        1.0, 1.0));
    }
    // W^{al}_{ij}: C[l][(i,j,a)] = VeT[l][f0.. K] UA[(i,j,a)][K], stored [a][l][i][j]
    RCK(nt_or_generic(ctx, o, (int)((long long)o * o * v), KA, VeT + (long long)f0 * v2, (long long)o * v2,
                      o2v2 - (long long)f0 * v2, UA, KA, slab, ctx->Wvooo, idx1((long long)o * o),
                      idx2(v, 1, (long long)o * o * o), (long long)v * o * o * o, 1.0, 1.0));
    // X2[(i,a,b)][j] -= UB[(i,a,b)][K] VcT[j][f0.. K]
    RCK(nt_or_generic(ctx, (int)(o * v2), o, KB, UB, KB, slab, VcT + (long long)f0 * ov, (long long)o * ov,
                      (long long)o * o * ov - (long long)f0 * ov, ctx->X2, idx2((int)v2, (long long)o * v2, 1),
                      idx1(v2), o2v2, -1.0, 1.0));
    // W^{ab}_{dj}: C[d][(j,b,a)] -= VdT[d][f0.. K] UB[(j,b,a)][K], stored [d][j][b][a]
    RCK(nt_or_generic(ctx, v, (int)(o * v2), KB, VdT + (long long)f0 * ov, (long long)o * ov,
                      o2v2 - (long long)f0 * ov, UB, KB, slab, ctx->Wt, idx1((long long)o * v2), idx1(1),
                      (long long)v * o * v2, -1.0, 1.0));
    HIPCK(feedback_r1(UA, vvT, ctx->r1, o, v, S, f0, s));
    ws.reset(mk);
  }
  ws.reset(mk0);
  return CCT_OK;
}

// Low-precision operand storage: FP32 values, or split BF16 as two planes
// (hi, lo); both take four bytes per element.
int lp_fmt(Prec p) { return p == Prec::F32 ? OUT_F32 : OUT_BF16X2; }
void* alloc_lp(Arena& ws, long long n) { return ws.alloc((size_t)((n + 1) / 2)); }
// Operands of the split ladder and the rings (K = the contracted length):
// split-BF16 rows with K >= lp_block_k (a context option, 1024 by default)
// are stored by blocks of 32 and padded to 32, so that hi and lo of 32 values
// share one 128-byte line and each K tile of the GEMM reads whole lines;
// shorter ones as two planes padded to 8; FP32 rows padded to 32 and FP64
// rows to 16 (one K tile of those kernels, which then copy whole tiles).
bool lp_blocked(const cct_ctx* ctx, long long K) { return ctx->prec == Prec::BF16X3 && K >= ctx->lp_block_k; }
int lp_fmt_gemm(const cct_ctx* ctx, long long K) {
  const Prec p = ctx->prec;
  return p == Prec::F64 ? OUT_F64 : (p == Prec::F32 ? OUT_F32 : (lp_blocked(ctx, K) ? OUT_BF16X2I : OUT_BF16X2));
}
long long lp_kpad(const cct_ctx* ctx, long long K) {
  const Prec p = ctx->prec;
  return p == Prec::F64 ? 16 : (p == Prec::F32 ? 32 : (lp_blocked(ctx, K) ? 32 : 8));
}

// Ladder with operands stored in the working precision: W converted once,
// then per chunk of blocks the three K-contiguous views of T3 (plain,
// axes 0/1 swapped, (d,e) rotated to the back) are written in that precision
// and multiplied by the low-precision K-contiguous kernel (FP64 output).
int r3_pp_lp(cct_ctx* ctx, const Idx2 cm[3], const Idx2 cn[3]) {
  const int v = ctx->v;
  const long long v2 = (long long)v * v, v3 = ctx->v3, v4 = v2 * v2, nt = ctx->ntri;
  const int fmt = lp_fmt(ctx->prec);
  Arena& ws = ctx->ws;
  const size_t mk = ws.mark();
  void* Wl = alloc_lp(ws, v4);
  if (!Wl) { ctx->err = "workspace exhausted (ladder W)"; return CCT_ENOMEM; }
  HIPCK(convert(ctx->Wvvvv, OutSpec{Wl, fmt, v4}, v4, ctx->s));
  long long chunk = (long long)(ws.available() / 4 / (size_t)v3) - 1;
  if (chunk < 1) { ctx->err = "workspace exhausted (ladder copy)"; return CCT_ENOMEM; }
  if (chunk > nt) chunk = nt;
  ctx->lad_chunks = (nt + chunk - 1) / chunk;
  void* Tc = alloc_lp(ws, chunk * v3);
  if (!Tc) { ctx->err = "workspace exhausted (ladder copy)"; return CCT_ENOMEM; }
  for (long long t0 = 0; t0 < nt; t0 += chunk) {
    const long long nb = std::min(chunk, nt - t0);
    const double* src = ctx->t3 + t0 * v3;
    const OutSpec os{Tc, fmt, nb * v3};
    for (int term = 2; term >= 0; --term) {
      if (term == 2) HIPCK(convert(src, os, nb * v3, ctx->s));
      else if (term == 1) HIPCK(swap01_batched(src, os, nb, v, v, v, ctx->s));
      else HIPCK(transpose_batched(src, os, nb, (int)v2, v, ctx->s));
      NtLpArgs g{};
      g.M = (int)(nb * v); g.N = (int)v2; g.K = (int)v2; g.batch = 1;
      g.A = Tc; g.lda = v2; g.a_plane = nb * v3;
      g.B = Wl; g.ldb = v2; g.b_plane = v4;
      g.C = ctx->r3 + t0 * v3; g.cm = cm[term]; g.cn = cn[term];
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = nb * v3; g.b_len = v4; g.c_len = (nt - t0) * v3;
      g.variant = ctx->tune_ladder;
      lad_begin(ctx);
      HIPCK(gemm_nt_lp(g, ctx->prec, ctx->s));
      lad_end(ctx, (double)nb * v * v2 * v2, 1);
    }
  }
  ws.reset(mk);
  return CCT_OK;
}

// Ladder with each relabelled term split into symmetric and antisymmetric
// parts (the further factor-of-two reduction the paper points to in its
// section on contractions without unpacking, after Scuseria et al.): with
// W^{yz}_{de} = W^{zy}_{ed},
//   C^{yz} + C^{zy} = sum_{d<=e} (A^{de} + A^{ed}) (W^{yz}_{de} + W^{yz}_{ed}) [d=e: A 2x, W 1x]
//   C^{yz} - C^{zy} = sum_{d<e}  (A^{de} - A^{ed}) (W^{yz}_{de} - W^{yz}_{ed})
// for the output pairs y <= z only, so each term is two GEMMs of half the
// size in K and in N: half the multiply-adds of the direct traversal.  The
// split operands are written in the working precision, K padded with zeros to
// the vector width; products are FP64; a combine kernel rebuilds C^{yz} and
// C^{zy} and adds them into R3 through the term's relabelling.
long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }

int r3_pp_split(cct_ctx* ctx) {
  const int v = ctx->v;
  const long long v2 = (long long)v * v, v3 = ctx->v3, nt = ctx->ntri;
  const long long P = (long long)v * (v + 1) / 2, Q = (long long)v * (v - 1) / 2;
  const bool f64 = ctx->prec == Prec::F64;
  // one format for both products (it follows the longer K)
  const long long w = lp_kpad(ctx, P);
  const long long pp = round_up(P, w), pq = round_up(std::max<long long>(Q, 1), w);
  const int fmt = lp_fmt_gemm(ctx, P);
  const long long esz = f64 ? 8 : 4;  // bytes per stored operand element (hi+lo BF16: 2 x 2)
  Arena& ws = ctx->ws;
  const size_t mk0 = ws.mark();
  auto alloc_b = [&](long long bytes) { return (void*)ws.alloc((size_t)((bytes + 7) / 8)); };
  void* Wp = alloc_b(P * pp * esz);
  void* Wm = alloc_b(P * pq * esz);
  if (!Wp || !Wm) { ctx->err = "workspace exhausted (ladder split W)"; return CCT_ENOMEM; }
  // W+ / W- rows y <= z from W[(y,z)][(d,e)]; W+ keeps W^{yz}_{dd} once
  HIPCK(pair_split(ctx->Wvvvv, idx1(0), ctx->vpair_src, P, v, v, OutSpec{Wp, fmt, P * pp}, pp,
                   OutSpec{Wm, fmt, P * pq}, pq, 0.5, ctx->s));
  // products: FP32 in the split-BF16 mode (exact for its FP32 accumulation), else FP64
  const bool z32 = ctx->prec == Prec::BF16X3;
  const long long csz = z32 ? 4 : 8;
  // chunk of packed blocks: A+/A- (esz), C+/C- (csz), FP64 relabelled copy for term 0
  const long long per_block = v * (pp + pq) * esz + 2 * v * P * csz + v3 * 8;
  long long chunk = (long long)(ws.available() / (size_t)per_block) - 1;
  if (chunk < 1) { ctx->err = "workspace exhausted (ladder split)"; return CCT_ENOMEM; }
  if (chunk > nt) chunk = nt;
  ctx->lad_chunks = (nt + chunk - 1) / chunk;
  void* Ap = alloc_b(chunk * v * pp * esz);
  void* Am = alloc_b(chunk * v * pq * esz);
  void* Cp = alloc_b(chunk * v * P * csz);
  void* Cm = alloc_b(chunk * v * P * csz);
  double* Tc = ws.alloc((size_t)(chunk * v3));
  if (!Ap || !Am || !Cp || !Cm || !Tc) { ctx->err = "workspace exhausted (ladder split)"; return CCT_ENOMEM; }
  auto gemm_pair = [&](int M, int N, long long K, const void* A, long long lda, long long a_len, long long a_plane,
                       const void* B, long long ldb, long long b_len, long long b_plane, void* C, long long c_len,
                       Idx2 cm) -> int {
    if (f64) {
      NtArgs g{};
      g.M = M; g.N = N; g.K = (int)K; g.batch = 1;
      g.A = (const double*)A; g.lda = lda; g.B = (const double*)B; g.ldb = ldb;
      g.C = (double*)C; g.cm = cm; g.cn = idx1(1); g.alpha = 1.0; g.beta = 0.0;
      g.a_len = a_len; g.b_len = b_len; g.c_len = c_len; g.variant = ctx->tune_ladder;
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
    } else {
      NtLpArgs g{};
      g.M = M; g.N = N; g.K = (int)K; g.batch = 1;
      g.A = A; g.lda = lda; g.a_plane = a_plane; g.B = B; g.ldb = ldb; g.b_plane = b_plane;
      if (z32) g.C32 = (float*)C;
      else g.C = (double*)C;
      g.cm = cm; g.cn = idx1(1); g.alpha = 1.0; g.beta = 0.0;
      g.a_len = a_len; g.b_len = b_len; g.c_len = c_len; g.variant = ctx->tune_ladder;
      g.il = fmt == OUT_BF16X2I;
      HIPCK(gemm_nt_lp(g, ctx->prec, ctx->s));
    }
    return CCT_OK;
  };
  for (long long t0 = 0; t0 < nt; t0 += chunk) {
    const long long nb = std::min(chunk, nt - t0), rows = nb * v;
    const double* src = ctx->t3 + t0 * v3;
    double* Rc = ctx->r3 + t0 * v3;
    const OutSpec ap{Ap, fmt, rows * pp}, am{Am, fmt, rows * pq};
    for (int term = 2; term >= 0; --term) {
      // A^{de} rows (t,x): term 2 T[t][x][d][e]; term 1 T[t][d][x][e]; term 0 T[t][d][e][x] via a copy
      if (term == 2) HIPCK(pair_split(src, idx2(v, v3, v2), nullptr, rows, v, v, ap, pp, am, pq, 1.0, ctx->s));
      else if (term == 1) HIPCK(pair_split(src, idx2(v, v3, v), nullptr, rows, v2, v, ap, pp, am, pq, 1.0, ctx->s));
      else {
        HIPCK(transpose_batched(src, OutSpec{Tc, OUT_F64, 0}, nb, (int)v2, v, ctx->s));  // [t][x][(d,e)]
        HIPCK(pair_split(Tc, idx2(v, v3, v2), nullptr, rows, v, v, ap, pp, am, pq, 1.0, ctx->s));
      }
      lad_begin(ctx);
      if (term > 0) {
        // C+-[(t,x)][p] = A+-[(t,x)][k] W+-[p][k]
        RCK(gemm_pair((int)rows, (int)P, pp, Ap, pp, rows * pp, rows * pp, Wp, pp, P * pp, P * pp, Cp, rows * P,
                      idx1(P)));
        RCK(gemm_pair((int)rows, (int)P, pq, Am, pq, rows * pq, rows * pq, Wm, pq, P * pq, P * pq, Cm, rows * P,
                      idx1(P)));
        lad_end(ctx, (double)rows * P * (P + Q), 2);
        const Idx2 cmap = term == 2 ? idx2(v, v3, v2) : idx2(v, v3, v);
        const long long sy = term == 2 ? v : v2;
        if (z32) HIPCK(pair_combine_rows((const float*)Cp, (const float*)Cm, P, P, rows, v, Rc, cmap, sy, 1, ctx->s));
        else HIPCK(pair_combine_rows((const double*)Cp, (const double*)Cm, P, P, rows, v, Rc, cmap, sy, 1, ctx->s));
      } else {
        // transposed products C+-T[p][(t,x)] so that the output runs along x
        RCK(gemm_pair((int)P, (int)rows, pp, Wp, pp, P * pp, P * pp, Ap, pp, rows * pp, rows * pp, Cp, rows * P,
                      idx1(rows)));
        RCK(gemm_pair((int)P, (int)rows, pq, Wm, pq, P * pq, P * pq, Am, pq, rows * pq, rows * pq, Cm, rows * P,
                      idx1(rows)));
        lad_end(ctx, (double)rows * P * (P + Q), 2);
        if (z32)
          HIPCK(pair_combine_cols((const float*)Cp, (const float*)Cm, rows, ctx->vpair_yz, v, Rc, idx2(v, v3, 1), v2, v,
                                  ctx->s));
        else
          HIPCK(pair_combine_cols((const double*)Cp, (const double*)Cm, rows, ctx->vpair_yz, v, Rc, idx2(v, v3, 1), v2,
                                  v, ctx->s));
      }
    }
  }
  ws.reset(mk0);
  return CCT_OK;
}

// Particle-particle ladder by direct traversal of the stored blocks (paper,
// Sec. "RCCSDT contractions without unpacking"): for each stored (i,j,k)
//   R[abc] += sum_de W^{ab}_{de} t^{dec} + W^{ac}_{de} t^{dbe} + W^{bc}_{de} t^{ade},
// i.e. three GEMMs over all blocks at once with M = (block, free virtual),
// N = (two output virtuals), K = (d,e), W shared.  In FP64 each term reads a
// K-contiguous copy of T3 (term 3 reads T3 itself; terms 2 and 1 a copy with
// the block axes swapped or rotated) through the NT matrix-core kernel.
int r3_pp(cct_ctx* ctx) {
  const int v = ctx->v;
  const long long v2 = (long long)v * v, v3 = ctx->v3, nt = ctx->ntri;
  const int M = (int)(nt * v);
  // output maps of the three terms: C[(t,x)][(y,z)] -> R[t][..]
  const Idx2 cm[3] = {idx2(v, v3, 1), idx2(v, v3, v), idx2(v, v3, v2)};
  const Idx2 cn[3] = {idx1(v), idx2(v, v2, 1), idx1(1)};
  if (ctx->ladder_split && v >= 2) return r3_pp_split(ctx);
  if (ctx->prec != Prec::F64) return r3_pp_lp(ctx, cm, cn);
  if (v2 & 1) {
    // generic strided kernel reading T3 in place
    const Idx2 am[3] = {idx2(v, v3, 1), idx2(v, v3, v), idx2(v, v3, v2)};
    const Idx2 ak[3] = {idx1(v), idx2(v, v2, 1), idx1(1)};
    for (int term = 0; term < 3; ++term) {
      GemmArgs g{};
      g.M = M; g.N = (int)v2; g.K = (int)v2; g.batch = 1;
      g.A = ctx->t3; g.am = am[term]; g.ak = ak[term];
      g.B = ctx->Wvvvv; g.bk = idx1(1); g.bn = idx1(v2);
      g.C = ctx->r3; g.cm = cm[term]; g.cn = cn[term];
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = nt * v3; g.b_len = v2 * v2; g.c_len = nt * v3;
      HIPCK(gemm(g, Prec::F64, ctx->s));
    }
    return CCT_OK;
  }
  // term 3 straight from T3 ([t][x][(d,e)] is already K-contiguous)
  {
    NtArgs g{};
    g.M = M; g.N = (int)v2; g.K = (int)v2; g.batch = 1;
    g.A = ctx->t3; g.lda = v2;
    g.B = ctx->Wvvvv; g.ldb = v2;
    g.C = ctx->r3; g.cm = idx1(v2); g.cn = idx1(1);
    g.alpha = 1.0; g.beta = 1.0;
    g.a_len = nt * v3; g.b_len = v2 * v2; g.c_len = nt * v3;
    g.variant = ctx->tune_ladder;
    lad_begin(ctx);
    HIPCK(gemm_nt(g, Prec::F64, ctx->s));
    lad_end(ctx, (double)M * v2 * v2, 1);
  }
  // terms 2 and 1 from relabelled copies, in chunks of blocks that fit the workspace
  Arena& ws = ctx->ws;
  const size_t mk = ws.mark();
  long long chunk = (long long)(ws.available() / sizeof(double) / (size_t)v3) - 1;
  if (chunk < 1) { ctx->err = "workspace exhausted (ladder copy)"; return CCT_ENOMEM; }
  if (chunk > nt) chunk = nt;
  ctx->lad_chunks = (nt + chunk - 1) / chunk;
  double* Tc = ws.alloc((size_t)(chunk * v3));
  if (!Tc) { ctx->err = "workspace exhausted (ladder copy)"; return CCT_ENOMEM; }
  for (int term = 1; term >= 0; --term) {
    for (long long t0 = 0; t0 < nt; t0 += chunk) {
      const long long nb = std::min(chunk, nt - t0);
      const double* src = ctx->t3 + t0 * v3;
      const OutSpec os{Tc, OUT_F64, 0};
      if (term == 1) HIPCK(swap01_batched(src, os, nb, v, v, v, ctx->s));  // [t][x][d][e] = T[t][d][x][e]
      else HIPCK(transpose_batched(src, os, nb, (int)v2, v, ctx->s));      // [t][x][(d,e)] = T[t][(d,e)][x]
      NtArgs g{};
      g.M = (int)(nb * v); g.N = (int)v2; g.K = (int)v2; g.batch = 1;
      g.A = Tc; g.lda = v2;
      g.B = ctx->Wvvvv; g.ldb = v2;
      g.C = ctx->r3 + t0 * v3; g.cm = cm[term]; g.cn = cn[term];
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = nb * v3; g.b_len = v2 * v2; g.c_len = (nt - t0) * v3;
      g.variant = ctx->tune_ladder;
      lad_begin(ctx);
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
      lad_end(ctx, (double)nb * v * v2 * v2, 1);
    }
  }
  ws.reset(mk);
  return CCT_OK;
}

int r3_f1(cct_ctx* ctx) {
  // sum_d F^a_d t^{dbc} + F^b_d t^{adc} + F^c_d t^{abd}, one GEMM per axis, batched over blocks
  const int v = ctx->v;
  const long long v2 = (long long)v * v, v3 = ctx->v3, nt3 = ctx->ntri * v3;
  const int nt = (int)ctx->ntri;
  if (!(v & 1)) {
    // matrix-core kernel: axis 0 reads the block as [K][N], axis 2 as [M][K]
    for (int start = 0; start < nt; start += 65535) {
      const int nb = std::min(65535, nt - start);
      const long long off = (long long)start * v3;
      NtArgs g{};
      g.M = v; g.N = (int)v2; g.K = v; g.batch = nb;  // C[a][(b,c)] += F[a][d] T[d][(b,c)]
      g.A = ctx->Fvv; g.lda = v; g.a_batch = 0;
      g.B = ctx->t3 + off; g.ldb = v2; g.b_batch = v3; g.b_kn = 1;
      g.C = ctx->r3 + off; g.cm = idx1(v2); g.cn = idx1(1); g.c_batch = v3;
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = v2; g.b_len = nt3 - off; g.c_len = nt3 - off;
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
      NtArgs h{};
      h.M = (int)v2; h.N = v; h.K = v; h.batch = nb;  // C[(a,b)][c] += T[(a,b)][d] F[c][d]
      h.A = ctx->t3 + off; h.lda = v; h.a_batch = v3;
      h.B = ctx->Fvv; h.ldb = v; h.b_batch = 0;
      h.C = ctx->r3 + off; h.cm = idx1(v); h.cn = idx1(1); h.c_batch = v3;
      h.alpha = 1.0; h.beta = 1.0;
      h.a_len = nt3 - off; h.b_len = v2; h.c_len = nt3 - off;
      HIPCK(gemm_nt(h, Prec::F64, ctx->s));
    }
    // axis 1: C[b][(a,c)] += F[b][d] T[a][d][c], the block read as [K][N]
    // rows d (stride v) whose columns (a,c) sit at a v^2 + c
    for (int start = 0; start < nt; start += 65535) {
      const int nb = std::min(65535, nt - start);
      const long long off = (long long)start * v3;
      NtArgs g{};
      g.M = v; g.N = (int)v2; g.K = v; g.batch = nb;
      g.A = ctx->Fvv; g.lda = v; g.a_batch = 0;
      g.B = ctx->t3 + off; g.ldb = v; g.b_batch = v3; g.b_kn = 1; g.b_map = 1; g.bnm = idx2(v, v2, 1);
      g.C = ctx->r3 + off; g.cm = idx1(v); g.cn = idx2(v, v2, 1); g.c_batch = v3;
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = v2; g.b_len = nt3 - off; g.c_len = nt3 - off;
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
    }
    return CCT_OK;
  }
  for (int start = 0; start < nt; start += 65535) {
    const int nb = std::min(65535, nt - start);
    const long long off = (long long)start * v3;
    for (int axis = 0; axis < 3; ++axis) {
      GemmArgs g{};
      g.M = v; g.K = v; g.N = (int)v2; g.batch = nb;
      g.A = ctx->Fvv; g.am = idx1(v); g.ak = idx1(1); g.a_batch = 0;
      g.B = ctx->t3 + off; g.b_batch = v3;
      g.C = ctx->r3 + off; g.c_batch = v3;
      if (axis == 0) { g.bk = idx1(v2); g.bn = idx1(1); g.cm = idx1(v2); g.cn = idx1(1); }
      if (axis == 1) { g.bk = idx1(v); g.bn = idx2(v, v2, 1); g.cm = idx1(v); g.cn = idx2(v, v2, 1); }
      if (axis == 2) { g.bk = idx1(1); g.bn = idx1(v); g.cm = idx1(1); g.cn = idx1(v); }
      g.alpha = 1.0; g.beta = 1.0;
      g.a_len = v2; g.b_len = nt3 - off; g.c_len = nt3 - off;
      HIPCK(gemm(g, Prec::F64, ctx->s));
    }
  }
  return CCT_OK;
}

// Rings (paper, Sec. "RCCSDT contractions with unpacking" and the compact
// ring expansions of the operation-count table).  For a batch of occupied
// pairs (q,r) the unpacked, spin-combined operand U[(q,r)][(y,z)][(l,d)] is
// built once; one batched GEMM gives Z[(q,r)][(p,x)][(y,z)] =
// sum_(l,d) Wbar[(p,x)][(l,d)] U[(q,r)][(y,z)][(l,d)] for every p, and an
// output-stationary fold adds each Z block into the packed R3 blocks it
// belongs to with the right virtual permutation and coefficient.
int r3_rings(cct_ctx* ctx, int kind) {
  const int o = ctx->o, v = ctx->v;
  const long long v2 = (long long)v * v;
  const long long ov = (long long)o * v;
  Arena& ws = ctx->ws;
  const bool lp = ctx->prec != Prec::F64;
  // K = (l,d) padded with zeros to the vector width of the working precision,
  // so that every shape runs on the K-contiguous kernels
  const long long kp = round_up(ov, lp_kpad(ctx, ov));
  const int fmt = lp_fmt_gemm(ctx, ov);
  // A[(p,x)][(l,d)] = Wbar^{lx}_{dp} (ring A) or Wbar^{lx}_{pd} (rings B, C), row-major [p][x][l][d]
  const double* Aw = kind == 0 ? ctx->Wb1 : ctx->Wb2;
  const size_t mk0 = ws.mark();
  void* Ap = lp ? alloc_lp(ws, ov * kp) : (void*)ws.alloc((size_t)(ov * kp));
  if (!Ap) { ctx->err = "workspace exhausted (rings)"; return CCT_ENOMEM; }
  HIPCK(copy_pad_rows(Aw, ov, ov, OutSpec{Ap, fmt, ov * kp}, kp, ctx->s));
  for (const Batch& b : ctx->ring[kind].batches) {
    const size_t mk = ws.mark();
    const long long ulen = b.nslots * v2 * kp;
    void* U = lp ? alloc_lp(ws, ulen) : (void*)ws.alloc((size_t)ulen);
    // contracted blocks: FP32 in the split-BF16 mode (its accumulation is
    // FP32, so nothing is lost), FP64 otherwise
    const bool z32 = ctx->prec == Prec::BF16X3;
    const long long zlen = b.nslots * ov * v2;
    void* Z = z32 ? alloc_lp(ws, zlen) : (void*)ws.alloc((size_t)zlen);
    if (!U || !Z) { ctx->err = "workspace exhausted (rings)"; return CCT_ENOMEM; }
    const OutSpec uo{U, fmt, ulen};
    if (kp != ov) HIPCK(zero_cols(uo, b.nslots * v2, kp, ov, ctx->s));
    UnpackArgs ua{};
    ua.o = o; ua.v = v; ua.nslots = b.nslots; ua.nfree = 1;
    // U[s][(y,z)][(l,d)] (rows of kp): (x, y, z) of the unpack are (d, y, z); d runs fastest
    ua.s_slot = v2 * kp; ua.s_free[0] = v; ua.s_free[1] = 0;
    ua.s_x = 1; ua.s_y = kp * v; ua.s_z = kp; ua.fast = 2;
    if (kind == 0) {
      const int occ[3] = {2, 0, 1};  // S1 t~_{l q r}^{d y z}
      set_s1(ua, occ);
    } else if (kind == 1) {
      ua.nterms = 2;  // t_{q l r}^{d y z} + t_{r l q}^{d z y}
      ua.terms[0] = UnpackTerm{1.0, {0, 2, 1}, {0, 1, 2}};
      ua.terms[1] = UnpackTerm{1.0, {1, 2, 0}, {0, 2, 1}};
    } else {
      const int occ[3] = {0, 2, 1};  // t_{q l r}^{d x z}
      set_ident(ua, occ);
    }
    HIPCK(unpack_t3_fmt(ctx->t3, ctx->tbl, b.d_slots, uo, ua, ctx->s));
    // Z[s][(p,x)][(y,z)] = sum_(l,d) A[(p,x)][(l,d)] U[s][(y,z)][(l,d)]
    if (lp) {
      NtLpArgs g{};
      g.M = (int)ov; g.N = (int)v2; g.K = (int)kp; g.batch = b.nslots;
      g.A = Ap; g.lda = kp; g.a_batch = 0; g.a_plane = ov * kp;
      g.B = U; g.ldb = kp; g.b_batch = v2 * kp; g.b_plane = ulen;
      if (z32) g.C32 = (float*)Z;
      else g.C = (double*)Z;
      g.cm = idx1(v2); g.cn = idx1(1); g.c_batch = ov * v2;
      g.alpha = 1.0; g.beta = 0.0;
      g.a_len = ov * kp; g.b_len = ulen; g.c_len = zlen;
      g.variant = ctx->tune_rings;
      g.il = fmt == OUT_BF16X2I;
      HIPCK(gemm_nt_lp(g, ctx->prec, ctx->s));
    } else {
      NtArgs g{};
      g.M = (int)ov; g.N = (int)v2; g.K = (int)kp; g.batch = b.nslots;
      g.A = (const double*)Ap; g.lda = kp; g.a_batch = 0;
      g.B = (const double*)U; g.ldb = kp; g.b_batch = v2 * kp;
      g.C = (double*)Z; g.cm = idx1(v2); g.cn = idx1(1); g.c_batch = ov * v2;
      g.alpha = 1.0; g.beta = 0.0;
      g.a_len = ov * kp; g.b_len = ulen; g.c_len = zlen;
      g.variant = ctx->tune_rings;
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
    }
    if (z32) HIPCK(fold_r3(ctx->r3, ctx->v3, v, (const float*)Z, b.d_tasks, b.ntasks, b.d_contribs, ctx->s));
    else HIPCK(fold_r3(ctx->r3, ctx->v3, v, (const double*)Z, b.d_tasks, b.ntasks, b.d_contribs, ctx->s));
    ws.reset(mk);
  }
  ws.reset(mk0);
  return CCT_OK;
}

int r3_hh(cct_ctx* ctx, bool with_hh, bool with_f2) {
  const int o = ctx->o, v = ctx->v;
  const long long v3 = ctx->v3, o2v3 = (long long)o * o * v3, o4 = (long long)o * o * o * o;
  const long long o2 = (long long)o * o, npair = (long long)o * (o + 1) / 2;
  // Wh = W^{lm}_{pq} - 1/2 (delta_mq F^l_p + delta_lp F^m_q)
  if (with_hh) HIPCK(axpby(1.0, ctx->Woooo, 0.0, ctx->Wh, o4, ctx->s));
  else HIPCK(fill(ctx->Wh, 0.0, o4, ctx->s));
  if (with_f2) HIPCK(add_pair_diag(ctx->Wh, ctx->Foo, o, o, -0.5, ctx->s));
  Arena& ws = ctx->ws;
  const size_t mk0 = ws.mark();
  // A[pair(p<=q)][(l,m)] = Wh[(l,m)][(p,q)]: transpose, then keep the ordered pairs
  double* WhT = ws.alloc((size_t)o4);
  double* WhP = ws.alloc((size_t)(npair * o2));
  if (!WhT || !WhP) { ctx->err = "workspace exhausted (hole ladder)"; return CCT_ENOMEM; }
  HIPCK(transpose_batched(ctx->Wh, OutSpec{WhT, OUT_F64, 0}, 1, (int)o2, (int)o2, ctx->s));
  HIPCK(gather_rows(WhT, o2, ctx->pair_rows, (int)npair, o2, WhP, o2, ctx->s));
  const bool nt = !(o2 & 1) && !(v3 & 1);
  for (const Batch& b : ctx->hh.batches) {
    const size_t mk = ws.mark();
    double* U = ws.alloc((size_t)(b.nslots * o2v3));
    double* Z = ws.alloc((size_t)(b.nslots * npair * v3));
    if (!U || !Z) { ctx->err = "workspace exhausted (hole ladder)"; return CCT_ENOMEM; }
    UnpackArgs ua{};
    ua.o = o; ua.v = v; ua.nslots = b.nslots; ua.nfree = 2;
    const int occ[3] = {2, 3, 0};  // t_{l m r}^{xyz}
    set_ident(ua, occ);
    ua.s_slot = o2v3; ua.s_free[0] = (long long)o * v3; ua.s_free[1] = v3;
    ua.s_x = (long long)v * v; ua.s_y = v; ua.s_z = 1;
    HIPCK(unpack_t3(ctx->t3, ctx->tbl, b.d_slots, U, ua, ctx->s));
    // Z[r][pair][xyz] = sum_(l,m) WhP[pair][(l,m)] U[r][(l,m)][xyz]
    if (nt) {
      NtArgs g{};
      g.M = (int)npair; g.N = (int)v3; g.K = (int)o2; g.batch = b.nslots;
      g.A = WhP; g.lda = o2; g.a_batch = 0;
      g.B = U; g.ldb = v3; g.b_batch = o2v3; g.b_kn = 1;
      g.C = Z; g.cm = idx1(v3); g.cn = idx1(1); g.c_batch = npair * v3;
      g.alpha = 1.0; g.beta = 0.0;
      g.a_len = npair * o2; g.b_len = b.nslots * o2v3; g.c_len = b.nslots * npair * v3;
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
    } else {
      GemmArgs g{};
      g.M = (int)npair; g.N = (int)v3; g.K = (int)o2; g.batch = b.nslots;
      g.A = WhP; g.am = idx1(o2); g.ak = idx1(1); g.a_batch = 0;
      g.B = U; g.bk = idx1(v3); g.bn = idx1(1); g.b_batch = o2v3;
      g.C = Z; g.cm = idx1(v3); g.cn = idx1(1); g.c_batch = npair * v3;
      g.alpha = 1.0; g.beta = 0.0;
      g.a_len = npair * o2; g.b_len = b.nslots * o2v3; g.c_len = b.nslots * npair * v3;
      HIPCK(gemm(g, Prec::F64, ctx->s));
    }
    HIPCK(fold_r3(ctx->r3, v3, v, Z, b.d_tasks, b.ntasks, b.d_contribs, ctx->s));
    ws.reset(mk);
  }
  ws.reset(mk0);
  return CCT_OK;
}

int r3_drivers(cct_ctx* ctx, int which) {
  const int o = ctx->o, v = ctx->v;
  const long long v2 = (long long)v * v, v3 = ctx->v3, o2v3 = (long long)o * o * v3;
  Arena& ws = ctx->ws;
  const Job& J = which == 0 ? ctx->d1 : ctx->d2;
  const size_t mk0 = ws.mark();
  // K-contiguous copies for the matrix-core kernel (driver 1, even v):
  //   WtT[q][(x,y)][d] = W^{xy}_{dq},  t2T[(p,r,z)][d] = t_pr^dz
  const bool nt = which == 0 && !(v & 1);
  double *WtT = nullptr, *t2T = nullptr;
  if (nt) {
    WtT = ws.alloc((size_t)(o * v3));
    t2T = ws.alloc((size_t)o * o * v2);
    if (!WtT || !t2T) { ctx->err = "workspace exhausted (drivers)"; return CCT_ENOMEM; }
    STCK(accumulate(ctx->s, 1.0, dense(ctx->Wt, {v, o, v, v}), "dqyx", 0.0, dense(WtT, {o, v, v, v}), "qxyd"));
    STCK(accumulate(ctx->s, 1.0, dense(ctx->t2, {o, o, v, v}), "prdz", 0.0, dense(t2T, {o, o, v, v}), "przd"));
  }
  for (const Batch& b : J.batches) {
    const size_t mk = ws.mark();
    double* Z = ws.alloc((size_t)(b.nslots * o2v3));
    if (!Z) { ctx->err = "workspace exhausted (drivers)"; return CCT_ENOMEM; }
    if (nt) {
      // Z[q][(x,y)][(p,r,z)] = sum_d WtT[q][(x,y)][d] t2T[(p,r,z)][d]
      NtArgs g{};
      g.M = (int)v2; g.N = o * o * v; g.K = v; g.batch = b.nslots;
      g.A = WtT + (long long)b.slot0 * v3; g.lda = v; g.a_batch = v3;
      g.B = t2T; g.ldb = v; g.b_batch = 0;
      g.C = Z; g.cm = idx1((long long)o * o * v); g.cn = idx1(1); g.c_batch = o2v3;
      g.alpha = 1.0; g.beta = 0.0;
      g.a_len = (long long)(o - b.slot0) * v3; g.b_len = (long long)o * o * v2; g.c_len = b.nslots * o2v3;
      HIPCK(gemm_nt(g, Prec::F64, ctx->s));
      HIPCK(fold_r3(ctx->r3, v3, v, Z, b.d_tasks, b.ntasks, b.d_contribs, ctx->s));
      ws.reset(mk);
      continue;
    }
    GemmArgs g{};
    g.batch = b.nslots;
    if (which == 0) {
      // Z[q][(x,y)][(p,r,z)] = sum_d W^{xy}_{dq} t_pr^dz ; Wt[d][q][y][x]
      g.M = (int)v2; g.N = o * o * v; g.K = v;
      g.A = ctx->Wt + (long long)b.slot0 * v2; g.am = idx2(v, 1, v); g.ak = idx1((long long)o * v2); g.a_batch = v2;
      g.B = ctx->t2; g.bk = idx1(v); g.bn = idx2(v, v2, 1); g.b_batch = 0;
      g.C = Z; g.cm = idx1((long long)o * o * v); g.cn = idx1(1); g.c_batch = o2v3;
      g.a_len = v3 * o - (long long)b.slot0 * v2; g.b_len = (long long)o * o * v2;
    } else {
      // Z[r][(x,p,q)][(y,z)] = sum_l W^{xl}_{pq} t_lr^yz ; Wvooo[x][l][p][q]
      g.M = v * o * o; g.N = (int)v2; g.K = o;
      g.A = ctx->Wvooo; g.am = idx2(o * o, (long long)o * o * o, 1); g.ak = idx1((long long)o * o); g.a_batch = 0;
      g.B = ctx->t2 + (long long)b.slot0 * v2; g.bk = idx1((long long)o * v2); g.bn = idx1(1); g.b_batch = v2;
      g.C = Z; g.cm = idx1(v2); g.cn = idx1(1); g.c_batch = o2v3;
      g.a_len = (long long)v * o * o * o; g.b_len = (long long)o * o * v2 - (long long)b.slot0 * v2;
    }
    g.c_len = b.nslots * o2v3;
    g.alpha = 1.0; g.beta = 0.0;
    HIPCK(gemm(g, Prec::F64, ctx->s));
    HIPCK(fold_r3(ctx->r3, v3, v, Z, b.d_tasks, b.ntasks, b.d_contribs, ctx->s));
    ws.reset(mk);
  }
  ws.reset(mk0);
  return CCT_OK;
}

void count_macs(cct_ctx* ctx, unsigned mask) {
  const double t = (double)ctx->ntri, o = ctx->o, v = ctx->v;
  const double full[9] = {6 * t * v * v * v * v, 6 * t * o * v * v * v, 3 * t * v * v * v * v, 3 * t * o * v * v * v,
                          3 * t * o * v * v * v * v, 3 * t * o * v * v * v * v, 6 * t * o * v * v * v * v,
                          3 * t * o * o * v * v * v, 3 * t * v * v * v * v * v};
  for (int i = 0; i < 9; ++i) ctx->macs[i] = (mask & (1u << i)) ? full[i] : 0.0;
}

int finite_or_err(cct_ctx* ctx, double x) {
  if (!std::isfinite(x)) {
    ctx->err = "non-finite residual norm or energy";
    return CCT_ENUMERIC;
  }
  return CCT_OK;
}

// Full residual evaluation; R3 post-processed; optionally T3 += R3 / eps.
// Enqueue one residual evaluation (and, with update_t3, the T3 Jacobi step)
// on the context's stream.  No host synchronisation and no allocation: the
// squared norms are left in scal[0..2].  Safe to record into a HIP graph.
int enqueue_residual(cct_ctx* ctx, unsigned mask, bool update_t3) {
  if (!ctx->have_f || !ctx->have_B) {
    ctx->err = "integrals not set (cct_set_fock / cct_set_eri_df)";
    return CCT_ESTATE;
  }
  hipStream_t s = ctx->s;
  ctx->ws.reset(0);  // the arena holds only per-evaluation scratch; drop what a failed call left
  ctx->lad_nev = 0;
  ctx->lad_macs = ctx->lad_launches = ctx->lad_ms = 0.0;
  ctx->lad_chunks = 0;
  mark(ctx, 0);
  RCK(dress(ctx));
  RCK(ccsd_part(ctx));
  mark(ctx, 1);
  RCK(feedback(ctx));
  {
    DT X2 = dense(ctx->X2, {ctx->o, ctx->o, ctx->v, ctx->v});
    DT R2 = dense(ctx->r2, {ctx->o, ctx->o, ctx->v, ctx->v});
    STCK(accumulate(s, 1.0, X2, "ijab", 0.0, R2, "ijab"));
    STCK(accumulate(s, 1.0, X2, "jiba", 1.0, R2, "ijab"));
  }
  HIPCK(fill(ctx->r3, 0.0, ctx->ntri * ctx->v3, s));
  mark(ctx, 2);
  if (mask & CCT_TERM_PP) RCK(r3_pp(ctx));
  mark(ctx, 3);
  if (mask & CCT_TERM_RA) RCK(r3_rings(ctx, 0));
  if (mask & CCT_TERM_RB) RCK(r3_rings(ctx, 1));
  if (mask & CCT_TERM_RC) RCK(r3_rings(ctx, 2));
  mark(ctx, 4);
  if (mask & (CCT_TERM_HH | CCT_TERM_F2)) RCK(r3_hh(ctx, mask & CCT_TERM_HH, mask & CCT_TERM_F2));
  mark(ctx, 5);
  if (mask & CCT_TERM_D1) RCK(r3_drivers(ctx, 0));
  if (mask & CCT_TERM_D2) RCK(r3_drivers(ctx, 1));
  mark(ctx, 6);
  if (mask & CCT_TERM_F1) RCK(r3_f1(ctx));
  mark(ctx, 7);
  PostArgs pa{ctx->o, ctx->v, (int)ctx->ntri, ctx->v3, update_t3 ? 1 : 0, 1};
  int np = 0;
  const long long part_max = ctx->red_n - 1024;
  if (64LL * ctx->ntri > part_max) {
    ctx->err = "reduction scratch too small";
    return CCT_EDEVICE;
  }
  HIPCK(post_update(ctx->r3, ctx->t3, ctx->tri, ctx->eps, ctx->red + 1024, &np, pa, s));
  HIPCK(reduce_sum(ctx->red + 1024, np, ctx->scal + 2, ctx->red, s));
  HIPCK(dot(ctx->r1, ctx->r1, (long long)ctx->o * ctx->v, ctx->scal + 0, ctx->red, s));
  HIPCK(dot(ctx->r2, ctx->r2, (long long)ctx->o * ctx->o * ctx->v * ctx->v, ctx->scal + 1, ctx->red, s));
  mark(ctx, 8);
  count_macs(ctx, mask);
  return CCT_OK;
}

// Wait for an enqueued residual, read the squared norms back, check them.
int finish_residual(cct_ctx* ctx, double norms[3]) {
  double h[3];
  HIPCK(hipMemcpyAsync(h, ctx->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  if (ctx->events) {
    for (int i = 0; i < PH_DIIS; ++i) {
      float msv = 0.f;
      if (hipEventElapsedTime(&msv, ctx->ev[i], ctx->ev[i + 1]) == hipSuccess) ctx->ms[i] = msv;
    }
    for (int i = 0; i + 1 < ctx->lad_nev; i += 2) {
      float msv = 0.f;
      if (hipEventElapsedTime(&msv, ctx->lad_ev[i], ctx->lad_ev[i + 1]) == hipSuccess) ctx->lad_ms += msv;
    }
  }
  ctx->have_res = true;
  for (int i = 0; i < 3; ++i) {
    if (norms) norms[i] = h[i];
    RCK(finite_or_err(ctx, h[i]));
  }
  return CCT_OK;
}

int compute(cct_ctx* ctx, unsigned mask, bool update_t3, double norms[3]) {
  RCK(enqueue_residual(ctx, mask, update_t3));
  return finish_residual(ctx, norms);
}

// Energy of the current amplitudes into scal[6] (device; no synchronisation):
// E = sum (2 v^{ij}_{ab} - v^{ij}_{ba}) (t_ij^ab + t_i^a t_j^b) + 2 sum f_ia t_i^a.
// out (may be null) also receives the squared norms scal[0..2] and E.
int enqueue_energy(cct_ctx* ctx, double* out) {
  const int o = ctx->o, v = ctx->v;
  hipStream_t s = ctx->s;
  // tau = t2 + t1 t1
  DT tau = dense(ctx->tau_e, {o, o, v, v});
  DT t1 = dense(ctx->t1, {o, v});
  STCK(accumulate(s, 1.0, dense(ctx->t2, {o, o, v, v}), "ijab", 0.0, tau, "ijab"));
  STCK(contract(ctx->ws, s, Prec::F64, 1.0, t1, "ia", t1, "jb", 1.0, tau, "ijab"));
  HIPCK(dot(ctx->vbare_c, ctx->tau_e, (long long)o * o * v * v, ctx->scal + 4, ctx->red, s));
  HIPCK(dot(ctx->fov, ctx->t1, (long long)o * v, ctx->scal + 5, ctx->red, s));
  HIPCK(energy_scalars(ctx->scal, out, s));
  return CCT_OK;
}

int energy_dev(cct_ctx* ctx, double* e) {
  RCK(enqueue_energy(ctx, nullptr));
  HIPCK(hipMemcpyAsync(e, ctx->scal + 6, sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  return finite_or_err(ctx, *e);
}

// --- perturbative quadruples correction ----------------------------------
// E_(Q) of the (Q) appendix (Eq. ener-pt-q with Eq. resi-pt-q), by the
// occupied-tuple traversal of the "IJK-based algorithm" section: one task per
// i <= j <= k <= l (no three equal: those blocks of the spin-summed quadruples
// vanish).  With G = X + Y and A = X + V, the task accumulates
//   R[w]    = sum over the 24 column permutations s of G_{o.s}[w.s]
//   Abar[w] = sum over the distinct orderings q = o.s of A_q[w.s]
// and contributes <Abar, S(R) / eps_o>, S the full spin summation; since S
// commutes with column permutations and z = P(X + V), this equals the
// task's share of 1/24 sum z tchk.  The blocks X_q, Y_q of an ordered tuple q
// cost two dense contractions of 2 v^5 (X from T3, Y from the resident
// Wbar_ejk^abc) plus two of 2 o v^4; all orderings of a task stay resident
// and one permuted-combine pass writes R and Abar.
DT Vview(cct_ctx* c, double* base, const char* blk) {
  DT t = Vv(c, blk);
  t.p = base + (t.p - c->V);
  return t;
}

// Device buffers of one (Q) evaluation: from the caller's allocator or
// hipMalloc (returned when the evaluation ends), or carved from a fixed
// device region (base != nullptr: nothing is allocated; `used` counts the
// bytes asked for, also past `cap`, so that the caller can report the need
// before any device work has started).
struct QMem {
  cct_ctx* c;
  std::vector<void*> ps;
  char* base = nullptr;
  size_t cap = 0, used = 0;
  explicit QMem(cct_ctx* cc, char* region = nullptr, size_t region_bytes = 0)
      : c(cc), base(region), cap(region_bytes) {}
  ~QMem() {
    if (!ps.empty() || used) (void)hipStreamSynchronize(c->s);
    for (void* p : ps) dev_free(c, p);
  }
  bool fits() const { return used <= cap; }
  template <typename T>
  int get(T** p, long long n) {
    const size_t bytes = (size_t)std::max<long long>(n, 1) * sizeof(T);
    if (base) {
      const size_t at = (used + 255) & ~(size_t)255;
      used = at + bytes;
      *p = used <= cap ? (T*)(base + at) : nullptr;
      return CCT_OK;
    }
    void* q = nullptr;
    RCK(dev_alloc(c, &q, bytes));
    ps.push_back(q);
    *p = (T*)q;
    return CCT_OK;
  }
};

long long q_task_count(int o) { return (long long)o * (o + 1) * (o + 2) * (o + 3) / 24; }

// region / region_bytes: a fixed device region to take every buffer from
// (no allocation); nullptr: the context's allocator, or hipMalloc.
int energy_q(cct_ctx* ctx, double* e_q, double* e_tasks, long long cap, char* region = nullptr,
             size_t region_bytes = 0) {
  const int o = ctx->o, v = ctx->v, n = ctx->n;
  const long long naux = ctx->naux, n2 = (long long)n * n, n4 = n2 * n2;
  const long long v2 = (long long)v * v, v3 = v2 * v, v4 = v3 * v, o2 = (long long)o * o;
  const long long ntask = q_task_count(o);
  if (e_tasks && cap < ntask) {
    ctx->err = "energy_q: task array holds " + std::to_string(cap) + " entries, " + std::to_string(ntask) + " needed";
    return CCT_EINVAL;
  }
  if ((long long)o * o * o > 65535) { ctx->err = "energy_q: nocc above 40"; return CCT_EINVAL; }
  if (v3 > INT_MAX || o2 * o * v3 > LLONG_MAX / 8) { ctx->err = "energy_q: nvir too large"; return CCT_EINVAL; }
  hipStream_t s = ctx->s;
  const long long arena_n = std::max(v4, o2 * o2 * v2) + (8LL << 20);
  // even v with o <= 16: the K=o updates write tile-major copies of the task
  // blocks (XT, GT), which the permuted combine reads as contiguous tiles
  const bool tl = (v % 2) == 0 && o <= 16;
  const long long T4 = tiled_len(v);
  const long long need = n4 + v4 + (long long)o * v3 + o2 * o * v + o2 * v2 + o2 * v4 + 2 * o2 * o2 * v2 +
                         o2 * o * v3 + 50 * v4 + (tl ? 48 * T4 : 0) + ntask + 1 + arena_n;
  if (!ctx->alloc_fn && !region) {
    size_t fr = 0, tot = 0;
    HIPCK(hipMemGetInfo(&fr, &tot));
    if ((double)need * 8.0 + 256e6 > (double)fr) {
      ctx->err = "energy_q: needs " + std::to_string(need * 8.0 / 1e9) + " GB of device memory, " +
                 std::to_string(fr / 1e9) + " GB free";
      return CCT_ENOMEM;
    }
  }
  QMem mem(ctx, region, region_bytes);
  double *Vb, *VVVV, *VVVO, *VOOO, *VVOO, *Wv, *g, *Wo, *T3u, *Xb, *Gb, *Rb, *Ab, *et, *ar;
  int2* slots;
  RCK(mem.get(&Vb, n4));
  RCK(mem.get(&VVVV, v4));
  RCK(mem.get(&VVVO, (long long)o * v3));
  RCK(mem.get(&VOOO, o2 * o * v));
  RCK(mem.get(&VVOO, o2 * v2));
  RCK(mem.get(&Wv, o2 * v4));
  RCK(mem.get(&g, o2 * o2 * v2));
  RCK(mem.get(&Wo, o2 * o2 * v2));
  RCK(mem.get(&T3u, o2 * o * v3));
  RCK(mem.get(&Xb, (tl ? 1 : 24) * v4));  // X of each distinct ordering of a task (tiled path: one scratch block)
  RCK(mem.get(&Gb, 24 * v4));  // Y of each distinct ordering
  RCK(mem.get(&Rb, v4));
  RCK(mem.get(&Ab, v4));
  RCK(mem.get(&et, ntask + 1));
  RCK(mem.get(&ar, arena_n));
  RCK(mem.get(&slots, o2));
  double* Bc;
  RCK(mem.get(&Bc, 24 * v2));  // t2 blocks of the orderings sharing one Y1 product
  double *XT = nullptr, *GT = nullptr;
  if (tl) {
    RCK(mem.get(&XT, 24 * T4));
    RCK(mem.get(&GT, 24 * T4));
  }
  if (!mem.fits()) {  // nothing has been launched yet
    ctx->err = "energy_q: this system needs " + std::to_string(mem.used >> 20) + " MiB of device scratch, the " +
               "fixed scratch region holds " + std::to_string(mem.cap >> 20) + " MiB";
    return CCT_ENOMEM;
  }
  Arena qa;
  qa.init((char*)ar, (size_t)arena_n * 8);
  const Prec F = Prec::F64;

  // bare integrals v^{pq}_{rs} = (pr|qs), stored like the dressed ones
  {
    GemmArgs ga{};
    ga.M = (int)n2; ga.N = (int)n2; ga.K = (int)naux; ga.batch = 1;
    ga.A = ctx->B; ga.am = idx1(1); ga.ak = idx1(n2);
    ga.B = ctx->B; ga.bk = idx1(n2); ga.bn = idx1(1);
    ga.C = Vb; ga.cm = idx1(n2); ga.cn = idx1(1);
    ga.alpha = 1.0; ga.beta = 0.0;
    ga.a_len = naux * n2; ga.b_len = naux * n2; ga.c_len = n4;
    HIPCK(gemm(ga, F, s));
  }
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vvvv"), "abef", 0.0, dense(VVVV, {v, v, v, v}), "abef"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vvvo"), "abej", 0.0, dense(VVVO, {o, v, v, v}), "jabe"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vooo"), "amij", 0.0, dense(VOOO, {o, o, v, o}), "ijam"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vvoo"), "abij", 0.0, dense(VVOO, {o, o, v, v}), "ijab"));
  // Wbar_eqr^abc (Eq. q_w_vvv_voo) as Wv[q][r][a][b][c][e], one (q, r) at a time
  for (int q = 0; q < o; ++q)
    for (int r = 0; r < o; ++r) {
      const DT w = dense(Wv + ((long long)q * o + r) * v4, {v, v, v, v});
      STCK(contract(qa, s, F, 0.5, dense(VVVV, {v, v, v, v}), "abef", dense(ctx->t2 + ((long long)q * o + r) * v2, {v, v}),
                    "fc", 0.0, w, "abce"));
      STCK(contract(qa, s, F, 0.5, dense(VVVV, {v, v, v, v}), "acef", dense(ctx->t2 + ((long long)r * o + q) * v2, {v, v}),
                    "fb", 1.0, w, "abce"));
    }
  // Wbar_ijk^abm (Eq. q_w_vvo_ooo) as Wo[i][j][k][a][b][m]
  {
    const DT t2 = dense(ctx->t2, {o, o, v, v});
    const DT gd = dense(g, {o, o, o, v, v, o}), wd = dense(Wo, {o, o, o, v, v, o});
    STCK(contract(qa, s, F, 1.0, Vview(ctx, Vb, "ovvo"), "maei", t2, "jkbe", 0.0, gd, "ijkabm"));
    STCK(contract(qa, s, F, 1.0, Vview(ctx, Vb, "ovov"), "make", t2, "jibe", 1.0, gd, "ijkabm"));
    STCK(contract(qa, s, F, -0.5, Vview(ctx, Vb, "oooo"), "mnki", t2, "njab", 1.0, gd, "ijkabm"));
    STCK(accumulate(s, 1.0, gd, "ijkabm", 0.0, wd, "ijkabm"));
    STCK(accumulate(s, 1.0, gd, "jikbam", 1.0, wd, "ijkabm"));
  }
  // T3u[r][s][m] = t_{m r s}^{xyz} (full v^3 blocks) for every ordered (r, s)
  {
    std::vector<int2> sl((size_t)o2);
    for (int r = 0; r < o; ++r)
      for (int t = 0; t < o; ++t) sl[(size_t)r * o + t] = make_int2(r, t);
    HIPCK(hipMemcpyAsync(slots, sl.data(), sizeof(int2) * sl.size(), hipMemcpyHostToDevice, s));
    HIPCK(hipStreamSynchronize(s));
    UnpackArgs ua{};
    ua.o = o; ua.v = v; ua.nslots = (int)o2; ua.nfree = 1;
    ua.s_slot = (long long)o * v3; ua.s_free[0] = v3; ua.s_free[1] = 0;
    ua.s_x = v2; ua.s_y = v; ua.s_z = 1; ua.fast = 0;
    const int occ[3] = {2, 0, 1};
    set_ident(ua, occ);
    HIPCK(unpack_t3(ctx->t3, ctx->tbl, slots, T3u, ua, s));
  }
  HIPCK(fill(et, 0.0, ntask + 1, s));

  std::vector<double> eps((size_t)n);
  HIPCK(hipMemcpyAsync(eps.data(), ctx->eps, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  const bool nt_ok = (v % 2) == 0;  // K-contiguous MFMA kernel: even K and 16-byte aligned rows
  auto gemm_x1_y1 = [&](const double* A, long long lda, const double* Bm, long long ldb, double* C, long long M,
                        long long N, double alpha) -> int {
    // C[M][N] = alpha * sum_e A[m][e] B[e][n], K = v
    if (nt_ok) {
      NtArgs na{};
      na.M = (int)M; na.N = (int)N; na.K = v; na.batch = 1;
      na.A = A; na.lda = lda; na.B = Bm; na.ldb = ldb; na.b_kn = 1;
      na.C = C; na.cm = idx1(N); na.cn = idx1(1);
      na.alpha = alpha; na.beta = 0.0;
      na.a_len = M * lda; na.b_len = (long long)v * ldb; na.c_len = M * N;
      HIPCK(gemm_nt(na, F, s));
    } else {
      GemmArgs ga{};
      ga.M = (int)M; ga.N = (int)N; ga.K = v; ga.batch = 1;
      ga.A = A; ga.am = idx1(lda); ga.ak = idx1(1);
      ga.B = Bm; ga.bk = idx1(ldb); ga.bn = idx1(1);
      ga.C = C; ga.cm = idx1(N); ga.cn = idx1(1);
      ga.alpha = alpha; ga.beta = 0.0;
      ga.a_len = M * lda; ga.b_len = (long long)v * ldb; ga.c_len = M * N;
      HIPCK(gemm(ga, F, s));
    }
    return CCT_OK;
  };
  auto gemm_k_o = [&](const double* A, const double* Bm, long long bk, double* C, long long M, long long N) -> int {
    // C[M][N] += -1/2 sum_m A[m][k] B[k][n], K = o, A rows of o, B rows at stride bk
    if (nt_ok && o <= 16) {  // a streaming read-modify-write of C (even v: aligned pairs)
      HIPCK(rank_k_update(C, N, A, o, Bm, bk, (int)M, N, o, -0.5, s));
      return CCT_OK;
    }
    GemmArgs ga{};
    ga.M = (int)M; ga.N = (int)N; ga.K = o; ga.batch = 1;
    ga.A = A; ga.am = idx1(o); ga.ak = idx1(1);
    ga.B = Bm; ga.bk = idx1(bk); ga.bn = idx1(1);
    ga.C = C; ga.cm = idx1(N); ga.cn = idx1(1);
    ga.alpha = -0.5; ga.beta = 1.0;
    ga.a_len = M * o; ga.b_len = (long long)(o - 1) * bk + N; ga.c_len = M * N;
    HIPCK(gemm(ga, F, s));
    return CCT_OK;
  };
  static const int P24[24][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 1, 3}, {0, 2, 3, 1}, {0, 3, 1, 2}, {0, 3, 2, 1},
                                 {1, 0, 2, 3}, {1, 0, 3, 2}, {1, 2, 0, 3}, {1, 2, 3, 0}, {1, 3, 0, 2}, {1, 3, 2, 0},
                                 {2, 0, 1, 3}, {2, 0, 3, 1}, {2, 1, 0, 3}, {2, 1, 3, 0}, {2, 3, 0, 1}, {2, 3, 1, 0},
                                 {3, 0, 1, 2}, {3, 0, 2, 1}, {3, 1, 0, 2}, {3, 1, 2, 0}, {3, 2, 0, 1}, {3, 2, 1, 0}};
  auto term = [](const double* in, const int* pm, double coef) {
    QPermTerm t{};
    t.in = in;
    t.dst = 1;
    for (int k = 0; k < 4; ++k) t.perm[k] = pm[k];
    t.coef = coef;
    return t;
  };
  static const int ID[4] = {0, 1, 2, 3};
  long long task = -1;
  for (int i = 0; i < o; ++i)
    for (int j = i; j < o; ++j)
      for (int k = j; k < o; ++k)
        for (int l = k; l < o; ++l) {
          ++task;
          if ((i == j && j == k) || (j == k && k == l)) continue;
          const int oc[4] = {i, j, k, l};
          // distinct orderings q = o.s with the permutations that reach them
          std::vector<std::array<int, 4>> qs;
          std::vector<std::vector<int>> sig;
          for (int p = 0; p < 24; ++p) {
            const std::array<int, 4> q = {oc[P24[p][0]], oc[P24[p][1]], oc[P24[p][2]], oc[P24[p][3]]};
            size_t x = 0;
            while (x < qs.size() && qs[x] != q) ++x;
            if (x == qs.size()) {
              qs.push_back(q);
              sig.emplace_back();
            }
            sig[x].push_back(p);
          }
          // slots in (q1, q2) order: orderings that share Wbar_{e q1 q2}^{abc}
          // sit in adjacent slots and take one Y1 product between them
          {
            std::vector<size_t> ord(qs.size());
            for (size_t x = 0; x < ord.size(); ++x) ord[x] = x;
            std::stable_sort(ord.begin(), ord.end(), [&](size_t a1, size_t b1) {
              return std::make_pair(qs[a1][1], qs[a1][2]) < std::make_pair(qs[b1][1], qs[b1][2]);
            });
            std::vector<std::array<int, 4>> qs2;
            std::vector<std::vector<int>> sig2;
            for (size_t x : ord) {
              qs2.push_back(qs[x]);
              sig2.push_back(sig[x]);
            }
            qs.swap(qs2);
            sig.swap(sig2);
          }
          QCombineArgs cr{};
          cr.v = v; cr.beta = 0.0; cr.tiled = tl ? 1 : 0;
          for (size_t x = 0; x < qs.size(); ++x) {
            const long long q0 = qs[x][0], q1 = qs[x][1], q2 = qs[x][2], q3 = qs[x][3];
            double* X = Xb + (long long)x * v4;
            double* G = Gb + (long long)x * v4;
            // Y1 = 1/2 sum_e Wbar_{e q1 q2}^{abc} t_{q0 q3}^{ed} for this ordering and
            // the following ones with the same (q1, q2): their t2 blocks side by side
            // as the [e][(member, d)] operand, outputs to their adjacent slots
            if (x == 0 || qs[x - 1][1] != q1 || qs[x - 1][2] != q2) {
              size_t k = 1;
              while (x + k < qs.size() && qs[x + k][1] == q1 && qs[x + k][2] == q2) ++k;
              const double* Bm = ctx->t2 + (q0 * o + q3) * v2;
              long long ldb = v;
              if (k > 1) {
                for (size_t j = 0; j < k; ++j)
                  HIPCK(hipMemcpy2DAsync(Bc + (long long)j * v, sizeof(double) * k * v,
                                         ctx->t2 + ((long long)qs[x + j][0] * o + qs[x + j][3]) * v2,
                                         sizeof(double) * v, sizeof(double) * v, v, hipMemcpyDeviceToDevice, s));
                Bm = Bc;
                ldb = (long long)k * v;
              }
              const long long N = (long long)k * v;
              const Idx2 cn = idx2(v, v4, 1);
              const long long c_len = (24 - (long long)x) * v4;
              if (nt_ok) {
                NtArgs na{};
                na.M = (int)v3; na.N = (int)N; na.K = v; na.batch = 1;
                na.A = Wv + (q1 * o + q2) * v4; na.lda = v; na.B = Bm; na.ldb = ldb; na.b_kn = 1;
                na.C = G; na.cm = idx1(v); na.cn = cn;
                na.alpha = 0.5; na.beta = 0.0;
                na.a_len = v4; na.b_len = (long long)v * ldb; na.c_len = c_len;
                HIPCK(gemm_nt(na, F, s));
              } else {
                GemmArgs ga{};
                ga.M = (int)v3; ga.N = (int)N; ga.K = v; ga.batch = 1;
                ga.A = Wv + (q1 * o + q2) * v4; ga.am = idx1(v); ga.ak = idx1(1);
                ga.B = Bm; ga.bk = idx1(ldb); ga.bn = idx1(1);
                ga.C = G; ga.cm = idx1(v); ga.cn = cn;
                ga.alpha = 0.5; ga.beta = 0.0;
                ga.a_len = v4; ga.b_len = (long long)v * ldb; ga.c_len = c_len;
                HIPCK(gemm(ga, F, s));
              }
            }
            // X = 1/2 sum_e v^{ab}_{e q1} t_{q0 q2 q3}^{ecd} - 1/2 sum_m v^{am}_{q0 q1} t_{m q2 q3}^{bcd}
            const double* t3r = T3u + (q2 * o + q3) * o * v3;
            if (tl) X = Xb;  // one plain-layout scratch block; the sum goes to XT[x]
            RCK(gemm_x1_y1(VVVO + q1 * v3, v, t3r + q0 * v3, v2, X, v2, v2, 0.5));
            const double* VO = VOOO + (q0 * o + q1) * v * o;
            // Y2 = -1/2 sum_m Wbar_{q0 q1 q2}^{abm} t_{m q3}^{cd}
            const double* WO = Wo + ((q0 * o + q1) * o + q2) * v2 * o;
            if (tl) {
              HIPCK(rank_k_update_tiled(X, XT + (long long)x * T4, v, 1, VO, o, t3r, v3, o, -0.5, s));
              HIPCK(rank_k_update_tiled(G, GT + (long long)x * T4, v, 2, WO, o, ctx->t2 + q3 * v2, o * v2, o, -0.5, s));
              X = XT + (long long)x * T4;
              G = GT + (long long)x * T4;
            } else {
              RCK(gemm_k_o(VO, t3r, v3, X, v, v3));
              RCK(gemm_k_o(WO, ctx->t2 + q3 * v2, o * v2, G, v2, v2));
            }
            // R gets X + Y under every permutation reaching q; Abar gets
            // X + 1/4 v^{ab}_{q0 q1} t_{q2 q3}^{cd} under the first of them
            for (size_t k = 0; k < sig[x].size(); ++k) {
              QPermTerm tx = term(X, P24[sig[x][k]], 1.0);
              if (k == 0) {
                tx.dst = 3;
                tx.va = VVOO + (q0 * o + q1) * v2;
                tx.vb = ctx->t2 + (q2 * o + q3) * v2;
                tx.vcoef = 0.25;
              }
              cr.t[cr.nterms++] = tx;
              cr.t[cr.nterms++] = term(G, P24[sig[x][k]], 1.0);
            }
          }
          // one pass writes R and Abar (24 permutations: 48 terms, QMAXT)
          HIPCK(perm_combine(Rb, Ab, cr, s));
          // S(R) / eps_o: S = 2 (2 - P_cd) (2 - P_bc - P_bd) (2 - P_ab - P_ac - P_ad)
          static const int Sab[4] = {1, 0, 2, 3}, Sac[4] = {2, 1, 0, 3}, Sad[4] = {3, 1, 2, 0};
          static const int Sbc[4] = {0, 2, 1, 3}, Sbd[4] = {0, 3, 2, 1}, Scd[4] = {0, 1, 3, 2};
          QCombineArgs c1{};
          c1.v = v; c1.nterms = 4; c1.beta = 0.0;
          c1.t[0] = term(Rb, ID, 2.0); c1.t[1] = term(Rb, Sab, -1.0);
          c1.t[2] = term(Rb, Sac, -1.0); c1.t[3] = term(Rb, Sad, -1.0);
          HIPCK(perm_combine(Xb, nullptr, c1, s));
          QCombineArgs c2{};
          c2.v = v; c2.nterms = 3; c2.beta = 0.0;
          c2.t[0] = term(Xb, ID, 2.0); c2.t[1] = term(Xb, Sbc, -1.0); c2.t[2] = term(Xb, Sbd, -1.0);
          HIPCK(perm_combine(Gb, nullptr, c2, s));
          QCombineArgs c3{};
          c3.v = v; c3.nterms = 2; c3.beta = 0.0;
          c3.t[0] = term(Gb, ID, 4.0); c3.t[1] = term(Gb, Scd, -2.0);
          c3.eps_v = ctx->eps + o;
          c3.eps_occ = eps[i] + eps[j] + eps[k] + eps[l];
          HIPCK(perm_combine(Rb, nullptr, c3, s));
          HIPCK(dot(Ab, Rb, v4, et + task, ctx->red, s));
        }
  HIPCK(reduce_sum(et, ntask, et + ntask, ctx->red, s));
  std::vector<double> h((size_t)ntask + 1);
  HIPCK(hipMemcpyAsync(h.data(), et, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (e_tasks) std::copy(h.begin(), h.begin() + ntask, e_tasks);
  *e_q = h[(size_t)ntask];
  return finite_or_err(ctx, *e_q);
}

// --- perturbative quadruples in the virtual-tuple order --------------------
// E_(Q) summed over virtual tuples a <= b <= c <= d as in Eq. ener-pt-q-abc,
// with the alternative Wbar intermediates of Eq. q_w_alter (Sec. "ABC-based
// algorithm").  The virtual labels are cut into tiles of nb; a task is a tile
// quadruple tA <= tB <= tC <= tD and covers the dense box of tuples
// tau = (a, b, c, d), a in tA, ..., d in tD (the four "slots").  In the frame
// of tau (occupied index i_s paired with the label tau_s) the task
// accumulates
//   Xt[tau](i) = the sum over the 24 simultaneous column permutations of X,
//   Yt[tau](i) = the same sum of Y,
// without forming any ordered tuple's block: two permutations that differ
// by a column symmetry of a term's factors (T3 in two columns, Wbar^{vvv}_{voo}
// in (jb)(kc), Wbar^{vvo}_{ooo} in (ia)(jb)) give equal terms, so each kind of
// term reduces to 12 distinct contractions of weight 2, and those sharing
// the slots of the output rows are one matrix-core product with concatenated
// K segments (X1: 4 products of K = 3v, X2: 6 of K = 2o, Y1: 6 of K = 2v,
// Y2: 4 of K = 3o).  Then R = Xt + Yt is the full permutation sum of X + Y at
// tau, U = S(R) / eps with S the spin summation, and tau contributes
// (Xt + Vt, U) / |Stab(tau)| (Vt the six distinct rank-one V terms); only
// tuples with a <= b <= c <= d count, so every orbit is counted once.
long long q_abc_tiles(int v, int nb) { return (v + nb - 1) / nb; }
long long q_abc_task_count(int v, int nb) {
  const long long t = q_abc_tiles(v, nb);
  return t * (t + 1) * (t + 2) * (t + 3) / 24;
}

int energy_q_abc(cct_ctx* ctx, int nb, const int64_t* tasks, long long ntasks, double* e_q, double* e_tasks,
                 double* e_tuples, double* stats) {
  const int o = ctx->o, v = ctx->v, n = ctx->n;
  if (nb < 1 || nb > 16 || nb > v) {
    ctx->err = "energy_q_abc: block must be in [1, min(16, nvir)]";
    return CCT_EINVAL;
  }
  const long long ntile = q_abc_tiles(v, nb), ntot = q_abc_task_count(v, nb);
  if (!tasks) ntasks = ntot;
  if (ntasks < 0) return CCT_EINVAL;
  std::vector<long long> tlist((size_t)ntasks);
  for (long long i = 0; i < ntasks; ++i) {
    tlist[(size_t)i] = tasks ? (long long)tasks[i] : i;
    if (tlist[(size_t)i] < 0 || tlist[(size_t)i] >= ntot) {
      ctx->err = "energy_q_abc: task index " + std::to_string(tlist[(size_t)i]) + " outside [0, " +
                 std::to_string(ntot) + ")";
      return CCT_EINVAL;
    }
  }
  // task index -> tile quadruple (lexicographic over t0 <= t1 <= t2 <= t3)
  std::vector<std::array<int, 4>> quad;
  quad.reserve((size_t)ntot);
  for (int a = 0; a < ntile; ++a)
    for (int b = a; b < ntile; ++b)
      for (int c = b; c < ntile; ++c)
        for (int d = c; d < ntile; ++d) quad.push_back({a, b, c, d});
  const long long naux = ctx->naux, n2 = (long long)n * n, n4 = n2 * n2;
  const long long o2 = (long long)o * o, o3 = o2 * o, o4 = o2 * o2, v2 = (long long)v * v, o2v = o2 * v;
  const long long nvt = (long long)v * (v + 1) * (v + 2) / 6;
  const long long b2 = (long long)nb * nb, b3 = b2 * nb, b4 = b2 * b2;
  const std::vector<int> orbits = q_abc_orbits(o);
  const long long norb = (long long)orbits.size() / 25;
  // the T3 transposition works on cubes of 16^3 labels, A <= B <= C
  std::vector<int4> units;
  const int ncb = (v + 15) / 16;
  for (int a = 0; a < ncb; ++a)
    for (int b = a; b < ncb; ++b)
      for (int c = b; c < ncb; ++c) units.push_back(int4{a, b, c, 0});
  const long long nunit = (long long)units.size();
  const long long ntup = e_tuples ? b4 * ntasks : b4;
  const long long need = nvt * o3 + v2 * v2 + v2 * v * o + 2 * (long long)v * o3 + 3 * o2 * v2 + o4 +
                         3 * o2 * v2 + 12 * b2 * v * o3 + 12 * b3 * o3 + 36 * b3 * o2v + 12 * b2 * o4 +
                         2 * b4 * o4 + b4 * norb + ntup + ntasks + 2 * nunit + (long long)orbits.size() + 64 * 256;
  const double peak_gb = (double)(need + n4) * 8.0 / 1e9;
  // buffers from the context's workspace when it holds them, else from one
  // allocation for the duration of the call
  const size_t bytes = (size_t)(need + n4) * 8 + (size_t)64 * 256 * 64;
  Arena own_arena;
  Arena* ar = &ctx->ws;
  struct Own {
    cct_ctx* c;
    void* p = nullptr;
    ~Own() {
      if (p) {
        (void)hipStreamSynchronize(c->s);
        dev_free(c, p);
      }
    }
  } own{ctx};
  if ((double)ctx->ws.available() < (double)bytes) {
    if (!ctx->alloc_fn) {
      size_t fr = 0, tot = 0;
      HIPCK(hipMemGetInfo(&fr, &tot));
      if ((double)bytes + 256e6 > (double)fr) {
        ctx->err = "energy_q_abc: needs " + std::to_string(peak_gb) + " GB; the context workspace holds " +
                   std::to_string(ctx->ws.available() / 1e9) + " GB and the device has " + std::to_string(fr / 1e9) +
                   " GB free";
        return CCT_ENOMEM;
      }
    }
    RCK(dev_alloc(ctx, &own.p, bytes));
    own_arena.init((char*)own.p, bytes);
    ar = &own_arena;
  }
  struct Mark {
    Arena& a;
    size_t m;
    ~Mark() { a.reset(m); }
  } mark{*ar, ar->mark()};
  hipStream_t s = ctx->s;
  const Prec F = Prec::F64;
  auto get = [&](long long cnt) { return ar->alloc((size_t)std::max<long long>(cnt, 1)); };
  double* T3v = get(nvt * o3);
  double* VVVV = get(v2 * v2);
  double* VVVO = get(v2 * v * o);  // [x][y][j][e] = v^{xy}_{ej}
  double* VO1 = get((long long)v * o3);  // [x][i][j][m] = v^{xm}_{ij}
  double* VO2 = get((long long)v * o3);  // [x][i][j][m] = v^{xm}_{ji}
  double* Vmyje = get(o2 * v2);  // [m][y][j][e] = v^{my}_{ej}
  double* Vmxje = get(o2 * v2);  // [m][x][j][e] = v^{mx}_{je}
  double* Voooo = get(o4);        // [n][k][i][m] = v^{mn}_{ki}
  double* Vvvoo = get(o2 * v2);   // [x][y][i][j] = v^{xy}_{ij}
  double* t2R = get(o2 * v2);     // [d][e][i][j] = t_ij^ed
  double* t2L = get(o2 * v2);     // [x][e][i][j] = t_ij^xe
  double* t2Q = get(o2 * v2);     // [x][m][y][n] = t_mn^xy
  double* frag[4][4] = {};
  for (int r = 0; r < 4; ++r)
    for (int s0 = 0; s0 < 4; ++s0)
      if (s0 != r) frag[r][s0] = get(b2 * v * o3);
  double* x2b[4][4] = {};  // [s1][s0]: the T3 blocks of the X2 term with (s0, s1) on the rows
  for (int r0 = 0; r0 < 4; ++r0)
    for (int r1 = r0 + 1; r1 < 4; ++r1) {
      x2b[r1][r0] = get(b3 * o3);
      x2b[r0][r1] = get(b3 * o3);
    }
  double* Z[4][4][4] = {};
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int c = 0; c < 4; ++c)
        if (a != b && b != c && a != c) Z[a][b][c] = get(b3 * o2v);
  double* Wo[4][4] = {};  // [s3][s2]
  for (int s3 = 0; s3 < 4; ++s3)
    for (int s2 = 0; s2 < 4; ++s2)
      if (s2 != s3) Wo[s3][s2] = get(b2 * o4);
  auto pid = [](int r0, int r1) { return r0 * 4 + r1; };
  double* WvS[4][16] = {};  // [s0][pair id of the row slots (r0, r1)]
  for (int s0 = 0; s0 < 4; ++s0)
    for (int r0 = 0; r0 < 4; ++r0)
      for (int r1 = r0 + 1; r1 < 4; ++r1)
        if (s0 != r0 && s0 != r1) WvS[s0][pid(r0, r1)] = get(b3 * o2v);
  double* Xt = get(b4 * o4);
  double* Yt = get(b4 * o4);
  double* part = get(b4 * norb);
  int* d_orb = (int*)get(((long long)orbits.size() + 1) / 2);
  double* etup = get(ntup);
  double* etask = get(ntasks);
  int4* d_units = (int4*)get(2 * nunit);
  double* Vb = get(n4);
  if (!Vb || !d_units || !d_orb || !etask || !etup || !part || !Yt || !Xt) {
    ctx->err = "energy_q_abc: workspace exhausted (" + std::to_string(peak_gb) + " GB needed)";
    return CCT_ENOMEM;
  }
  hipEvent_t ev[4] = {};
  struct Ev {
    hipEvent_t* e;
    ~Ev() {
      for (int i = 0; i < 4; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } evguard{ev};
  for (auto& e : ev) HIPCK(hipEventCreate(&e));
  HIPCK(hipEventRecord(ev[0], s));
  // bare integrals v^{pq}_{rs} = (pr|qs), then the slices the task products read
  {
    GemmArgs ga{};
    ga.M = (int)n2; ga.N = (int)n2; ga.K = (int)naux; ga.batch = 1;
    ga.A = ctx->B; ga.am = idx1(1); ga.ak = idx1(n2);
    ga.B = ctx->B; ga.bk = idx1(n2); ga.bn = idx1(1);
    ga.C = Vb; ga.cm = idx1(n2); ga.cn = idx1(1);
    ga.alpha = 1.0; ga.beta = 0.0;
    ga.a_len = naux * n2; ga.b_len = naux * n2; ga.c_len = n4;
    HIPCK(gemm(ga, F, s));
  }
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vvvv"), "xyef", 0.0, dense(VVVV, {v, v, v, v}), "xyef"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vvvo"), "xyej", 0.0, dense(VVVO, {v, v, o, v}), "xyje"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vooo"), "xmij", 0.0, dense(VO1, {v, o, o, o}), "xijm"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vooo"), "xmji", 0.0, dense(VO2, {v, o, o, o}), "xijm"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "ovvo"), "myej", 0.0, dense(Vmyje, {o, v, o, v}), "myje"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "ovov"), "mxje", 0.0, dense(Vmxje, {o, v, o, v}), "mxje"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "oooo"), "mnki", 0.0, dense(Voooo, {o, o, o, o}), "nkim"));
  STCK(accumulate(s, 1.0, Vview(ctx, Vb, "vvoo"), "xyij", 0.0, dense(Vvvoo, {v, v, o, o}), "xyij"));
  {
    const DT t2 = dense(ctx->t2, {o, o, v, v});
    STCK(accumulate(s, 1.0, t2, "ijed", 0.0, dense(t2R, {v, v, o, o}), "deij"));
    STCK(accumulate(s, 1.0, t2, "ijxe", 0.0, dense(t2L, {v, v, o, o}), "xeij"));
    STCK(accumulate(s, 1.0, t2, "mnxy", 0.0, dense(t2Q, {v, o, v, o}), "xmyn"));
  }
  // T3 in the virtual-triangular layout (the one-time transposition of the
  // compact amplitudes, Fig. q_operation_counts(a))
  HIPCK(hipMemcpyAsync(d_units, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice, s));
  HIPCK(hipMemcpyAsync(d_orb, orbits.data(), sizeof(int) * orbits.size(), hipMemcpyHostToDevice, s));
  HIPCK(hipStreamSynchronize(s));  // the host tables are released below
  HIPCK(t3v_transpose(ctx->t3, ctx->tbl, T3v, d_units, nunit, o, v, s));
  HIPCK(fill(etup, 0.0, ntup, s));
  HIPCK(hipEventRecord(ev[1], s));

  // Two streams per task: the X chain (T3 gathers, X1, X2 into Xt) on the
  // context's stream, the Y chain (Z, Wbar^{vvv}, Wbar^{vvo}, Y1, Y2 into Yt)
  // on a side stream, so that the bandwidth-bound passes of one chain overlap
  // the matrix-core products of the other; the side stream joins before the
  // energy, which forms R = Xt + Yt.  (Default priority, created for the call.)
  struct Side {
    hipStream_t st = nullptr;
    hipEvent_t ready = nullptr, ydone = nullptr, yfree = nullptr;
    ~Side() {
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
      for (hipEvent_t e : {ready, ydone, yfree})
        if (e) (void)hipEventDestroy(e);
    }
  } side;
  HIPCK(hipStreamCreateWithFlags(&side.st, hipStreamNonBlocking));
  HIPCK(hipEventCreateWithFlags(&side.ready, hipEventDisableTiming));
  HIPCK(hipEventCreateWithFlags(&side.ydone, hipEventDisableTiming));
  HIPCK(hipEventCreateWithFlags(&side.yfree, hipEventDisableTiming));
  hipStream_t sy = side.st;
  HIPCK(hipEventRecord(side.ready, s));
  HIPCK(hipStreamWaitEvent(sy, side.ready, 0));

  double macs_mfma = 0.0, macs_valu = 0.0;
  auto run = [&](QGemmArgs& g, hipStream_t st) -> int {
    long long batch = 1;
    for (int d = 0; d < g.nd; ++d) batch *= g.rad[d];
    long long K = 0;
    for (int k = 0; k < g.nseg; ++k) K += g.K[k];
    macs_mfma += (double)g.M * g.N * K * batch;
    HIPCK(qgemm(g, st));
    return CCT_OK;
  };
  const long long pw[4] = {o3, o2, (long long)o, 1};
  auto lin = [](long long st) { return Idx4{1, 1, 1, st, 0, 0, 0}; };
  auto pair_map = [&](int u, int w) { return Idx4{1, 1, o, pw[u], 0, 0, pw[w]}; };       // (i_u, i_w)
  auto trip_map = [&](int a, int b, int c) { return Idx4{1, o, o, pw[a], 0, pw[b], pw[c]}; };  // (i_a, i_b, i_c)

  for (long long ti = 0; ti < ntasks; ++ti) {
    const std::array<int, 4>& tq = quad[(size_t)tlist[(size_t)ti]];
    QSlots sl{};
    for (int k = 0; k < 4; ++k) {
      sl.st[k] = tq[k] * nb;
      sl.n[k] = std::min(nb, v - sl.st[k]);
    }
    long long S[4];
    for (int k = 0; k < 4; ++k) {
      S[k] = o4;
      for (int t = k + 1; t < 4; ++t) S[k] *= sl.n[t];
    }
    const long long ntau = (long long)sl.n[0] * sl.n[1] * sl.n[2] * sl.n[3];
    const long long tlen = ntau * o4;
    // T3 slices: X1 fragments [lx][ly][e][i_u][i_v][i_w] (u < v < w the slots
    // other than r; column pairs (i_s0, e), (i_x, tau_x), (i_y, tau_y))
    for (int r = 0; r < 4; ++r) {
      int oth[3], k = 0;
      for (int t = 0; t < 4; ++t)
        if (t != r) oth[k++] = t;
      for (int a = 0; a < 3; ++a) {
        const int s0 = oth[a], x = oth[a == 0 ? 1 : 0], y = oth[a == 2 ? 1 : 2];
        T3Gather g{};
        g.o = o; g.v = v; g.nd = 2; g.ne = v;
        g.rad[0] = sl.n[x]; g.rad[1] = sl.n[y];
        g.st[0] = sl.st[x]; g.st[1] = sl.st[y];
        auto pos = [&](int sl_) { return sl_ == oth[0] ? 0 : (sl_ == oth[1] ? 1 : 2); };
        g.lab[0] = 3; g.ax[0] = pos(s0);
        g.lab[1] = 0; g.ax[1] = pos(x);
        g.lab[2] = 1; g.ax[2] = pos(y);
        HIPCK(t3v_gather(T3v, frag[r][s0], g, s));
      }
    }
    // X2 blocks [l_s1][l_c0][l_c1][m][i_c0][i_c1], column pairs (m, tau_s1),
    // (i_c0, tau_c0), (i_c1, tau_c1), for the rows (s0, s1)
    for (int r0 = 0; r0 < 4; ++r0)
      for (int r1 = r0 + 1; r1 < 4; ++r1) {
        int cc[2], k = 0;
        for (int t = 0; t < 4; ++t)
          if (t != r0 && t != r1) cc[k++] = t;
        for (int w = 0; w < 2; ++w) {
          const int s1 = w == 0 ? r1 : r0, s0 = w == 0 ? r0 : r1;
          T3Gather g{};
          g.o = o; g.v = v; g.nd = 3; g.ne = 1;
          g.rad[0] = sl.n[s1]; g.rad[1] = sl.n[cc[0]]; g.rad[2] = sl.n[cc[1]];
          g.st[0] = sl.st[s1]; g.st[1] = sl.st[cc[0]]; g.st[2] = sl.st[cc[1]];
          for (int c = 0; c < 3; ++c) {
            g.lab[c] = c;
            g.ax[c] = c;
          }
          HIPCK(t3v_gather(T3v, x2b[s1][s0], g, s));
        }
      }
    // Z_abc[la][lb][lc][j][k][e] = 1/2 sum_f v^{xy}_{ef} t_jk^{fz}
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c) {
          if (a == b || b == c || a == c) continue;
          QGemmArgs g{};
          g.M = (int)(sl.n[c] * o2); g.N = v; g.nseg = 1; g.K[0] = v;
          g.nd = 2; g.rad[0] = sl.n[a]; g.rad[1] = sl.n[b];
          g.akm = true; g.bkn = false;
          g.a[0].p = t2L + (long long)sl.st[c] * o2; g.a[0].ld = (long long)v * o2; g.a[0].len = o2 * v2 - (long long)sl.st[c] * o2;
          g.b[0].p = VVVV + ((long long)sl.st[a] * v + sl.st[b]) * v2; g.b[0].ld = v;
          g.b[0].sd[0] = (long long)v * v2; g.b[0].sd[1] = v2;
          g.b[0].len = v2 * v2 - ((long long)sl.st[a] * v + sl.st[b]) * v2;
          g.C = Z[a][b][c]; g.cm = lin(v); g.cn = lin(1);
          g.sc[0] = (long long)sl.n[b] * sl.n[c] * o2v; g.sc[1] = (long long)sl.n[c] * o2v;
          g.c_len = b3 * o2v;
          g.alpha = 0.5; g.accumulate = 0;
          RCK(run(g, sy));
        }
    // Wbar^{vvv}_{voo} for x in slot s0, (y, z) in the row slots (r0, r1)
    for (int s0 = 0; s0 < 4; ++s0)
      for (int r0 = 0; r0 < 4; ++r0)
        for (int r1 = r0 + 1; r1 < 4; ++r1) {
          if (s0 == r0 || s0 == r1) continue;
          HIPCK(q_wv_build(WvS[s0][pid(r0, r1)], Z[s0][r0][r1], Z[s0][r1][r0], Vmyje, Vmxje, ctx->t2, o, v, sl.st[s0],
                           sl.n[s0], sl.st[r0], sl.n[r0], sl.st[r1], sl.n[r1], sy));
          macs_valu += 4.0 * o * sl.n[s0] * sl.n[r0] * sl.n[r1] * o2v;
        }
    // Wbar^{vvo}_{ooo} for (x, y) in slots (s0 < s1), rows = the slots other than s3
    for (int s3 = 0; s3 < 4; ++s3)
      for (int s2 = 0; s2 < 4; ++s2) {
        if (s2 == s3) continue;
        int rs[3], k = 0, p01[2], kk = 0;
        for (int t = 0; t < 4; ++t)
          if (t != s3) rs[k++] = t;
        for (int t = 0; t < 4; ++t)
          if (t != s3 && t != s2) p01[kk++] = t;
        auto pos = [&](int sl_) { return sl_ == rs[0] ? 0 : (sl_ == rs[1] ? 1 : 2); };
        const int rowpos[3] = {pos(p01[0]), pos(p01[1]), pos(s2)};
        HIPCK(q_wo_build(Wo[s3][s2], Voooo, ctx->t2, o, v, sl.st[p01[0]], sl.n[p01[0]], sl.st[p01[1]], sl.n[p01[1]],
                         rowpos, sy));
        macs_valu += 2.0 * o * sl.n[p01[0]] * sl.n[p01[1]] * o4;
      }
    // X1: per row slot r, K segments over s0 (the slot whose label is summed)
    for (int r = 0; r < 4; ++r) {
      int oth[3], k = 0;
      for (int t = 0; t < 4; ++t)
        if (t != r) oth[k++] = t;
      QGemmArgs g{};
      g.nseg = 3; g.nd = 3;
      for (int d = 0; d < 3; ++d) {
        g.rad[d] = sl.n[oth[d]];
        g.sc[d] = S[oth[d]];
      }
      const bool sw = r == 3;  // the unit-stride axis i_3 on the rows side
      for (int a = 0; a < 3; ++a) {
        const int s0 = oth[a];
        const int xd = a == 0 ? 1 : 0, yd = a == 2 ? 1 : 2;  // digits of x and y
        QgOperand V{}, Fr{};
        V.p = VVVO + ((long long)sl.st[s0] * v + sl.st[r]) * o * v;
        V.ld = v;
        V.sd[a] = v2 * o;
        V.len = v2 * v * o - ((long long)sl.st[s0] * v + sl.st[r]) * o * v;
        Fr.p = frag[r][s0];
        Fr.ld = o3;
        Fr.sd[xd] = (long long)sl.n[oth[yd]] * v * o3;
        Fr.sd[yd] = (long long)v * o3;
        Fr.len = b2 * v * o3;
        g.K[a] = v;
        g.a[a] = sw ? Fr : V;
        g.b[a] = sw ? V : Fr;
      }
      const Idx4 rowm = Idx4{1, 1, o, S[r], 0, 0, pw[r]};
      const Idx4 colm = trip_map(oth[0], oth[1], oth[2]);
      g.akm = sw; g.bkn = !sw;
      g.M = (int)(sw ? o3 : sl.n[r] * o);
      g.N = (int)(sw ? sl.n[r] * o : o3);
      g.cm = sw ? colm : rowm;
      g.cn = sw ? rowm : colm;
      g.C = Xt; g.c_len = tlen;
      g.alpha = 1.0; g.accumulate = r == 0 ? 0 : 1;
      RCK(run(g, s));
    }
    // X2: per row pair (r0, r1), segments (s0, s1) = (r0, r1) and (r1, r0)
    for (int r0 = 0; r0 < 4; ++r0)
      for (int r1 = r0 + 1; r1 < 4; ++r1) {
        int cc[2], k = 0;
        for (int t = 0; t < 4; ++t)
          if (t != r0 && t != r1) cc[k++] = t;
        QGemmArgs g{};
        g.nseg = 2; g.nd = 4;
        for (int d = 0; d < 4; ++d) {
          g.rad[d] = sl.n[d];
          g.sc[d] = S[d];
        }
        const bool sw = r1 == 3;
        for (int w = 0; w < 2; ++w) {
          const int s0 = w == 0 ? r0 : r1, s1 = w == 0 ? r1 : r0;
          QgOperand A{}, B{};
          A.p = (w == 0 ? VO1 : VO2) + (long long)sl.st[s0] * o3;
          A.ld = o;
          A.sd[s0] = o3;
          A.len = (long long)v * o3 - (long long)sl.st[s0] * o3;
          B.p = x2b[s1][s0];
          B.ld = o2;
          B.sd[s1] = (long long)sl.n[cc[0]] * sl.n[cc[1]] * o3;
          B.sd[cc[0]] = (long long)sl.n[cc[1]] * o3;
          B.sd[cc[1]] = o3;
          B.len = b3 * o3;
          g.K[w] = o;
          g.a[w] = sw ? B : A;
          g.b[w] = sw ? A : B;
        }
        const Idx4 rowm = pair_map(r0, r1), colm = pair_map(cc[0], cc[1]);
        g.akm = sw; g.bkn = !sw;
        g.M = (int)o2; g.N = (int)o2;
        g.cm = sw ? colm : rowm;
        g.cn = sw ? rowm : colm;
        g.C = Xt; g.c_len = tlen;
        g.alpha = -1.0; g.accumulate = 1;
        RCK(run(g, s));
      }
    // Y1: per column pair (c0, c1), segments (s0, s3) = (c0, c1) and (c1, c0);
    // rows (l_r0, l_r1, i_r0, i_r1).  Yt is overwritten only after the
    // previous task's energy has read it.
    if (ti > 0) HIPCK(hipStreamWaitEvent(sy, side.yfree, 0));
    bool firsty = true;
    for (int c0 = 0; c0 < 4; ++c0)
      for (int c1 = c0 + 1; c1 < 4; ++c1) {
        int rr[2], k = 0;
        for (int t = 0; t < 4; ++t)
          if (t != c0 && t != c1) rr[k++] = t;
        QGemmArgs g{};
        g.nseg = 2; g.nd = 2;
        g.rad[0] = sl.n[c0]; g.rad[1] = sl.n[c1];
        g.sc[0] = S[c0]; g.sc[1] = S[c1];
        const bool sw = c1 != 3;  // i_3 among the row slots
        const long long wvb = (long long)sl.n[rr[0]] * sl.n[rr[1]] * o2v;
        for (int w = 0; w < 2; ++w) {
          const int s0 = w == 0 ? c0 : c1;
          QgOperand A{}, B{};
          A.p = WvS[s0][pid(rr[0], rr[1])];
          A.ld = v;
          A.sd[w] = wvb;
          A.len = (long long)sl.n[s0] * wvb;
          if (w == 0) {  // t_{i_c0 i_c1}^{e tau_c1}
            B.p = t2R + (long long)sl.st[c1] * v * o2;
            B.sd[1] = (long long)v * o2;
            B.len = o2 * v2 - (long long)sl.st[c1] * v * o2;
          } else {  // t_{i_c1 i_c0}^{e tau_c0} = t_{i_c0 i_c1}^{tau_c0 e}
            B.p = t2L + (long long)sl.st[c0] * v * o2;
            B.sd[0] = (long long)v * o2;
            B.len = o2 * v2 - (long long)sl.st[c0] * v * o2;
          }
          B.ld = o2;
          g.K[w] = v;
          g.a[w] = sw ? B : A;
          g.b[w] = sw ? A : B;
        }
        const Idx4 rowm = Idx4{sl.n[rr[1]], o, o, S[rr[0]], S[rr[1]], pw[rr[0]], pw[rr[1]]};
        const Idx4 colm = pair_map(c0, c1);
        const long long Mr = (long long)sl.n[rr[0]] * sl.n[rr[1]] * o2;
        g.akm = sw; g.bkn = !sw;
        g.M = (int)(sw ? o2 : Mr);
        g.N = (int)(sw ? Mr : o2);
        g.cm = sw ? colm : rowm;
        g.cn = sw ? rowm : colm;
        g.C = Yt; g.c_len = tlen;
        g.alpha = 1.0; g.accumulate = firsty ? 0 : 1;
        firsty = false;
        RCK(run(g, sy));
      }
    // Y2: per column slot s3, segments over s2 (the Wbar^{vvo}_{ooo} pair is
    // the other two slots)
    for (int s3 = 0; s3 < 4; ++s3) {
      int rs[3], k = 0;
      for (int t = 0; t < 4; ++t)
        if (t != s3) rs[k++] = t;
      QGemmArgs g{};
      g.nseg = 3; g.nd = 3;
      for (int d = 0; d < 3; ++d) {
        g.rad[d] = sl.n[rs[d]];
        g.sc[d] = S[rs[d]];
      }
      const bool sw = s3 != 3;
      for (int a = 0; a < 3; ++a) {
        const int s2 = rs[a];
        const int d0 = a == 0 ? 1 : 0, d1 = a == 2 ? 1 : 2;  // digits of the pair (s0 < s1)
        QgOperand A{}, B{};
        A.p = Wo[s3][s2];
        A.ld = o;
        A.sd[d0] = (long long)sl.n[rs[d1]] * o4;
        A.sd[d1] = o4;
        A.len = b2 * o4;
        B.p = t2Q + (long long)sl.st[s2] * o * v * o + (long long)sl.st[s3] * o;
        B.ld = (long long)v * o;
        B.sd[a] = (long long)o * v * o;
        B.len = o2 * v2 - ((long long)sl.st[s2] * o * v * o + (long long)sl.st[s3] * o);
        g.K[a] = o;
        g.a[a] = sw ? B : A;
        g.b[a] = sw ? A : B;
      }
      const Idx4 rowm = trip_map(rs[0], rs[1], rs[2]);
      const Idx4 colm = Idx4{1, 1, o, S[s3], 0, 0, pw[s3]};
      g.akm = sw; g.bkn = !sw;
      g.M = (int)(sw ? sl.n[s3] * o : o3);
      g.N = (int)(sw ? o3 : sl.n[s3] * o);
      g.cm = sw ? colm : rowm;
      g.cn = sw ? rowm : colm;
      g.C = Yt; g.c_len = tlen;
      g.alpha = -1.0; g.accumulate = 1;
      RCK(run(g, sy));
    }
    // energies of the box's tuples (R = Xt + Yt formed inside)
    HIPCK(hipEventRecord(side.ydone, sy));
    HIPCK(hipStreamWaitEvent(s, side.ydone, 0));
    HIPCK(q_abc_energy(Xt, Yt, Vvvoo, t2R, ctx->eps, sl, o, v, d_orb, (int)norb, part,
                       etup + (e_tuples ? ti * b4 : 0), etask + ti, s));
    HIPCK(hipEventRecord(side.yfree, s));  // Yt read: free for the next task's Y chain
  }
  HIPCK(hipEventRecord(ev[2], s));
  std::vector<double> h((size_t)ntasks);
  if (ntasks > 0) HIPCK(hipMemcpyAsync(h.data(), etask, sizeof(double) * ntasks, hipMemcpyDeviceToHost, s));
  if (e_tuples && ntasks > 0) HIPCK(hipMemcpyAsync(e_tuples, etup, sizeof(double) * b4 * ntasks, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  double sum = 0.0;
  for (double x : h) sum += x;
  if (e_tasks) std::copy(h.begin(), h.end(), e_tasks);
  *e_q = sum;
  if (stats) {
    float t01 = 0.f, t12 = 0.f;
    HIPCK(hipEventElapsedTime(&t01, ev[0], ev[1]));
    HIPCK(hipEventElapsedTime(&t12, ev[1], ev[2]));
    stats[0] = t01;
    stats[1] = t12;
    stats[2] = macs_mfma;
    stats[3] = macs_valu;
  }
  return finite_or_err(ctx, sum);
}

// --- DIIS ---------------------------------------------------------------
// T3 elements per packed block that take part in DIIS (Sec. "Distributed
// DIIS": all of T3, none of it, or only the low-energy virtual subspace)
long long diis_block(const cct_ctx* ctx) {
  if (!ctx->diis_t3) return 0;
  const long long s = ctx->diis_sv > 0 ? ctx->diis_sv : ctx->v;
  return s * s * s;
}

long long diis_len(cct_ctx* ctx) {
  const long long n12 = (long long)ctx->o * ctx->v + (long long)ctx->o * ctx->o * ctx->v * ctx->v;
  return n12 + ctx->ntri * diis_block(ctx);
}

int copy_amps_to(cct_ctx* ctx, double* dst) {
  const long long n1 = (long long)ctx->o * ctx->v, n2 = n1 * n1;
  HIPCK(axpby(1.0, ctx->t1, 0.0, dst, n1, ctx->s));
  HIPCK(axpby(1.0, ctx->t2, 0.0, dst + n1, n2, ctx->s));
  if (ctx->diis_t3 && ctx->diis_sv > 0)
    HIPCK(t3_subcube(ctx->t3, dst + n1 + n2, ctx->ntri, ctx->v, ctx->diis_sv, true, ctx->s));
  else if (ctx->diis_t3)
    HIPCK(axpby(1.0, ctx->t3, 0.0, dst + n1 + n2, ctx->ntri * ctx->v3, ctx->s));
  return CCT_OK;
}

// The DIIS part of a vector back into the amplitudes (inverse of copy_amps_to).
int copy_amps_from(cct_ctx* ctx, const double* src) {
  const long long n1 = (long long)ctx->o * ctx->v, n2 = n1 * n1;
  HIPCK(axpby(1.0, src, 0.0, ctx->t1, n1, ctx->s));
  HIPCK(axpby(1.0, src + n1, 0.0, ctx->t2, n2, ctx->s));
  if (ctx->diis_t3 && ctx->diis_sv > 0)
    HIPCK(t3_subcube(ctx->t3, const_cast<double*>(src + n1 + n2), ctx->ntri, ctx->v, ctx->diis_sv, false, ctx->s));
  else if (ctx->diis_t3)
    HIPCK(axpby(1.0, src + n1 + n2, 0.0, ctx->t3, ctx->ntri * ctx->v3, ctx->s));
  return CCT_OK;
}

DiisArgs diis_args(const cct_ctx* ctx) {
  DiisArgs a{};
  a.L = ctx->diis_len;
  a.n12 = (long long)ctx->o * ctx->v + (long long)ctx->o * ctx->o * ctx->v * ctx->v;
  a.bs = diis_block(ctx);
  a.tri = ctx->tri;
  a.ntri = (int)ctx->ntri;
  a.M = ctx->diis_space;
  a.start = ctx->diis_start;
  return a;
}

// Empty DIIS history.  Enqueued on the context's stream (a kernel).
int diis_reset(cct_ctx* ctx) {
  if (ctx->diis_st) HIPCK(diis_device_reset(ctx->diis_st, ctx->s));
  return CCT_OK;
}

// After the Jacobi step: T holds the Jacobi-updated amplitudes, diis_old the
// amplitudes before it.  The Jacobi vector is gathered, the device step
// (overlaps, bordered solve, history update, extrapolation) runs, and the
// result is written back; no synchronisation.
int diis_step(cct_ctx* ctx) {
  RCK(copy_amps_to(ctx, ctx->diis_new));
  const DiisArgs a = diis_args(ctx);
  HIPCK(diis_device_step(ctx->diis_new, ctx->diis_old, ctx->dvecs, ctx->derrs, ctx->diis_part, ctx->diis_d,
                         ctx->diis_B, ctx->diis_st, ctx->diis_coef, a, ctx->s));
  RCK(copy_amps_from(ctx, ctx->diis_new));
  return CCT_OK;
}

// One whole iteration on the context's stream: save the amplitudes for DIIS,
// residual, T3 and T1/T2 Jacobi steps, DIIS, energy; the squared norms and the
// energy are left in scal[0..2] and scal[6] (and copied to out, if given).
// No host synchronisation and no allocation: safe to record into a graph.
int enqueue_iteration(cct_ctx* ctx, double* out = nullptr) {
  const bool use_diis = ctx->diis_on && ctx->diis_space > 0;
  if (use_diis) RCK(copy_amps_to(ctx, ctx->diis_old));
  RCK(enqueue_residual(ctx, CCT_TERM_ALL, true));
  HIPCK(jacobi_t1t2(ctx->t1, ctx->r1, ctx->t2, ctx->r2, ctx->eps, ctx->o, ctx->v, ctx->s));
  mark(ctx, PH_DIIS);
  if (use_diis) RCK(diis_step(ctx));
  RCK(enqueue_energy(ctx, out));
  mark(ctx, PH_N);
  return CCT_OK;
}

// Read back the norms and energy of an enqueued iteration (one copy, one
// synchronisation) and check them.
int finish_iteration(cct_ctx* ctx, double* e, double norms[3]) {
  double h[7];
  HIPCK(hipMemcpyAsync(h, ctx->scal, 7 * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  if (ctx->events) {
    for (int i = 0; i < PH_N; ++i) {
      float msv = 0.f;
      if (hipEventElapsedTime(&msv, ctx->ev[i], ctx->ev[i + 1]) == hipSuccess) ctx->ms[i] = msv;
    }
    for (int i = 0; i + 1 < ctx->lad_nev; i += 2) {
      float msv = 0.f;
      if (hipEventElapsedTime(&msv, ctx->lad_ev[i], ctx->lad_ev[i + 1]) == hipSuccess) ctx->lad_ms += msv;
    }
  }
  ctx->have_res = true;
  if (e) *e = h[6];
  if (norms) for (int i = 0; i < 3; ++i) norms[i] = h[i];
  for (int i = 0; i < 3; ++i) RCK(finite_or_err(ctx, h[i]));
  return finite_or_err(ctx, h[6]);
}

int update(cct_ctx* ctx, double* e, double norms[3]) {
  RCK(enqueue_iteration(ctx));
  return finish_iteration(ctx, e, norms);
}

// --- autotuner ------------------------------------------------------------
// The ladder and ring GEMMs are timed in each available tile variant on this
// context's own shapes (the ladder on a truncated M, writing scratch output);
// the fastest variant of each class is used from then on.  Choices persist in
// a flat JSON file named by the CCT_TUNE_CACHE environment variable, keyed by
// (o, v, precision, class).
const char* prec_name(Prec p) { return p == Prec::F64 ? "fp64" : (p == Prec::F32 ? "fp32" : "bf16x3"); }

// the two ladder forms have different GEMM shapes and are tuned apart
const char* ladder_class(const cct_ctx* ctx) { return ctx->ladder_split && ctx->v >= 2 ? "ladder_split" : "ladder"; }

std::string tune_key(const cct_ctx* ctx, const char* cls) {
  return "o" + std::to_string(ctx->o) + "_v" + std::to_string(ctx->v) + "_" + prec_name(ctx->prec) + "_" + cls;
}

std::map<std::string, int> read_tune_cache() {
  std::map<std::string, int> m;
  const char* path = std::getenv("CCT_TUNE_CACHE");
  if (!path || !*path) return m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  std::string js;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) js.append(buf, k);
  std::fclose(f);
  size_t p = 0;
  while ((p = js.find('"', p)) != std::string::npos) {
    const size_t q = js.find('"', p + 1);
    if (q == std::string::npos) break;
    const std::string key = js.substr(p + 1, q - p - 1);
    const size_t c = js.find(':', q);
    if (c == std::string::npos) break;
    m[key] = std::atoi(js.c_str() + c + 1);
    p = c + 1;
  }
  return m;
}

void write_tune_cache(const std::map<std::string, int>& m) {
  const char* path = std::getenv("CCT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{");
  bool first = true;
  for (const auto& kv : m) {
    std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  std::fprintf(f, "\n}\n");
  std::fclose(f);
}

void apply_tune_cache(cct_ctx* ctx) {
  const auto m = read_tune_cache();
  auto it = m.find(tune_key(ctx, ladder_class(ctx)));
  if (it != m.end()) ctx->tune_ladder = it->second;
  it = m.find(tune_key(ctx, "rings"));
  if (it != m.end()) ctx->tune_rings = it->second;
}

// Time one launch after a warm-up launch; -1 if the variant cannot run.
template <typename F>
float time_launch(hipStream_t s, F launch) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
  float ms = -1.f;
  if (launch() == hipSuccess && hipEventRecord(e0, s) == hipSuccess && launch() == hipSuccess &&
      hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.f;
  }
  (void)hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

int autotune(cct_ctx* ctx, double budget_ms, double* spent) {
  const int o = ctx->o, v = ctx->v;
  const long long v2 = (long long)v * v, v4 = v2 * v2, ov = (long long)o * v, ov3 = o * ctx->v3;
  const bool f64 = ctx->prec == Prec::F64;
  Arena& ws = ctx->ws;
  ws.reset(0);
  double used = 0.0;
  auto pick = [&](std::vector<int> cands, auto run) -> int {
    int best = 0;
    float tbest = 0.f;
    for (int c : cands) {
      if (used > budget_ms && best != 0) break;
      const float t = time_launch(ctx->s, [&] { return run(c); });
      if (t < 0.f) continue;
      used += 2.0 * t;
      // a later candidate has to be clearly faster (2 %) to replace the
      // earlier one, so that near-ties keep the first-listed shape
      if (best == 0 || t < 0.98f * tbest) { best = c; tbest = t; }
    }
    return best;
  };
  // ---- ladder: one relabelled term on the first Mt rows of the stored blocks,
  // in the shape of the form in use (split: N = pairs y <= z, K = pairs d <= e
  // padded to the vector width; direct: N = K = v^2)
  const bool split = ctx->ladder_split && v >= 2;
  const long long vp = (long long)v * (v + 1) / 2;
  const long long lN = split ? vp : v2, lK = split ? round_up(vp, lp_kpad(ctx, vp)) : v2;
  const bool lad_lp = !f64, lad_nt = f64 && (split || !(v2 & 1));
  if ((lad_lp || lad_nt) && lN * lK <= v4) {
    const long long M = std::min(ctx->ntri * v, ctx->ntri * ctx->v3 / lK);
    const long long Mt = std::min(M, std::max<long long>(1024, (long long)(2e9 / 8.0 / (double)lN)));
    const size_t mk = ws.mark();
    double* C = ws.alloc((size_t)(Mt * lN));
    if (!C) { ctx->err = "workspace exhausted (autotune)"; return CCT_ENOMEM; }
    // operands: T3 and W read as Mt x lK and lN x lK matrices (values only
    // matter for timing; both fit inside the stored arrays)
    if (lad_nt) {
      ctx->tune_ladder = pick({9, 10, 1, 2, 3, 4}, [&](int var) {
        NtArgs g{};
        g.M = (int)Mt; g.N = (int)lN; g.K = (int)lK; g.batch = 1;
        g.A = ctx->t3; g.lda = lK; g.B = ctx->Wvvvv; g.ldb = lK;
        g.C = C; g.cm = idx1(lN); g.cn = idx1(1); g.alpha = 1.0; g.beta = 0.0;
        g.a_len = ctx->ntri * ctx->v3; g.b_len = v4; g.c_len = Mt * lN; g.variant = var;
        return gemm_nt(g, Prec::F64, ctx->s);
      });
    } else {
      void* Al = alloc_lp(ws, Mt * lK);
      void* Bl = alloc_lp(ws, lN * lK);
      if (!Al || !Bl) { ctx->err = "workspace exhausted (autotune)"; return CCT_ENOMEM; }
      // the operand format of the ladder form in use
      const int fmt = split ? lp_fmt_gemm(ctx, vp) : lp_fmt(ctx->prec);
      HIPCK(convert(ctx->t3, OutSpec{Al, fmt, Mt * lK}, Mt * lK, ctx->s));
      HIPCK(convert(ctx->Wvvvv, OutSpec{Bl, fmt, lN * lK}, lN * lK, ctx->s));
      ctx->tune_ladder = pick(ctx->prec == Prec::BF16X3 ? std::vector<int>{5, 4, 1, 2, 3} : std::vector<int>{5, 1, 2, 3},
                              [&](int var) {
        NtLpArgs g{};
        g.M = (int)Mt; g.N = (int)lN; g.K = (int)lK; g.batch = 1;
        g.A = Al; g.lda = lK; g.a_plane = Mt * lK; g.B = Bl; g.ldb = lK; g.b_plane = lN * lK;
        g.C = C; g.cm = idx1(lN); g.cn = idx1(1); g.alpha = 1.0; g.beta = 0.0;
        g.a_len = Mt * lK; g.b_len = lN * lK; g.c_len = Mt * lN; g.variant = var;
        g.il = fmt == OUT_BF16X2I;
        return gemm_nt_lp(g, ctx->prec, ctx->s);
      });
    }
    ws.reset(mk);
  }
  // ---- rings: one batch of occupied pairs with the planned batch size (at
  // most 8), in the padded shape the ring contraction uses
  if (!ctx->ring[0].batches.empty()) {
    const bool ring_lp = !f64;
    const long long kp = round_up(ov, lp_kpad(ctx, ov));
    const int fmt = lp_fmt_gemm(ctx, ov);
    const int S = std::min(8, ctx->ring[0].per_batch);
    const long long ulen = S * v2 * kp;
    const size_t mk = ws.mark();
    double* Z = ws.alloc((size_t)(S * ov3));
    void* U = ring_lp ? alloc_lp(ws, ulen) : (void*)ws.alloc((size_t)ulen);
    void* Al = ring_lp ? alloc_lp(ws, ov * kp) : (void*)ws.alloc((size_t)(ov * kp));
    if (!Z || !U || !Al) { ctx->err = "workspace exhausted (autotune)"; return CCT_ENOMEM; }
    // operand values only matter for timing: T3 data (in bounds of both), the ring matrix padded
    if (ring_lp) HIPCK(convert(ctx->t3, OutSpec{U, fmt, ulen}, std::min<long long>(ulen, ctx->ntri * ctx->v3), ctx->s));
    else HIPCK(fill((double*)U, 0.01, ulen, ctx->s));
    HIPCK(copy_pad_rows(ctx->Wb1, ov, ov, OutSpec{Al, fmt, ov * kp}, kp, ctx->s));
    const std::vector<int> ring_cands = !ring_lp ? std::vector<int>{9, 10, 1, 2, 3, 4}
                                        : (ctx->prec == Prec::BF16X3 ? std::vector<int>{5, 4, 1, 2, 3} : std::vector<int>{5, 1, 2, 3});
    ctx->tune_rings = pick(ring_cands, [&](int var) {
      if (ring_lp) {
        NtLpArgs g{};
        g.M = (int)ov; g.N = (int)v2; g.K = (int)kp; g.batch = S;
        g.A = Al; g.lda = kp; g.a_batch = 0; g.a_plane = ov * kp;
        g.B = U; g.ldb = kp; g.b_batch = v2 * kp; g.b_plane = ulen;
        g.C = Z; g.cm = idx1(v2); g.cn = idx1(1); g.c_batch = ov3; g.alpha = 1.0; g.beta = 0.0;
        g.a_len = ov * kp; g.b_len = ulen; g.c_len = S * ov3; g.variant = var;
        g.il = fmt == OUT_BF16X2I;
        return gemm_nt_lp(g, ctx->prec, ctx->s);
      }
      NtArgs g{};
      g.M = (int)ov; g.N = (int)v2; g.K = (int)kp; g.batch = S;
      g.A = (const double*)Al; g.lda = kp; g.a_batch = 0;
      g.B = (const double*)U; g.ldb = kp; g.b_batch = v2 * kp;
      g.C = Z; g.cm = idx1(v2); g.cn = idx1(1); g.c_batch = ov3; g.alpha = 1.0; g.beta = 0.0;
      g.a_len = ov * kp; g.b_len = ulen; g.c_len = S * ov3; g.variant = var;
      return gemm_nt(g, Prec::F64, ctx->s);
    });
    ws.reset(mk);
  }
  HIPCK(hipStreamSynchronize(ctx->s));
  auto m = read_tune_cache();
  m[tune_key(ctx, ladder_class(ctx))] = ctx->tune_ladder;
  m[tune_key(ctx, "rings")] = ctx->tune_rings;
  write_tune_cache(m);
  if (spent) *spent = used;
  return CCT_OK;
}

// --- fixed device scratch of the no-allocation (Q) entry point -------------
// One file-scope device array, one copy per GPU, held until the process ends.
// Its name is a host-side stand-in in host code: the device address of each
// GPU's copy is looked up once per device (with that device current) and kept;
// kernels and copies only ever receive that address.
constexpr size_t kQScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kQScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

int scratch_address(cct_ctx* ctx, void** out) {
  if (ctx->dev < 0 || ctx->dev >= kMaxDevices) {
    ctx->err = "scratch: device index out of range";
    return CCT_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[ctx->dev]) {
    int cur = 0;
    HIPCK(hipGetDevice(&cur));
    if (cur != ctx->dev) HIPCK(hipSetDevice(ctx->dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != ctx->dev) HIPCK(hipSetDevice(cur));
    if (e != hipSuccess || !p) {
      ctx->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return CCT_EDEVICE;
    }
    g_scratch_addr[ctx->dev] = p;
  }
  *out = g_scratch_addr[ctx->dev];
  return CCT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* cct_strerror(int code) {
  if (code > 0 || code < -6) return "unknown error";
  return kErr[-code];
}

const char* cct_last_error(const cct_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int64_t cct_packed_index(int nocc, int i, int j, int k) {
  if (nocc <= 0 || i < 0 || i > j || j > k || k >= nocc) return -1;
  // triples before first index i, then pairs (j,k) before j within i, then k offset
  const long long o = nocc;
  auto c3 = [](long long x) { return x * (x + 1) * (x + 2) / 6; };
  auto c2 = [](long long x) { return x * (x + 1) / 2; };
  const long long m = o - i;
  return c3(o) - c3(m) + c2(m) - c2(m - (j - i)) + (k - j);
}

void cct_destroy(cct_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->s);  // nothing in flight may touch what is freed below
  for (void* p : ctx->owned) dev_free(ctx, p);
  dev_free(ctx, ctx->wsbuf);
  for (int i = 0; i <= PH_N; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  for (hipEvent_t e : ctx->lad_ev) (void)hipEventDestroy(e);
  delete ctx;
}

int cct_create(int nocc, int nvir, int naux, cct_precision prec, const char* opts_json, cct_alloc_fn alloc,
               cct_free_fn free_fn, void* alloc_user, void* hip_stream, cct_ctx** out) {
  if (!out) return CCT_EINVAL;
  *out = nullptr;
  if (nocc < 1 || nvir < 1 || naux < 1 || nocc > 200 || nvir > 1200 || (int)prec < 0 || (int)prec > 2)
    return CCT_EINVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) return CCT_EINVAL;
  cct_ctx* ctx = new cct_ctx();
  ctx->alloc_fn = alloc;
  ctx->free_fn = free_fn;
  ctx->alloc_user = alloc_user;
  ctx->o = nocc;
  ctx->v = nvir;
  ctx->n = nocc + nvir;
  ctx->naux = naux;
  ctx->ntri = tri_count(nocc);
  ctx->v3 = (long long)nvir * nvir * nvir;
  ctx->prec = (Prec)prec;
  ctx->s = (hipStream_t)hip_stream;
  if (ctx->ntri > 65535) { delete ctx; return CCT_EINVAL; }
  if (opts_json) {
    std::string js(opts_json), val;
    if (json_find(js, "diis_space", val)) ctx->diis_space = std::atoi(val.c_str());
    if (json_find(js, "diis_start", val)) ctx->diis_start = std::atoi(val.c_str());
    if (json_find(js, "diis_t3", val)) {
      if (val == "none") ctx->diis_t3 = false;
      else if (val == "full") ctx->diis_t3 = true;
      else if (val.rfind("subspace:", 0) == 0 && val.size() > 9 &&
               val.find_first_not_of("0123456789", 9) == std::string::npos && val.size() < 15 &&
               std::atoi(val.c_str() + 9) >= 1 && std::atoi(val.c_str() + 9) <= nvir) {
        ctx->diis_t3 = true;
        ctx->diis_sv = std::atoi(val.c_str() + 9);
        if (ctx->diis_sv == nvir) ctx->diis_sv = 0;  // the whole block: plain T3 DIIS
      }
      else { delete ctx; return CCT_EINVAL; }
    }
    if (json_find(js, "diis", val)) ctx->diis_on = (val != "false" && val != "0" && val != "off");
    if (json_find(js, "workspace_gb", val)) ctx->ws_gb = std::atof(val.c_str());
    if (json_find(js, "timers", val)) ctx->events = (val == "true" || val == "1");
    if (json_find(js, "ladder_split", val)) ctx->ladder_split = (val == "true" || val == "1");
    if (json_find(js, "lp_block_k", val)) {
      ctx->lp_block_k = std::atoll(val.c_str());
      if (ctx->lp_block_k < 0) { delete ctx; return CCT_EINVAL; }
    }
    if (json_find(js, "tol", val)) {
      ctx->tol = std::atof(val.c_str());
      if (!(ctx->tol > 0)) { delete ctx; return CCT_EINVAL; }
    }
    if (ctx->diis_space < 0 || ctx->diis_space > DIIS_MAX || ctx->diis_start < 1 || ctx->ws_gb < 0) {
      delete ctx;
      return CCT_EINVAL;
    }
  }
  const int o = nocc, v = nvir, n = ctx->n;
  const long long n2 = (long long)n * n, n4 = n2 * n2;
  const long long ov = (long long)o * v, o2v2 = ov * ov, v3 = ctx->v3, t3n = ctx->ntri * v3;
  const long long o2v3 = (long long)o * o * v3;
  // memory plan (doubles)
  long long fixed = 3 * n2 + n + ov + 2 * o2v2 + (long long)naux * n2 * 2 + n4 + 2 * n2 + naux + (long long)naux * n * o;
  fixed += 2 * ov + 3 * o2v2 + 2 * t3n;                       // t1 t2 t3 r1 r2 r3 X2
  fixed += 2 * o2v2 + 2 * (long long)o * v * v * o + (long long)o * v * v * v + (long long)o * o * v * o;  // tau, VC*
  fixed += v * v + o * o + 2LL * o * o * o * o + 4 * o2v2 + 2 * (long long)v * v * v * o + (long long)v * o * o * o;
  fixed += (long long)v * v * v * v + o2v2 + ov;
  const int M = ctx->diis_on ? ctx->diis_space : 0;
  const long long dlen = ov + o2v2 + ctx->ntri * diis_block(ctx);
  fixed += (long long)(2 * M + 2) * dlen;
  // workspace: enough for every job in one batch (two unpacked/contracted
  // slabs per slot, o^2 slots for the rings), capped by the option
  // the split ladder needs W+- (about v^4/2) and, per packed block, its split
  // operands, pair products and one relabelled copy (about 3 v^3)
  const long long vp = (long long)v * (v + 1) / 2, ntri_l = (long long)o * (o + 1) * (o + 2) / 6;
  const long long lad_w = vp * (2 * vp + 16), lad_blk = (long long)v * (2 * vp + 16) + 2 * (long long)v * vp + v3;
  const long long ws_min =
      std::max(6 * (long long)o * v3 + 2 * o2v3, lad_w + 2 * lad_blk) + (1 << 22);
  const long long need_ws =
      std::max(6 * (long long)o * v3 + 2 * o2v3 * o, lad_w + ntri_l * lad_blk) + (1 << 22);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    ctx->err = "hipMemGetInfo failed (no HIP device?)";
    *out = nullptr;
    delete ctx;
    return CCT_EDEVICE;
  }
  {
    hipDevice_t d = 0;
    const hipError_t e = ctx->s ? hipStreamGetDevice(ctx->s, &d) : hipGetDevice(&d);
    if (e != hipSuccess) {
      delete ctx;
      return CCT_EDEVICE;
    }
    ctx->dev = (int)d;
  }
  // workspace: everything in one batch if it fits, else what is left of the
  // device after the fixed allocations (minus a margin), capped by the option
  const double margin = 2e9;
  const long long avail = (long long)(((double)free_b - (double)fixed * 8.0 - margin) / 8.0);
  long long ws_doubles = std::min<long long>(need_ws, avail);
  if (ctx->ws_gb > 0) ws_doubles = std::min<long long>(ws_doubles, (long long)(ctx->ws_gb * 1e9 / 8.0));
  ws_doubles = std::max<long long>(ws_doubles, ws_min);
  const double need_b = (double)(fixed + ws_doubles) * 8.0 + 64e6;
  if (need_b > (double)free_b) {
    delete ctx;
    return CCT_ENOMEM;
  }
  int rc = CCT_OK;
#define AL(ptr, cnt) if (rc == CCT_OK) rc = dalloc(ctx, &ctx->ptr, (cnt))
  AL(f, n2); AL(B, (long long)naux * n2); AL(eps, n); AL(fov, ov);
  AL(vbare_c, o2v2); AL(vbare, o2v2);
  AL(Bt, (long long)naux * n2); AL(ft, n2); AL(V, n4); AL(fG, n2); AL(G, n2); AL(cP, naux);
  AL(Dt, (long long)naux * n * o);
  AL(t1, ov); AL(t2, o2v2); AL(t3, t3n); AL(r1, ov); AL(r2, o2v2); AL(r3, t3n); AL(X2, o2v2); AL(zero_r1, ov);
  AL(tau2, o2v2); AL(VCoovv, o2v2); AL(VCovvo, (long long)o * v * v * o); AL(VCovvv, (long long)o * v * v * v);
  AL(VCoovo, (long long)o * o * v * o);
  AL(Fvv, (long long)v * v); AL(Foo, (long long)o * o); AL(Woooo, (long long)o * o * o * o);
  AL(Wh, (long long)o * o * o * o); AL(Wovvo, o2v2); AL(Wovov, o2v2);
  AL(Wt, (long long)v * v * v * o); AL(Wvooo, (long long)v * o * o * o); AL(Wb1, o2v2); AL(Wb2, o2v2);
  AL(Wvvvv, (long long)v * v * v * v); AL(tau_e, o2v2);
  AL(scal, 256);
  ctx->red_n = 1024 + 64LL * ctx->ntri + 1024;
  AL(red, ctx->red_n);
  ctx->diis_len = diis_len(ctx);
  if (M > 0) {
    const long long nchunk = diis_chunks(diis_args(ctx));
    AL(diis_old, ctx->diis_len);
    AL(diis_new, ctx->diis_len);
    AL(dvecs, (long long)M * ctx->diis_len);
    AL(derrs, (long long)M * ctx->diis_len);
    AL(diis_part, (long long)(M + 1) * nchunk);
    AL(diis_d, M + 1);
    AL(diis_B, (long long)M * M);
    AL(diis_coef, M);
    if (rc == CCT_OK) rc = dalloc_t(ctx, &ctx->diis_st, DIIS_STATE);
  }
#undef AL
  if (rc == CCT_OK) {
    void* w = nullptr;
    rc = dev_alloc(ctx, &w, (size_t)ws_doubles * 8);
    if (rc == CCT_OK) {
      ctx->wsbuf = (char*)w;
      ctx->ws.init(ctx->wsbuf, (size_t)ws_doubles * 8);
    }
  }
  if (rc == CCT_OK && ctx->events) {
    for (int i = 0; i <= PH_N && rc == CCT_OK; ++i)
      if (hipEventCreate(&ctx->ev[i]) != hipSuccess) rc = CCT_EDEVICE;
  }
  if (rc == CCT_OK) rc = build_plans(ctx);
  if (rc == CCT_OK) apply_tune_cache(ctx);
  if (rc == CCT_OK) {
    if (fill(ctx->zero_r1, 0.0, ov, ctx->s) != hipSuccess) rc = CCT_EDEVICE;
    if (fill(ctx->t1, 0.0, ov, ctx->s) != hipSuccess) rc = CCT_EDEVICE;
    if (fill(ctx->t2, 0.0, o2v2, ctx->s) != hipSuccess) rc = CCT_EDEVICE;
    if (fill(ctx->t3, 0.0, t3n, ctx->s) != hipSuccess) rc = CCT_EDEVICE;
    if (rc == CCT_OK && diis_reset(ctx) != CCT_OK) rc = CCT_EDEVICE;
    if (hipStreamSynchronize(ctx->s) != hipSuccess) rc = CCT_EDEVICE;
  }
  if (rc != CCT_OK) {
    cct_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return CCT_OK;
}

int cct_set_fock(cct_ctx* ctx, const double* f) {
  if (!ctx || !f) return CCT_EINVAL;
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  HIPCK(hipMemcpyAsync(ctx->f, f, (size_t)n * n * 8, hipMemcpyHostToDevice, ctx->s));
  std::vector<double> e(n), fo((size_t)o * v);
  for (int p = 0; p < n; ++p) e[p] = f[(size_t)p * n + p];
  for (int i = 0; i < o; ++i)
    for (int a = 0; a < v; ++a) fo[(size_t)i * v + a] = f[(size_t)i * n + o + a];
  HIPCK(hipMemcpyAsync(ctx->eps, e.data(), (size_t)n * 8, hipMemcpyHostToDevice, ctx->s));
  HIPCK(hipMemcpyAsync(ctx->fov, fo.data(), fo.size() * 8, hipMemcpyHostToDevice, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  ctx->have_f = true;
  return CCT_OK;
}

int cct_set_eri_df(cct_ctx* ctx, const double* B) {
  if (!ctx || !B) return CCT_EINVAL;
  const int n = ctx->n, o = ctx->o, v = ctx->v;
  const long long naux = ctx->naux;
  const long long n2 = (long long)n * n;
  HIPCK(hipMemcpyAsync(ctx->B, B, (size_t)naux * n2 * 8, hipMemcpyHostToDevice, ctx->s));
  // bare v^{ij}_{ab} = (ia|jb) = sum_P B[P][i][o+a] B[P][j][o+b], stored [i][j][a][b]
  GemmArgs g{};
  g.M = o * v; g.N = o * v; g.K = (int)naux; g.batch = 1;
  g.A = ctx->B + o; g.am = idx2(v, n, 1); g.ak = idx1(n2);
  g.B = ctx->B + o; g.bk = idx1(n2); g.bn = idx2(v, n, 1);
  // C[(i,a)][(j,b)] -> vbare[i][j][a][b]
  g.C = ctx->vbare; g.cm = idx2(v, (long long)o * v * v, v); g.cn = idx2(v, (long long)v * v, 1);
  g.alpha = 1.0; g.beta = 0.0;
  g.a_len = naux * n2 - o; g.b_len = naux * n2 - o; g.c_len = (long long)o * o * v * v;
  HIPCK(gemm(g, Prec::F64, ctx->s));
  DT vb = dense(ctx->vbare, {o, o, v, v}), vc = dense(ctx->vbare_c, {o, o, v, v});
  STCK(accumulate(ctx->s, 2.0, vb, "ijab", 0.0, vc, "ijab"));
  STCK(accumulate(ctx->s, -1.0, vb, "ijba", 1.0, vc, "ijab"));
  HIPCK(hipStreamSynchronize(ctx->s));
  ctx->have_B = true;
  return CCT_OK;
}

int cct_init_mp2(cct_ctx* ctx) {
  if (!ctx) return CCT_EINVAL;
  if (!ctx->have_f || !ctx->have_B) { ctx->err = "integrals not set"; return CCT_ESTATE; }
  const long long ov = (long long)ctx->o * ctx->v;
  HIPCK(fill(ctx->t1, 0.0, ov, ctx->s));
  HIPCK(fill(ctx->t2, 0.0, ov * ov, ctx->s));
  HIPCK(fill(ctx->t3, 0.0, ctx->ntri * ctx->v3, ctx->s));
  HIPCK(jacobi_t1t2(ctx->t1, ctx->zero_r1, ctx->t2, ctx->vbare, ctx->eps, ctx->o, ctx->v, ctx->s));
  RCK(diis_reset(ctx));
  HIPCK(hipStreamSynchronize(ctx->s));
  return CCT_OK;
}

int cct_set_amplitudes(cct_ctx* ctx, const double* t1, const double* t2, const double* t3p) {
  if (!ctx || !t1 || !t2) return CCT_EINVAL;
  const long long ov = (long long)ctx->o * ctx->v;
  HIPCK(hipMemcpyAsync(ctx->t1, t1, ov * 8, hipMemcpyHostToDevice, ctx->s));
  HIPCK(hipMemcpyAsync(ctx->t2, t2, ov * ov * 8, hipMemcpyHostToDevice, ctx->s));
  if (t3p) HIPCK(hipMemcpyAsync(ctx->t3, t3p, ctx->ntri * ctx->v3 * 8, hipMemcpyHostToDevice, ctx->s));
  else HIPCK(fill(ctx->t3, 0.0, ctx->ntri * ctx->v3, ctx->s));
  RCK(diis_reset(ctx));
  HIPCK(hipStreamSynchronize(ctx->s));
  return CCT_OK;
}

int cct_get_amplitudes(cct_ctx* ctx, double* t1, double* t2, double* t3p) {
  if (!ctx) return CCT_EINVAL;
  const long long ov = (long long)ctx->o * ctx->v;
  if (t1) HIPCK(hipMemcpyAsync(t1, ctx->t1, ov * 8, hipMemcpyDeviceToHost, ctx->s));
  if (t2) HIPCK(hipMemcpyAsync(t2, ctx->t2, ov * ov * 8, hipMemcpyDeviceToHost, ctx->s));
  if (t3p) HIPCK(hipMemcpyAsync(t3p, ctx->t3, ctx->ntri * ctx->v3 * 8, hipMemcpyDeviceToHost, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  return CCT_OK;
}

int cct_residual(cct_ctx* ctx, unsigned term_mask, double* r1, double* r2, double* r3p, double norms[3]) {
  if (!ctx) return CCT_EINVAL;
  if (term_mask & ~(unsigned)CCT_TERM_ALL) { ctx->err = "bad term mask"; return CCT_EINVAL; }
  double nr[3];
  int rc = compute(ctx, term_mask, false, nr);
  if (rc != CCT_OK && rc != CCT_ENUMERIC) return rc;
  const long long ov = (long long)ctx->o * ctx->v;
  if (r1) HIPCK(hipMemcpyAsync(r1, ctx->r1, ov * 8, hipMemcpyDeviceToHost, ctx->s));
  if (r2) HIPCK(hipMemcpyAsync(r2, ctx->r2, ov * ov * 8, hipMemcpyDeviceToHost, ctx->s));
  if (r3p) HIPCK(hipMemcpyAsync(r3p, ctx->r3, ctx->ntri * ctx->v3 * 8, hipMemcpyDeviceToHost, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  if (norms) for (int i = 0; i < 3; ++i) norms[i] = nr[i];
  return rc;
}

int cct_copy_r3(cct_ctx* ctx, int64_t first, int64_t count, double* out) {
  if (!ctx || !out || first < 0 || count < 0 || first + count > ctx->ntri * ctx->v3) return CCT_EINVAL;
  if (!ctx->have_res) { ctx->err = "no residual computed yet"; return CCT_ESTATE; }
  HIPCK(hipMemcpyAsync(out, ctx->r3 + first, (size_t)count * 8, hipMemcpyDeviceToHost, ctx->s));
  HIPCK(hipStreamSynchronize(ctx->s));
  return CCT_OK;
}

int cct_update(cct_ctx* ctx, double* e_corr, double norms[3]) {
  if (!ctx) return CCT_EINVAL;
  return update(ctx, e_corr, norms);
}

int cct_energy(cct_ctx* ctx, double* e_corr) {
  if (!ctx || !e_corr) return CCT_EINVAL;
  if (!ctx->have_f || !ctx->have_B) { ctx->err = "integrals not set"; return CCT_ESTATE; }
  return energy_dev(ctx, e_corr);
}

int cct_energy_q(cct_ctx* ctx, double* e_q, double* e_tasks, int64_t cap) {
  if (!ctx || !e_q || (e_tasks && cap < 0)) return CCT_EINVAL;
  if (!ctx->have_f || !ctx->have_B) { ctx->err = "integrals not set"; return CCT_ESTATE; }
  return energy_q(ctx, e_q, e_tasks, (long long)cap);
}

int cct_energy_q_noalloc(cct_ctx* ctx, double* e_q, double* e_tasks, int64_t cap) {
  if (!ctx || !e_q || (e_tasks && cap < 0)) return CCT_EINVAL;
  if (!ctx->have_f || !ctx->have_B) { ctx->err = "integrals not set"; return CCT_ESTATE; }
  void* region = nullptr;
  RCK(scratch_address(ctx, &region));
  return energy_q(ctx, e_q, e_tasks, (long long)cap, (char*)region, kQScratchBytes);
}

int64_t cct_q_task_count(int nocc) { return nocc < 0 ? -1 : (int64_t)q_task_count(nocc); }

int64_t cct_q_abc_task_count(int nvir, int block) {
  if (nvir < 1 || block < 1) return -1;
  return (int64_t)q_abc_task_count(nvir, block);
}

int cct_energy_q_abc(cct_ctx* ctx, int block, const int64_t* tasks, int64_t ntasks, double* e_q, double* e_tasks,
                     double* e_tuples, double stats[4]) {
  if (!ctx || !e_q || (tasks && ntasks < 0)) return CCT_EINVAL;
  if (!ctx->have_f || !ctx->have_B) { ctx->err = "integrals not set"; return CCT_ESTATE; }
  return energy_q_abc(ctx, block, tasks, tasks ? (long long)ntasks : 0, e_q, e_tasks, e_tuples, stats);
}

int cct_gather_t3(cct_ctx* ctx, const int64_t* idx, int64_t n, double* out) {
  if (!ctx || n < 0 || (n > 0 && (!idx || !out))) return CCT_EINVAL;
  const long long len = ctx->ntri * ctx->v3;
  for (int64_t i = 0; i < n; ++i)
    if (idx[i] < 0 || idx[i] >= len) {
      ctx->err = "gather_t3: index " + std::to_string(idx[i]) + " outside the packed T3";
      return CCT_EINVAL;
    }
  // chunks of indices through the workspace
  const size_t mark = ctx->ws.mark();
  const long long chunk = std::min<long long>(std::max<long long>(n, 1), 1LL << 24);
  long long* di = (long long*)ctx->ws.alloc((size_t)chunk);
  double* dv = ctx->ws.alloc((size_t)chunk);
  if (!di || !dv) {
    ctx->ws.reset(mark);
    ctx->err = "gather_t3: workspace exhausted";
    return CCT_ENOMEM;
  }
  int rc = CCT_OK;
  for (long long a = 0; a < n && rc == CCT_OK; a += chunk) {
    const long long m = std::min(chunk, (long long)n - a);
    if (hipMemcpyAsync(di, idx + a, sizeof(long long) * m, hipMemcpyHostToDevice, ctx->s) != hipSuccess ||
        gather_idx(ctx->t3, di, m, dv, ctx->s) != hipSuccess ||
        hipMemcpyAsync(out + a, dv, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->s) != hipSuccess ||
        hipStreamSynchronize(ctx->s) != hipSuccess)
      rc = CCT_EDEVICE;
  }
  ctx->ws.reset(mark);
  if (rc != CCT_OK) ctx->err = "gather_t3: device error";
  return rc;
}

int cct_solve(cct_ctx* ctx, int max_iter, double tol, double* e_corr, int* iters) {
  if (!ctx || max_iter < 1 || std::isnan(tol)) return CCT_EINVAL;
  if (!(tol > 0)) tol = ctx->tol;  // the context's default (option "tol")
  double e = 0.0, nr[3] = {0, 0, 0};
  for (int it = 1; it <= max_iter; ++it) {
    RCK(update(ctx, &e, nr));
    if (e_corr) *e_corr = e;
    if (iters) *iters = it;
    if (std::sqrt(nr[0] + nr[1] + nr[2]) < tol) return CCT_OK;
  }
  ctx->err = "not converged";
  return CCT_ENOTCONV;
}

int cct_autotune(cct_ctx* ctx, double budget_ms, int* variants) {
  if (!ctx || !(budget_ms >= 0.0)) return CCT_EINVAL;
  RCK(autotune(ctx, budget_ms, nullptr));
  if (variants) {
    variants[0] = ctx->tune_ladder;
    variants[1] = ctx->tune_rings;
  }
  return CCT_OK;
}

int cct_get_counters(cct_ctx* ctx, double* macs_by_term, double* ms_by_phase, int cap) {
  if (!ctx || cap < 0) return CCT_EINVAL;
  for (int i = 0; i < std::min(cap, 9); ++i) {
    if (macs_by_term) macs_by_term[i] = ctx->macs[i];
    if (ms_by_phase) ms_by_phase[i] = ctx->ms[i];
  }
  if (cap > 9) {
    if (macs_by_term) macs_by_term[9] = ctx->lad_macs;
    if (ms_by_phase) ms_by_phase[9] = ctx->lad_ms;
  }
  if (cap > 10) {
    if (macs_by_term) macs_by_term[10] = ctx->lad_launches;
    if (ms_by_phase) ms_by_phase[10] = 0.0;
  }
  // batch plan: how many batches each unpack-and-contract job takes with
  // this context's workspace, and the ladder's chunks of packed blocks
  const double plan[8] = {(double)ctx->feed1.batches.size(), (double)ctx->ring[0].batches.size(),
                          (double)ctx->ring[1].batches.size(), (double)ctx->ring[2].batches.size(),
                          (double)ctx->hh.batches.size(), (double)ctx->d1.batches.size(),
                          (double)ctx->d2.batches.size(), (double)ctx->lad_chunks};
  for (int i = 11; i < std::min(cap, 19); ++i) {
    if (macs_by_term) macs_by_term[i] = plan[i - 11];
    if (ms_by_phase) ms_by_phase[i] = 0.0;
  }
  return CCT_OK;
}

}  // extern "C"

// ===========================================================================
// Batches of independent systems
//
// Each system is an ordinary context.  One whole iteration of every system
// (amplitude save for DIIS, residual, T3 and T1/T2 Jacobi steps, DIIS on the
// device, energy) is recorded once into a HIP graph, forked over a few
// streams so that independent systems can overlap, and replayed once per
// iteration; each system's squared norms and energy land in one device
// array, read back with a single copy and synchronisation per replay.
// ===========================================================================
struct cct_batch {
  std::vector<cct_ctx*> sys;
  std::vector<hipStream_t> streams;  // streams[0] may be the caller's (owned_first false)
  bool owned_first = true;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
  double* dout = nullptr;  // [nsys][4]: |R1|^2, |R2|^2, |R3|^2, energy of the last iteration
  cct_alloc_fn alloc_fn = nullptr;
  cct_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  std::string err;
};

namespace {

int batch_enqueue_all(cct_batch* b) {
  for (size_t i = 0; i < b->sys.size(); ++i) {
    cct_ctx* c = b->sys[i];
    const int rc = enqueue_iteration(c, b->dout + 4 * i);
    if (rc != CCT_OK) {
      b->err = c->err;
      return rc;
    }
  }
  return CCT_OK;
}

// Record the device part of one iteration of every system into a graph.
int batch_capture(cct_batch* b) {
  hipStream_t s0 = b->streams[0];
  if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    b->err = "hipStreamBeginCapture failed";
    return CCT_EDEVICE;
  }
  int rc = CCT_OK;
  if (hipEventRecord(b->fork, s0) != hipSuccess) rc = CCT_EDEVICE;
  for (size_t i = 1; i < b->streams.size() && rc == CCT_OK; ++i)
    if (hipStreamWaitEvent(b->streams[i], b->fork, 0) != hipSuccess) rc = CCT_EDEVICE;
  if (rc == CCT_OK) rc = batch_enqueue_all(b);
  for (size_t i = 1; i < b->streams.size() && rc == CCT_OK; ++i) {
    if (hipEventRecord(b->join[i], b->streams[i]) != hipSuccess || hipStreamWaitEvent(s0, b->join[i], 0) != hipSuccess)
      rc = CCT_EDEVICE;
  }
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(s0, &g);
  if (rc == CCT_OK && ee != hipSuccess) {
    b->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ee);
    rc = CCT_EDEVICE;
  }
  if (rc != CCT_OK) {
    if (g) (void)hipGraphDestroy(g);
    if (b->err.empty()) b->err = "graph capture failed";
    return rc;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ie);
    return CCT_EDEVICE;
  }
  b->graph = g;
  b->exec = ex;
  return CCT_OK;
}

}  // namespace

extern "C" {

void cct_batch_destroy(cct_batch* b) {
  if (!b) return;
  for (hipStream_t s : b->streams)
    if (s) (void)hipStreamSynchronize(s);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (cct_ctx* c : b->sys) cct_destroy(c);
  if (b->dout) {
    if (b->free_fn) b->free_fn(b->dout, b->alloc_user);
    else (void)hipFree(b->dout);
  }
  for (hipEvent_t e : b->join)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (size_t i = 0; i < b->streams.size(); ++i)
    if (b->streams[i] && (i > 0 || b->owned_first)) (void)hipStreamDestroy(b->streams[i]);
  delete b;
}

int cct_batch_create(int nsys, const int* nocc, const int* nvir, const int* naux, cct_precision prec,
                     const char* opts_json, cct_alloc_fn alloc, cct_free_fn free_fn, void* alloc_user,
                     void* hip_stream, cct_batch** out) {
  if (!out) return CCT_EINVAL;
  *out = nullptr;
  if (nsys < 1 || nsys > 4096 || !nocc || !nvir || !naux) return CCT_EINVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) return CCT_EINVAL;
  int nstreams = 4;
  bool use_graph = true;
  std::string sys_opts = "{\"timers\": false";
  if (opts_json) {
    std::string js(opts_json), val;
    if (json_find(js, "streams", val)) nstreams = std::atoi(val.c_str());
    if (json_find(js, "graph", val)) use_graph = (val == "true" || val == "1");
    for (const char* key : {"diis_space", "diis_start", "diis", "workspace_gb", "ladder_split", "tol"})
      if (json_find(js, key, val)) sys_opts += std::string(", \"") + key + "\": " + val;
    if (json_find(js, "diis_t3", val)) sys_opts += ", \"diis_t3\": \"" + val + "\"";
  }
  sys_opts += "}";
  if (nstreams < 1 || nstreams > 16) return CCT_EINVAL;
  cct_batch* b = new cct_batch();
  b->use_graph = use_graph;
  b->alloc_fn = alloc;
  b->free_fn = free_fn;
  b->alloc_user = alloc_user;
  int rc = CCT_OK;
  {
    const size_t bytes = sizeof(double) * 4 * (size_t)nsys;
    void* p = nullptr;
    if (alloc) p = alloc(bytes, alloc_user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (!p) rc = CCT_ENOMEM;
    b->dout = (double*)p;
  }
  for (int i = 0; i < nstreams && rc == CCT_OK; ++i) {
    hipStream_t s = nullptr;
    if (i == 0 && hip_stream) {
      s = (hipStream_t)hip_stream;
      b->owned_first = false;
    } else if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      rc = CCT_EDEVICE;
    }
    b->streams.push_back(s);
    hipEvent_t e = nullptr;
    if (rc == CCT_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = CCT_EDEVICE;
    b->join.push_back(e);
  }
  if (rc == CCT_OK && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) rc = CCT_EDEVICE;
  // spread the systems over the streams by longest-processing-time-first on
  // the leading triples work (ladder 3 ntri v^5 + rings 12 ntri o v^4)
  std::vector<int> stream_of(nsys, 0);
  {
    std::vector<double> cost(nsys);
    for (int i = 0; i < nsys; ++i) {
      const double o = nocc[i], v = nvir[i], nt = o * (o + 1) * (o + 2) / 6.0;
      cost[i] = 3.0 * nt * std::pow(v, 5) + 12.0 * nt * o * std::pow(v, 4);
    }
    std::vector<int> order(nsys);
    for (int i = 0; i < nsys; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<double> load(nstreams, 0.0);
    for (int i : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      stream_of[i] = k;
      load[k] += cost[i];
    }
  }
  for (int i = 0; i < nsys && rc == CCT_OK; ++i) {
    cct_ctx* c = nullptr;
    rc = cct_create(nocc[i], nvir[i], naux[i], prec, sys_opts.c_str(), alloc, free_fn, alloc_user,
                    b->streams[stream_of[i]], &c);
    if (rc == CCT_OK) b->sys.push_back(c);
  }
  if (rc != CCT_OK) {
    cct_batch_destroy(b);
    return rc;
  }
  *out = b;
  return CCT_OK;
}

cct_ctx* cct_batch_system(cct_batch* b, int s) {
  if (!b || s < 0 || s >= (int)b->sys.size()) return nullptr;
  return b->sys[s];
}

int cct_batch_set_system(cct_batch* b, int s, const double* f, const double* B) {
  if (!b || s < 0 || s >= (int)b->sys.size()) return CCT_EINVAL;
  cct_ctx* c = b->sys[s];
  int rc = cct_set_fock(c, f);
  if (rc == CCT_OK) rc = cct_set_eri_df(c, B);
  if (rc == CCT_OK) rc = cct_init_mp2(c);
  if (rc != CCT_OK) b->err = c->err;
  return rc;
}

int cct_batch_iterate(cct_batch* b, int niter, double* e_corr, double* norms) {
  if (!b || niter < 0) return CCT_EINVAL;
  for (cct_ctx* c : b->sys)
    if (!c->have_f || !c->have_B) {
      b->err = "integrals not set for every system (cct_batch_set_system)";
      return CCT_ESTATE;
    }
  if (b->use_graph && !b->exec) RCK(batch_capture(b));
  const int ns = (int)b->sys.size();
  std::vector<double> h((size_t)4 * ns);
  for (int it = 0; it < niter; ++it) {
    if (b->use_graph) {
      const hipError_t e = hipGraphLaunch(b->exec, b->streams[0]);
      if (e != hipSuccess) {
        b->err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
        return CCT_EDEVICE;
      }
    } else {
      RCK(batch_enqueue_all(b));
      // the eager launches of the other streams join the first before the read-back
      for (size_t i = 1; i < b->streams.size(); ++i)
        if (hipEventRecord(b->join[i], b->streams[i]) != hipSuccess ||
            hipStreamWaitEvent(b->streams[0], b->join[i], 0) != hipSuccess) {
          b->err = "stream join failed";
          return CCT_EDEVICE;
        }
    }
    if (hipMemcpyAsync(h.data(), b->dout, sizeof(double) * h.size(), hipMemcpyDeviceToHost, b->streams[0]) !=
            hipSuccess ||
        hipStreamSynchronize(b->streams[0]) != hipSuccess) {
      b->err = "read-back after the batch iteration failed";
      return CCT_EDEVICE;
    }
    for (int s = 0; s < ns; ++s) {
      b->sys[s]->have_res = true;
      for (int k = 0; k < 4; ++k)
        if (!std::isfinite(h[4 * s + k])) {
          b->err = "system " + std::to_string(s) + ": non-finite residual norm or energy";
          b->sys[s]->err = "non-finite residual norm or energy";
          return CCT_ENUMERIC;
        }
      if (e_corr) e_corr[s] = h[4 * s + 3];
      if (norms)
        for (int k = 0; k < 3; ++k) norms[3 * s + k] = h[4 * s + k];
    }
  }
  return CCT_OK;
}

int cct_batch_autotune(cct_batch* b, double budget_ms) {
  if (!b || !(budget_ms >= 0.0)) return CCT_EINVAL;
  // one tuning per distinct size, shared by the systems of that size
  std::map<std::pair<int, int>, cct_ctx*> tuned;
  for (cct_ctx* c : b->sys) tuned[{c->o, c->v}] = nullptr;
  const double per = budget_ms / (double)tuned.size();
  for (cct_ctx* c : b->sys) {
    cct_ctx*& t = tuned[{c->o, c->v}];
    if (!t) {
      const int rc = autotune(c, per, nullptr);
      if (rc != CCT_OK) { b->err = c->err; return rc; }
      t = c;
    } else {
      c->tune_ladder = t->tune_ladder;
      c->tune_rings = t->tune_rings;
    }
  }
  // the recorded graph holds the old launches: record again on the next iterate
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return CCT_OK;
}

const char* cct_batch_last_error(const cct_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
