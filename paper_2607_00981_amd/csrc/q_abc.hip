// Perturbative quadruples in the virtual-tuple order (Sec. "ABC-based
// algorithm", Eq. ener-pt-q-abc with the intermediates of Eq. q_w_alter):
// the T3 transposition to virtual-triangular blocks, the gathers of T3
// slices for one virtual tile task, the Wbar builds, a segmented FP64
// matrix-core product whose output is the task's tuple-frame accumulators,
// and the per-tuple energy with the spin summation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace cct {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
constexpr int QBK = 16;

// Four-level map of an index below 2^31 (32-bit digit arithmetic).
__device__ __forceinline__ long long map4(const Idx4& d, int i) {
  const unsigned u = (unsigned)i;
  const unsigned d3 = u % (unsigned)d.n3, r3 = u / (unsigned)d.n3;
  const unsigned d2 = r3 % (unsigned)d.n2, r2 = r3 / (unsigned)d.n2;
  const unsigned d1 = r2 % (unsigned)d.n1, d0 = r2 / (unsigned)d.n1;
  return (long long)d0 * d.s0 + (long long)d1 * d.s1 + (long long)d2 * d.s2 + (long long)d3 * d.s3;
}

// blockIdx.x -> output tile; consecutive workgroups go to different XCDs
// (round-robin dispatch), so the tile order is strided by 8 and grouped by 8
// rows of tiles so that the tiles resident on one XCD share operand panels.
__device__ __forceinline__ bool q_tile(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int nb = tiles_m * tiles_n;
  const int per = (nb + 7) / 8;
  const int bid = blockIdx.x;
  const int pid = (bid % 8) * per + bid / 8;
  if (pid >= nb) return false;
  constexpr int GM = 8;
  const int group = pid / (GM * tiles_n);
  const int first_m = group * GM;
  const int gsize = min(tiles_m - first_m, GM);
  const int r = pid - group * GM * tiles_n;
  tm = first_m + r % gsize;
  tn = r / gsize;
  return true;
}

// Tile BM x BN = (16 TM WM) x (16 TN WN), WM x WN waves; K tiles of 16 over
// the concatenated segments; LDS double-buffered as [k][m] and [k][n].
// Each thread's load units keep their offsets inside the operand (set when a
// segment starts, advanced by one K tile per step), so the main loop does no
// index arithmetic beyond an add; the epilogue maps its rows and columns
// once.
template <int TM, int TN, int WM, int WN, bool AKM, bool BKN, bool VEC>
__global__ __launch_bounds__(64 * WM * WN) void qgemm_kernel(QGemmArgs g, int tiles_m, int tiles_n, int batch) {
  constexpr int NTH = 64 * WM * WN, BM = 16 * TM * WM, BN = 16 * TN * WN;
  constexpr int LA = BM + 2, LB = BN + 2;
  constexpr int W = VEC ? 2 : 1;
  constexpr int UA = BM * QBK / W, UB = BN * QBK / W;  // load units per K tile
  constexpr int NA = (UA + NTH - 1) / NTH, NB = (UB + NTH - 1) / NTH;
  __shared__ double As[2][QBK * LA];
  __shared__ double Bs[2][QBK * LB];
  int tm, tn;
  if (!q_tile(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x;
  int z = blockIdx.y * gridDim.z + blockIdx.z;
  if (z >= batch) return;
  int dig[QG_MAXD] = {0, 0, 0, 0};
  for (int d = g.nd - 1; d >= 0; --d) {
    dig[d] = z % g.rad[d];
    z /= g.rad[d];
  }
  const int m0 = tm * BM, n0 = tn * BN;
  // this thread's load units: position in the tile (row or column, k)
  int ar[NA], ak[NA], br[NB], bk[NB];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int u = tid + i * NTH;
    if constexpr (AKM) {
      ak[i] = u / (BM / W);
      ar[i] = (u % (BM / W)) * W;
    } else {
      ar[i] = u / (QBK / W);
      ak[i] = (u % (QBK / W)) * W;
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int u = tid + i * NTH;
    if constexpr (BKN) {
      bk[i] = u / (BN / W);
      br[i] = (u % (BN / W)) * W;
    } else {
      br[i] = u / (QBK / W);
      bk[i] = (u % (QBK / W)) * W;
    }
  }
  // segment state
  int seg = -1, seg_first = 0, seg_k = 0;
  const double* Ab = nullptr;
  const double* Bb = nullptr;
  long long aoff[NA], boff[NB], astep = 0, bstep = 0;
  int total = 0;
  for (int s = 0; s < g.nseg; ++s) total += (g.K[s] + QBK - 1) / QBK;
  auto enter = [&](int s) {
    seg = s;
    seg_k = g.K[s];
    long long ao = 0, bo = 0;
    for (int d = 0; d < g.nd; ++d) {
      ao += dig[d] * g.a[s].sd[d];
      bo += dig[d] * g.b[s].sd[d];
    }
    Ab = g.a[s].p + ao;
    Bb = g.b[s].p + bo;
    const long long lda = g.a[s].ld, ldb = g.b[s].ld;
    astep = AKM ? QBK * lda : QBK;
    bstep = BKN ? QBK * ldb : QBK;
#pragma unroll
    for (int i = 0; i < NA; ++i)
      aoff[i] = AKM ? (long long)ak[i] * lda + (m0 + ar[i]) : (long long)(m0 + ar[i]) * lda + ak[i];
#pragma unroll
    for (int i = 0; i < NB; ++i)
      boff[i] = BKN ? (long long)bk[i] * ldb + (n0 + br[i]) : (long long)(n0 + br[i]) * ldb + bk[i];
  };
  dbl2 ra[NA], rb[NB];
  bool oa[NA], ob[NB];
  int kt_in_seg = 0;  // K tile index inside the current segment
  auto load = [&](int t) {
    // t runs over the concatenated K tiles; move to the segment holding it
    if (seg < 0 || t - seg_first >= (seg_k + QBK - 1) / QBK) {
      int s = seg < 0 ? 0 : seg + 1, first = seg < 0 ? 0 : seg_first + (seg_k + QBK - 1) / QBK;
      while (s + 1 < g.nseg && t - first >= (g.K[s] + QBK - 1) / QBK) first += (g.K[s++] + QBK - 1) / QBK;
      seg_first = first;
      enter(s);
    }
    kt_in_seg = t - seg_first;
    const int k0 = kt_in_seg * QBK;
    const long long ash = kt_in_seg * astep, bsh = kt_in_seg * bstep;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      oa[i] = (tid + i * NTH) < UA && m0 + ar[i] < g.M && k0 + ak[i] < seg_k;
      const double* p = Ab + (oa[i] ? aoff[i] + ash : 0);
      if constexpr (VEC) ra[i] = *(const dbl2*)p;
      else ra[i].x = *p;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      ob[i] = (tid + i * NTH) < UB && n0 + br[i] < g.N && k0 + bk[i] < seg_k;
      const double* p = Bb + (ob[i] ? boff[i] + bsh : 0);
      if constexpr (VEC) rb[i] = *(const dbl2*)p;
      else rb[i].x = *p;
    }
  };
  auto store = [&](double* as, double* bs) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (tid + i * NTH >= UA) continue;
      if constexpr (AKM) {
        as[ak[i] * LA + ar[i]] = oa[i] ? ra[i].x : 0.0;
        if constexpr (VEC) as[ak[i] * LA + ar[i] + 1] = oa[i] ? ra[i].y : 0.0;
      } else {
        as[ak[i] * LA + ar[i]] = oa[i] ? ra[i].x : 0.0;
        if constexpr (VEC) as[(ak[i] + 1) * LA + ar[i]] = oa[i] ? ra[i].y : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (tid + i * NTH >= UB) continue;
      if constexpr (BKN) {
        bs[bk[i] * LB + br[i]] = ob[i] ? rb[i].x : 0.0;
        if constexpr (VEC) bs[bk[i] * LB + br[i] + 1] = ob[i] ? rb[i].y : 0.0;
      } else {
        bs[bk[i] * LB + br[i]] = ob[i] ? rb[i].x : 0.0;
        if constexpr (VEC) bs[(bk[i] + 1) * LB + br[i]] = ob[i] ? rb[i].y : 0.0;
      }
    }
  };

  const int wave = tid / 64, lane = tid & 63;
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (total > 0) {
    load(0);
    store(As[0], Bs[0]);
  }
  // output rows and columns of this lane
  long long coff = 0;
  for (int d = 0; d < g.nd; ++d) coff += dig[d] * g.sc[d];
  long long cof[TN];
  bool cin[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn0 + j * 16 + (lane & 15);
    cin[j] = n < g.N;
    cof[j] = cin[j] ? map4(g.cn, n) : 0;
  }
  double* rowp[TM][4];
  bool rin[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm0 + i * 16 + 4 * r + lane / 16;
      rin[i][r] = m < g.M;
      rowp[i][r] = g.C + coff + (rin[i][r] ? map4(g.cm, m) : 0);
    }
  __syncthreads();
  for (int t = 0; t < total; ++t) {
    const int cur = t & 1;
    if (t + 1 < total) load(t + 1);
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int ks = 0; ks < QBK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = as[kr * LA + wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = bs[kr * LB + wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (t + 1 < total) store(As[cur ^ 1], Bs[cur ^ 1]);
    __syncthreads();
  }
  // accumulator register r of lane l: row 4r + l/16, column l%16; per
  // group of 16 rows every load of C is issued before any store
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    double cur[4][TN];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < TN; ++j) cur[r][j] = (g.accumulate && rin[i][r] && cin[j]) ? rowp[i][r][cof[j]] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        if (rin[i][r] && cin[j]) rowp[i][r][cof[j]] = cur[r][j] + g.alpha * acc[i][j][r];
  }
}

template <int TM, int TN, int WM, int WN, bool AKM, bool BKN, bool VEC>
hipError_t qlaunch(const QGemmArgs& g, long long batch, hipStream_t s) {
  constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN;
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long gx = ((nb + 7) / 8) * 8;
  if (gx > INT_MAX) return hipErrorInvalidValue;
  // the batch over grid z (at most 65535) and y
  const long long gz = std::min<long long>(batch, 65535), gy = (batch + gz - 1) / gz;
  hipLaunchKernelGGL((qgemm_kernel<TM, TN, WM, WN, AKM, BKN, VEC>), dim3((unsigned)gx, (unsigned)gy, (unsigned)gz),
                     dim3(64 * WM * WN), 0, s, g, tiles_m, tiles_n, (int)batch);
  return hipGetLastError();
}

template <bool AKM, bool BKN, bool VEC>
hipError_t qdispatch(int cfg, const QGemmArgs& g, long long batch, hipStream_t s) {
  switch (cfg) {
    case 0: return qlaunch<5, 2, 1, 8, AKM, BKN, VEC>(g, batch, s);   // 80 x 256, 8 waves
    case 1: return qlaunch<2, 5, 8, 1, AKM, BKN, VEC>(g, batch, s);   // 256 x 80, 8 waves
    case 2: return qlaunch<2, 4, 4, 2, AKM, BKN, VEC>(g, batch, s);   // 128 x 128, 8 waves
    case 3: return qlaunch<5, 3, 2, 2, AKM, BKN, VEC>(g, batch, s);   // 160 x 96
    case 4: return qlaunch<3, 5, 2, 2, AKM, BKN, VEC>(g, batch, s);   // 96 x 160
    case 5: return qlaunch<4, 4, 2, 4, AKM, BKN, VEC>(g, batch, s);   // 128 x 256, 8 waves
    case 6: return qlaunch<4, 4, 4, 2, AKM, BKN, VEC>(g, batch, s);   // 256 x 128, 8 waves
    default: return qlaunch<2, 2, 2, 2, AKM, BKN, VEC>(g, batch, s);  // 64 x 64
  }
}

constexpr int QCFG_N = 8;
constexpr int QCFG_BM[QCFG_N] = {80, 256, 128, 160, 96, 128, 256, 64};
constexpr int QCFG_BN[QCFG_N] = {256, 80, 128, 96, 160, 256, 128, 64};

// Tile choice: the best operand reuse (BM BN / (BM + BN)) weighted by the
// square of the useful fraction of the padded output (padding costs both
// matrix-core time and the loads that feed it).
int qpick(int M, int N) {
  int best = QCFG_N - 1;
  double best_score = -1.0;
  for (int c = 0; c < QCFG_N; ++c) {
    const double bm = QCFG_BM[c], bn = QCFG_BN[c];
    const double padded = std::ceil(M / bm) * bm * std::ceil(N / bn) * bn;
    const double useful = (double)M * N / padded;
    const double reuse = bm * bn / (bm + bn);
    const double score = useful * useful * reuse;
    if (score > best_score) {
      best_score = score;
      best = c;
    }
  }
  return best;
}

__device__ __forceinline__ long long c3(long long n) { return n * (n - 1) * (n - 2) / 6; }
__device__ __forceinline__ long long c2(long long n) { return n * (n - 1) / 2; }
// Position of the virtual triple a <= b <= c among all such triples of [0, v)
// in lexicographic order: the triples with a smaller first label, then the
// pairs (b', c') >= (a, a) before (b, c), then c - b.
__device__ __forceinline__ long long vtri(int a, int b, int c, int v) {
  const long long m = v - a;
  return (c3(v + 2) - c3(m + 2)) + (c2(m + 1) - c2(m - (b - a) + 1)) + (c - b);
}

// Tiled transposition: a workgroup takes one cube of 16^3 virtual labels
// (cube indices A <= B <= C) and QC consecutive ordered occupied triples q.
// For each q the cube is read along the stored axis of unit stride (runs of
// 16 doubles), staged in LDS, and every canonical a <= b <= c of the cube is
// written at its QC consecutive q.  Work items are dealt to the XCDs in
// contiguous ranges, so the partial lines that neighbouring q chunks of one
// cube write meet in the same L2.
constexpr int TQ_CT = 16, TQ_QC = 2;
__global__ __launch_bounds__(256) void t3v_transpose_kernel(const double* __restrict__ T,
                                                            const BlockRef* __restrict__ tbl,
                                                            double* __restrict__ T3v,
                                                            const int4* __restrict__ cubes, long long nwork,
                                                            int nqc, int o, int v) {
  __shared__ double lds[TQ_QC][TQ_CT * TQ_CT * TQ_CT];
  const long long per = (nwork + 7) / 8;
  const long long w = (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (w >= nwork) return;
  const int4 cb = cubes[w / nqc];
  const int qc = (int)(w % nqc);
  const long long o3 = (long long)o * o * o;
  const int a0 = cb.x * TQ_CT, b0 = cb.y * TQ_CT, c0 = cb.z * TQ_CT;
  const int na = min(TQ_CT, v - a0), nb = min(TQ_CT, v - b0), nc = min(TQ_CT, v - c0);
  for (int qq = 0; qq < TQ_QC; ++qq) {
    const long long q = (long long)qc * TQ_QC + qq;
    if (q >= o3) break;
    const BlockRef r = tbl[q];
    // local axis order: the label whose stored stride is 1 varies fastest
    const int fast = r.s[0] == 1 ? 0 : (r.s[1] == 1 ? 1 : 2);
    const int s1 = fast == 0 ? 1 : 0, s2 = fast == 2 ? 1 : 2;  // the other two, in order
    const int n3[3] = {na, nb, nc}, o3l[3] = {a0, b0, c0};
    for (int e = threadIdx.x; e < TQ_CT * TQ_CT * TQ_CT; e += blockDim.x) {
      int l[3];
      l[fast] = e % TQ_CT;
      l[s2] = (e / TQ_CT) % TQ_CT;
      l[s1] = e / (TQ_CT * TQ_CT);
      double x = 0.0;
      if (l[0] < n3[0] && l[1] < n3[1] && l[2] < n3[2])
        x = T[r.off + (long long)(o3l[0] + l[0]) * r.s[0] + (long long)(o3l[1] + l[1]) * r.s[1] +
              (long long)(o3l[2] + l[2]) * r.s[2]];
      lds[qq][(l[0] * TQ_CT + l[1]) * TQ_CT + l[2]] = x;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TQ_CT * TQ_CT * TQ_CT * TQ_QC; e += blockDim.x) {
    const int qq = e % TQ_QC, t = e / TQ_QC;
    const int la = t / (TQ_CT * TQ_CT), lb = (t / TQ_CT) % TQ_CT, lc = t % TQ_CT;
    const int a = a0 + la, b = b0 + lb, c = c0 + lc;
    const long long q = (long long)qc * TQ_QC + qq;
    if (la >= na || lb >= nb || lc >= nc || a > b || b > c || q >= o3) continue;
    T3v[vtri(a, b, c, v) * o3 + q] = lds[qq][t];
  }
}

// One workgroup per output block (label digits, e): the column pairs are
// ordered by virtual label once, which fixes the source block and the
// stride of each output axis inside it; the threads then copy the o^3
// block (reads stay inside one 8 o^3-byte block of T3v).
__global__ __launch_bounds__(256) void t3v_gather_kernel(const double* __restrict__ T3v, double* __restrict__ out,
                                                         T3Gather g) {
  const long long o3 = (long long)g.o * g.o * g.o;
  const int e = (int)(blockIdx.x % g.ne);
  long long r = blockIdx.x / g.ne;
  int dig[3] = {0, 0, 0};
  for (int d = g.nd - 1; d >= 0; --d) {
    dig[d] = (int)(r % g.rad[d]);
    r /= g.rad[d];
  }
  int lab[3], ax[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lab[c] = g.lab[c] == 3 ? e : g.st[g.lab[c]] + dig[g.lab[c]];
    ax[c] = g.ax[c];
  }
  // order the column pairs by virtual label (ties: equal values by column symmetry)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2 - i; ++j)
      if (lab[j] > lab[j + 1]) {
        const int tl = lab[j], ta = ax[j];
        lab[j] = lab[j + 1];
        ax[j] = ax[j + 1];
        lab[j + 1] = tl;
        ax[j + 1] = ta;
      }
  // sorted position k of the source block holds the occupied index of output axis ax[k]
  long long st[3];
  st[ax[0]] = (long long)g.o * g.o;
  st[ax[1]] = g.o;
  st[ax[2]] = 1;
  const double* src = T3v + vtri(lab[0], lab[1], lab[2], g.v) * o3;
  double* dst = out + (long long)blockIdx.x * o3;
  const int o = g.o, o2 = o * o;
  for (int q = threadIdx.x; q < (int)o3; q += blockDim.x)
    dst[q] = src[(q / o2) * st[0] + ((q / o) % o) * st[1] + (q % o) * st[2]];
}

// Wbar_{ijk}^{xym} (alternative form) = -1/2 sum_n (v^{mn}_{ki} t_{nj}^{xy} + v^{mn}_{kj} t_{ni}^{yx})
// for x = x0 + lx, y = y0 + ly; element [lx][ly][rows][m] with the row index
// holding i, j, k at the positions rowpos[0..2].  VT[n][k][i][m] = v^{mn}_{ki}
// (m fastest, as the output).
__global__ __launch_bounds__(256) void q_wo_kernel(double* __restrict__ out, const double* __restrict__ VT,
                                                   const double* __restrict__ t2, int o, int v, int x0, int nx,
                                                   int y0, int ny, int p0, int p1, int p2, long long total) {
  const long long vv = (long long)v * v;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(idx % o);
    long long r = idx / o;
    int w[3];
    w[2] = (int)(r % o);
    r /= o;
    w[1] = (int)(r % o);
    r /= o;
    w[0] = (int)(r % o);
    r /= o;
    const int ly = (int)(r % ny), lx = (int)(r / ny);
    const int i = w[p0], j = w[p1], k = w[p2];
    const int x = x0 + lx, y = y0 + ly;
    double s = 0.0;
    for (int n = 0; n < o; ++n) {
      const double* vr = VT + ((long long)n * o + k) * o * o + m;
      s += vr[(long long)i * o] * t2[((long long)n * o + j) * vv + (long long)x * v + y] +
           vr[(long long)j * o] * t2[((long long)n * o + i) * vv + (long long)y * v + x];
    }
    out[idx] = -0.5 * s;
  }
}

// Wbar_{ejk}^{xyz} in two passes for o <= QW_OMAX: pass A writes the two
// Z terms and the two K = o terms that do not involve k (v^{my}_{ej},
// v^{mx}_{je} held in registers across the k loop); pass B adds the two that
// do not involve j (v^{mz}_{ek}, v^{mx}_{ke} held across the j loop).  One
// workgroup per (lx, ly, lz, j) (pass A) or (lx, ly, lz, k) (pass B), the
// threads over e; the T2 factors of the workgroup's labels are staged in LDS
// and read as broadcasts.
constexpr int QW_OMAX = 32;
__global__ __launch_bounds__(256) void q_wv_a_kernel(double* __restrict__ out, const double* __restrict__ Zxy,
                                                     const double* __restrict__ Zxz, const double* __restrict__ Vmyje,
                                                     const double* __restrict__ Vmxje, const double* __restrict__ t2,
                                                     int o, int v, int x0, int ny, int y0, int nz, int z0) {
  __shared__ double ta[QW_OMAX * QW_OMAX], tb[QW_OMAX * QW_OMAX];
  const long long ov = (long long)o * v, vv = (long long)v * v, o2v = (long long)o * ov;
  int r = blockIdx.x;
  const int j = r % o;
  r /= o;
  const int lz = r % nz;
  r /= nz;
  const int ly = r % ny, lx = r / ny;
  const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
  for (int q = threadIdx.x; q < o * o; q += blockDim.x) {  // [m][k]
    const long long row = (long long)q * vv;               // (m o + k) vv
    ta[q] = t2[row + (long long)x * v + z];
    tb[q] = t2[row + (long long)y * v + z];
  }
  __syncthreads();
  const long long bxy = (((long long)lx * ny + ly) * nz + lz) * o2v, bxz = (((long long)lx * nz + lz) * ny + ly) * o2v;
  for (int e = threadIdx.x; e < v; e += blockDim.x) {
    double u1[QW_OMAX], u2[QW_OMAX];
#pragma unroll
    for (int m = 0; m < QW_OMAX; ++m) {
      u1[m] = m < o ? Vmyje[((long long)m * v + y) * ov + (long long)j * v + e] : 0.0;
      u2[m] = m < o ? Vmxje[((long long)m * v + x) * ov + (long long)j * v + e] : 0.0;
    }
    for (int k = 0; k < o; ++k) {
      double s = Zxy[bxy + ((long long)j * o + k) * v + e] + Zxz[bxz + ((long long)k * o + j) * v + e];
#pragma unroll
      for (int m = 0; m < QW_OMAX; ++m)
        if (m < o) s -= u1[m] * ta[m * o + k] + u2[m] * tb[m * o + k];
      out[bxy + ((long long)j * o + k) * v + e] = s;
    }
  }
}

__global__ __launch_bounds__(256) void q_wv_b_kernel(double* __restrict__ out, const double* __restrict__ Vmyje,
                                                     const double* __restrict__ Vmxje, const double* __restrict__ t2,
                                                     int o, int v, int x0, int ny, int y0, int nz, int z0) {
  __shared__ double ta[QW_OMAX * QW_OMAX], tb[QW_OMAX * QW_OMAX];
  const long long ov = (long long)o * v, vv = (long long)v * v, o2v = (long long)o * ov;
  int r = blockIdx.x;
  const int k = r % o;
  r /= o;
  const int lz = r % nz;
  r /= nz;
  const int ly = r % ny, lx = r / ny;
  const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
  for (int q = threadIdx.x; q < o * o; q += blockDim.x) {  // [m][j]
    const long long row = (long long)q * vv;
    ta[q] = t2[row + (long long)x * v + y];
    tb[q] = t2[row + (long long)z * v + y];
  }
  __syncthreads();
  const long long b = (((long long)lx * ny + ly) * nz + lz) * o2v;
  for (int e = threadIdx.x; e < v; e += blockDim.x) {
    double w1[QW_OMAX], w2[QW_OMAX];
#pragma unroll
    for (int m = 0; m < QW_OMAX; ++m) {
      w1[m] = m < o ? Vmyje[((long long)m * v + z) * ov + (long long)k * v + e] : 0.0;
      w2[m] = m < o ? Vmxje[((long long)m * v + x) * ov + (long long)k * v + e] : 0.0;
    }
    for (int j = 0; j < o; ++j) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < QW_OMAX; ++m)
        if (m < o) s += w1[m] * ta[m * o + j] + w2[m] * tb[m * o + j];
      out[b + ((long long)j * o + k) * v + e] -= s;
    }
  }
}

// Wbar_{ejk}^{xyz} (alternative form) as [lx][ly][lz][j][k][e].
__global__ __launch_bounds__(256) void q_wv_kernel(double* __restrict__ out, const double* __restrict__ Zxy,
                                                   const double* __restrict__ Zxz, const double* __restrict__ Vmyje,
                                                   const double* __restrict__ Vmxje, const double* __restrict__ t2,
                                                   int o, int v, int x0, int nx, int y0, int ny, int z0, int nz,
                                                   long long total) {
  const long long ov = (long long)o * v, vv = (long long)v * v, o2v = (long long)o * ov;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const int e = (int)(idx % v);
    long long r = idx / v;
    const int k = (int)(r % o);
    r /= o;
    const int j = (int)(r % o);
    r /= o;
    const int lz = (int)(r % nz);
    r /= nz;
    const int ly = (int)(r % ny);
    const int lx = (int)(r / ny);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    // Z_xy[z] at [lx][ly][lz][j][k][e]; Z_xz[y] at [lx][lz][ly][k][j][e]
    double s = Zxy[(((long long)lx * ny + ly) * nz + lz) * o2v + ((long long)j * o + k) * v + e] +
               Zxz[(((long long)lx * nz + lz) * ny + ly) * o2v + ((long long)k * o + j) * v + e];
    for (int m = 0; m < o; ++m) {
      const long long tm = (long long)m * o;
      s -= Vmyje[((long long)m * v + y) * ov + (long long)j * v + e] * t2[(tm + k) * vv + (long long)x * v + z];
      s -= Vmxje[((long long)m * v + x) * ov + (long long)j * v + e] * t2[(tm + k) * vv + (long long)y * v + z];
      s -= Vmyje[((long long)m * v + z) * ov + (long long)k * v + e] * t2[(tm + j) * vv + (long long)x * v + y];
      s -= Vmxje[((long long)m * v + x) * ov + (long long)k * v + e] * t2[(tm + j) * vv + (long long)z * v + y];
    }
    out[idx] = s;
  }
}

// The spin summation 2 (2 - P_cd)(2 - P_bc - P_bd)(2 - P_ab - P_ac - P_ad),
// multiplied out, is a class function of the permutation group: 16 on the
// identity, -8 on transpositions, 4 on three-cycles and on double
// transpositions, -2 on four-cycles.
struct QPerms {
  int p[24][4];
  double c[24];
  int w[24][4];  // in-block offset of the permuted element: sum_m j_m w[p][m]
};

// The occupied index space o^4 is cut into blocks of bs^4 (bs <= 5, nbk
// blocks per axis); the axis permutations act on whole blocks, so each orbit
// of blocks (at most 24) is closed under them.  One workgroup takes one
// tuple and one orbit: it stages R = X + Y on the orbit's blocks in LDS (each
// element of X and Y read once) and evaluates U = S(R) / den there, so the 24
// permuted reads of the spin summation are LDS reads.
constexpr int QE_BS = 4, QE_MAXB = 24;
__global__ __launch_bounds__(256) void q_abc_energy_kernel(const double* __restrict__ X, const double* __restrict__ Y,
                                                           const double* __restrict__ Vvvoo,
                                                           const double* __restrict__ t2R,
                                                           const double* __restrict__ eps, QSlots sl, QPerms P,
                                                           const int* __restrict__ orbits, int norb, int bs, int o,
                                                           int v, double* __restrict__ part) {
  __shared__ double Rl[QE_MAXB * QE_BS * QE_BS * QE_BS * QE_BS];
  __shared__ double red[256];
  __shared__ unsigned char smap[QE_MAXB][24];  // slot of block(slot) o pi
  __shared__ int btab[QE_MAXB];
  const int orb = blockIdx.x % norb;
  const int tau = blockIdx.x / norb;
  int lab[4];
  {
    int r = tau;
    for (int s = 3; s >= 0; --s) {
      lab[s] = sl.st[s] + r % sl.n[s];
      r /= sl.n[s];
    }
  }
  const bool canon = lab[0] <= lab[1] && lab[1] <= lab[2] && lab[2] <= lab[3] &&
                     !(lab[0] == lab[1] && lab[1] == lab[2]) && !(lab[1] == lab[2] && lab[2] == lab[3]);
  if (!canon) {
    if (threadIdx.x == 0) part[blockIdx.x] = 0.0;
    return;
  }
  const int* ob = orbits + orb * (QE_MAXB + 1);
  const int nblk = ob[0];
  if ((int)threadIdx.x < nblk) btab[threadIdx.x] = ob[1 + threadIdx.x];
  __syncthreads();
  for (int e = threadIdx.x; e < nblk * 24; e += blockDim.x) {
    const int sidx = e / 24, p = e % 24;
    const int b = btab[sidx];
    const int d[4] = {b & 255, (b >> 8) & 255, (b >> 16) & 255, (b >> 24) & 255};
    const int t = d[P.p[p][0]] | (d[P.p[p][1]] << 8) | (d[P.p[p][2]] << 16) | (d[P.p[p][3]] << 24);
    int k = 0;
    while (k < nblk && btab[k] != t) ++k;
    smap[sidx][p] = (unsigned char)k;
  }
  const long long o2 = (long long)o * o, o4 = o2 * o2;
  const double* x = X + (long long)tau * o4;
  const double* yy = Y + (long long)tau * o4;
  const int bs2 = bs * bs, bs4 = bs2 * bs2;
  for (int e = threadIdx.x; e < nblk * bs4; e += blockDim.x) {
    const int sidx = e / bs4, w = e % bs4;
    const int b = btab[sidx];
    const int i0 = (b & 255) * bs + w / (bs2 * bs), i1 = ((b >> 8) & 255) * bs + (w / bs2) % bs;
    const int i2 = ((b >> 16) & 255) * bs + (w / bs) % bs, i3 = ((b >> 24) & 255) * bs + w % bs;
    const long long at = ((long long)i0 * o + i1) * o2 + (long long)i2 * o + i3;
    Rl[e] = (i0 < o && i1 < o && i2 < o && i3 < o) ? x[at] + yy[at] : 0.0;
  }
  __syncthreads();
  const double ev = eps[o + lab[0]] + eps[o + lab[1]] + eps[o + lab[2]] + eps[o + lab[3]];
  double acc = 0.0;
  for (int e = threadIdx.x; e < nblk * bs4; e += blockDim.x) {
    const int sidx = e / bs4, w = e % bs4;
    const int b = btab[sidx];
    const int j[4] = {w / (bs2 * bs), (w / bs2) % bs, (w / bs) % bs, w % bs};
    const int i[4] = {(b & 255) * bs + j[0], ((b >> 8) & 255) * bs + j[1], ((b >> 16) & 255) * bs + j[2],
                      ((b >> 24) & 255) * bs + j[3]};
    if (i[0] >= o || i[1] >= o || i[2] >= o || i[3] >= o) continue;
    double u = 0.0;
#pragma unroll 4
    for (int p = 0; p < 24; ++p) {
      const int jj = j[0] * P.w[p][0] + j[1] * P.w[p][1] + j[2] * P.w[p][2] + j[3] * P.w[p][3];
      u += P.c[p] * Rl[smap[sidx][p] * bs4 + jj];
    }
    const double den = eps[i[0]] + eps[i[1]] + eps[i[2]] + eps[i[3]] - ev;
    // sum over the six splits {s0 < s1} | {s2 < s3} of v^{..}_{..} t_{..}^{..}
    double vs = 0.0;
#pragma unroll
    for (int s0 = 0; s0 < 4; ++s0)
#pragma unroll
      for (int s1 = s0 + 1; s1 < 4; ++s1) {
        int s2 = -1, s3 = -1;
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (t != s0 && t != s1) {
            if (s2 < 0) s2 = t;
            else s3 = t;
          }
        vs += Vvvoo[((long long)lab[s0] * v + lab[s1]) * o2 + (long long)i[s0] * o + i[s1]] *
              t2R[((long long)lab[s3] * v + lab[s2]) * o2 + (long long)i[s2] * o + i[s3]];
      }
    acc += (x[((long long)i[0] * o + i[1]) * o2 + (long long)i[2] * o + i[3]] + vs) * (u / den);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// etup[tau] = (sum of the tuple's chunk partials) / |Stab(tau)|; etask = sum
// over tau in order (one workgroup, fixed order).
__global__ __launch_bounds__(256) void q_abc_reduce_kernel(const double* __restrict__ part, QSlots sl, int ntau,
                                                           int nchunk, double* __restrict__ etup,
                                                           double* __restrict__ etask) {
  __shared__ double red[256];
  double tot = 0.0;
  for (int tau = threadIdx.x; tau < ntau; tau += blockDim.x) {
    int lab[4];
    int r = tau;
    for (int s = 3; s >= 0; --s) {
      lab[s] = sl.st[s] + r % sl.n[s];
      r /= sl.n[s];
    }
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)tau * nchunk + c];
    // |Stab|: the product of the factorials of the label multiplicities
    int stab = 1, run = 1;
    for (int k = 1; k < 4; ++k) {
      run = lab[k] == lab[k - 1] ? run + 1 : 1;
      stab *= run;
    }
    const double e = s / stab;
    if (etup) etup[tau] = e;
    tot += e;
  }
  red[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *etask = red[0];
}

__global__ __launch_bounds__(256) void gather_idx_kernel(const double* __restrict__ src,
                                                         const long long* __restrict__ idx, long long n,
                                                         double* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = src[idx[i]];
}

unsigned grid_for(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 1 << 20); }

}  // namespace

hipError_t qgemm(const QGemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.nseg < 1 || g.nseg > QG_MAXSEG || g.nd < 0 || g.nd > QG_MAXD) return hipErrorInvalidValue;
  long long batch = 1;
  for (int d = 0; d < g.nd; ++d) {
    if (g.rad[d] < 1) return hipErrorInvalidValue;
    batch *= g.rad[d];
  }
  if (batch > INT_MAX / 2) return hipErrorInvalidValue;
  // host bounds check: the largest offset each operand and C reach
  bool vec = true;
  for (int sg = 0; sg < g.nseg; ++sg) {
    if (g.K[sg] < 0) return hipErrorInvalidValue;
    const QgOperand* ops[2] = {&g.a[sg], &g.b[sg]};
    const int rows[2] = {g.M, g.N};
    const bool kmaj[2] = {g.akm, g.bkn};
    for (int w = 0; w < 2; ++w) {
      const QgOperand& op = *ops[w];
      long long hi = 0;
      for (int d = 0; d < g.nd; ++d) {
        if (op.sd[d] < 0) return hipErrorInvalidValue;
        hi += (long long)(g.rad[d] - 1) * op.sd[d];
      }
      if (g.K[sg] > 0) {
        hi += kmaj[w] ? (long long)(g.K[sg] - 1) * op.ld + (rows[w] - 1) : (long long)(rows[w] - 1) * op.ld + g.K[sg] - 1;
        if (op.len > 0 && hi >= op.len) return hipErrorInvalidValue;
      }
      vec = vec && (op.ld % 2 == 0) && ((uintptr_t)op.p % 16 == 0) && (g.K[sg] % 2 == 0) && (rows[w] % 2 == 0);
      for (int d = 0; d < g.nd; ++d) vec = vec && (op.sd[d] % 2 == 0);
    }
  }
  {
    // largest offset of a four-level map over [0, n): the digits of n - 1,
    // or a smaller leading part with every later digit at its maximum
    auto mx = [](const Idx4& d, long long n) {
      const long long r[4] = {0, d.n1, d.n2, d.n3}, st[4] = {d.s0, d.s1, d.s2, d.s3};
      long long dg[4], x = n - 1;
      for (int k = 3; k >= 1; --k) {
        dg[k] = x % r[k];
        x /= r[k];
      }
      dg[0] = x;
      long long best = 0;
      for (int k = 0; k < 4; ++k) best += dg[k] * st[k];
      for (int k = 0; k < 4; ++k) {
        if (dg[k] == 0) continue;
        long long alt = 0;
        for (int j = 0; j < k; ++j) alt += dg[j] * st[j];
        alt += (dg[k] - 1) * st[k];
        for (int j = k + 1; j < 4; ++j) alt += (r[j] - 1) * st[j];
        best = std::max(best, alt);
      }
      return best;
    };
    for (const Idx4* d : {&g.cm, &g.cn})
      if (d->n1 < 1 || d->n2 < 1 || d->n3 < 1 || d->s0 < 0 || d->s1 < 0 || d->s2 < 0 || d->s3 < 0)
        return hipErrorInvalidValue;
    long long hi = mx(g.cm, g.M) + mx(g.cn, g.N);
    for (int d = 0; d < g.nd; ++d) hi += (long long)(g.rad[d] - 1) * g.sc[d];
    if (g.c_len > 0 && hi >= g.c_len) return hipErrorInvalidValue;
  }
  // short contractions are bound by the update of C: small tiles, several
  // workgroups per compute unit
  long long ktot = 0;
  for (int sg = 0; sg < g.nseg; ++sg) ktot += g.K[sg];
  const int cfg = ktot <= 64 ? QCFG_N - 1 : qpick(g.M, g.N);
  if (g.akm && !g.bkn) return vec ? qdispatch<true, false, true>(cfg, g, batch, s) : qdispatch<true, false, false>(cfg, g, batch, s);
  if (!g.akm && g.bkn) return vec ? qdispatch<false, true, true>(cfg, g, batch, s) : qdispatch<false, true, false>(cfg, g, batch, s);
  return hipErrorInvalidValue;  // the two mirrored layouts are the ones used
}

hipError_t t3v_transpose(const double* T, const BlockRef* tbl, double* T3v, const int4* cubes, long long ncubes,
                         int o, int v, hipStream_t s) {
  if (ncubes <= 0) return hipSuccess;
  const long long o3 = (long long)o * o * o;
  const int nqc = (int)((o3 + TQ_QC - 1) / TQ_QC);
  const long long nwork = ncubes * nqc;
  const long long grid = ((nwork + 7) / 8) * 8;
  if (grid > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(t3v_transpose_kernel, dim3((unsigned)grid), dim3(256), 0, s, T, tbl, T3v, cubes, nwork, nqc, o,
                     v);
  return hipGetLastError();
}

hipError_t t3v_gather(const double* T3v, double* out, const T3Gather& g, hipStream_t s) {
  long long nblk = g.ne;
  for (int d = 0; d < g.nd; ++d) nblk *= g.rad[d];
  if (nblk <= 0 || g.o <= 0) return hipSuccess;
  if (nblk > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(t3v_gather_kernel, dim3((unsigned)nblk), dim3(256), 0, s, T3v, out, g);
  return hipGetLastError();
}

hipError_t q_wo_build(double* out, const double* Voooo, const double* t2, int o, int v, int x0, int nx, int y0, int ny,
                      const int rowpos[3], hipStream_t s) {
  const long long total = (long long)nx * ny * o * o * o * o;
  if (total <= 0) return hipSuccess;
  // rowpos[c]: position in the row index of i (c = 0), j (1), k (2); the
  // kernel reads i = w[p0] etc. with w the row digits
  hipLaunchKernelGGL(q_wo_kernel, dim3(grid_for(total)), dim3(256), 0, s, out, Voooo, t2, o, v, x0, nx, y0, ny,
                     rowpos[0], rowpos[1], rowpos[2], total);
  return hipGetLastError();
}

hipError_t q_wv_build(double* out, const double* Zxy, const double* Zxz, const double* Vmyje, const double* Vmxje,
                      const double* t2, int o, int v, int x0, int nx, int y0, int ny, int z0, int nz, hipStream_t s) {
  const long long total = (long long)nx * ny * nz * o * o * v;
  if (total <= 0) return hipSuccess;
  if (o <= QW_OMAX) {
    const unsigned nblk = (unsigned)((long long)nx * ny * nz * o);  // (lx, ly, lz, j) and (lx, ly, lz, k)
    const unsigned nth = (unsigned)std::min(256, ((v + 63) / 64) * 64);
    hipLaunchKernelGGL(q_wv_a_kernel, dim3(nblk), dim3(nth), 0, s, out, Zxy, Zxz, Vmyje, Vmxje, t2, o, v, x0, ny, y0,
                       nz, z0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(q_wv_b_kernel, dim3(nblk), dim3(nth), 0, s, out, Vmyje, Vmxje, t2, o, v, x0, ny, y0, nz, z0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(q_wv_kernel, dim3(grid_for(total)), dim3(256), 0, s, out, Zxy, Zxz, Vmyje, Vmxje, t2, o, v, x0,
                     nx, y0, ny, z0, nz, total);
  return hipGetLastError();
}

hipError_t gather_idx(const double* src, const long long* idx, long long n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_idx_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, idx, n, out);
  return hipGetLastError();
}

hipError_t q_abc_energy(const double* X, const double* Y, const double* Vvvoo, const double* t2R, const double* eps,
                        const QSlots& sl, int o, int v, const int* orbits, int norb, double* part, double* etup,
                        double* etask, hipStream_t s) {
  const long long ntau = (long long)sl.n[0] * sl.n[1] * sl.n[2] * sl.n[3];
  if (ntau <= 0) return hipSuccess;
  if (ntau * norb > INT_MAX) return hipErrorInvalidValue;
  const int nbk = (o + QE_BS - 1) / QE_BS, bs = (o + nbk - 1) / nbk;
  QPerms P{};
  int np = 0;
  int p[4] = {0, 1, 2, 3};
  do {
    // cycle type from the longest cycle and the number of cycles
    int seen[4] = {0, 0, 0, 0}, longest = 0, cycles = 0;
    for (int k = 0; k < 4; ++k) {
      if (seen[k]) continue;
      int len = 0;
      for (int x = k; !seen[x]; x = p[x]) {
        seen[x] = 1;
        ++len;
      }
      longest = std::max(longest, len);
      ++cycles;
    }
    double c = 0.0;
    if (longest == 1) c = 16.0;                       // identity
    else if (longest == 2 && cycles == 3) c = -8.0;   // transposition
    else if (longest == 2 && cycles == 2) c = 4.0;    // double transposition
    else if (longest == 3) c = 4.0;                   // three-cycle
    else c = -2.0;                                    // four-cycle
    for (int k = 0; k < 4; ++k) P.p[np][k] = p[k];
    // (j o pi)_k = j_{p[k]} sits at sum_k j_{p[k]} bs^(3-k): digit m = p[k] weighs bs^(3-k)
    for (int k = 0; k < 4; ++k) {
      int w = 1;
      for (int t = k + 1; t < 4; ++t) w *= bs;
      P.w[np][p[k]] = w;
    }
    P.c[np] = c;
    ++np;
  } while (std::next_permutation(p, p + 4));
  hipLaunchKernelGGL(q_abc_energy_kernel, dim3((unsigned)(ntau * norb)), dim3(256), 0, s, X, Y, Vvvoo, t2R, eps, sl, P,
                     orbits, norb, bs, o, v, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(q_abc_reduce_kernel, dim3(1), dim3(256), 0, s, part, sl, (int)ntau, norb, etup, etask);
  return hipGetLastError();
}

// Orbits of the occupied blocks under the axis permutations (see
// q_abc_energy_kernel): per orbit 1 + 24 ints, the block count and the
// blocks packed as b0 | b1 << 8 | b2 << 16 | b3 << 24.
std::vector<int> q_abc_orbits(int o) {
  const int nbk = (o + QE_BS - 1) / QE_BS;
  std::vector<int> out;
  for (int a = 0; a < nbk; ++a)
    for (int b = a; b < nbk; ++b)
      for (int c = b; c < nbk; ++c)
        for (int d = c; d < nbk; ++d) {
          int q[4] = {a, b, c, d};
          std::vector<int> blocks;
          do blocks.push_back(q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24));
          while (std::next_permutation(q, q + 4));
          out.push_back((int)blocks.size());
          for (int k = 0; k < QE_MAXB; ++k) out.push_back(k < (int)blocks.size() ? blocks[k] : -1);
        }
  return out;
}

}  // namespace cct
