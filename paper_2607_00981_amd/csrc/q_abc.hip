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

#include "internal.h"

namespace cct {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));
constexpr int QBK = 16;

__device__ __forceinline__ long long map4(const Idx4& d, long long i) {
  const long long d3 = i % d.n3;
  i /= d.n3;
  const long long d2 = i % d.n2;
  i /= d.n2;
  const long long d1 = i % d.n1;
  return (i / d.n1) * d.s0 + d1 * d.s1 + d2 * d.s2 + d3 * d.s3;
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
  long long aoff[QG_MAXSEG], boff[QG_MAXSEG];
  int ktl[QG_MAXSEG];
  int ntile = 0;
#pragma unroll
  for (int s = 0; s < QG_MAXSEG; ++s) {
    aoff[s] = 0;
    boff[s] = 0;
    ktl[s] = 0;
    if (s < g.nseg) {
      for (int d = 0; d < g.nd; ++d) {
        aoff[s] += dig[d] * g.a[s].sd[d];
        boff[s] += dig[d] * g.b[s].sd[d];
      }
      ktl[s] = (g.K[s] + QBK - 1) / QBK;
      ntile += ktl[s];
    }
  }
  long long coff = 0;
  for (int d = 0; d < g.nd; ++d) coff += dig[d] * g.sc[d];
  const int m0 = tm * BM, n0 = tn * BN;

  dbl2 ra[NA], rb[NB];
  bool oa[NA], ob[NB];
  auto load = [&](int t) {
    int s = 0;
    while (s + 1 < g.nseg && t >= ktl[s]) t -= ktl[s++];
    const int k0 = t * QBK, Ks = g.K[s];
    const double* A = g.a[s].p + aoff[s];
    const double* B = g.b[s].p + boff[s];
    const long long lda = g.a[s].ld, ldb = g.b[s].ld;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int u = tid + i * NTH;
      int row, kk;
      if constexpr (AKM) {
        kk = u / (BM / W);
        row = (u % (BM / W)) * W;
      } else {
        row = u / (QBK / W);
        kk = (u % (QBK / W)) * W;
      }
      const int m = m0 + row, k = k0 + kk;
      oa[i] = u < UA && m < g.M && k < Ks;
      const long long off = oa[i] ? (AKM ? (long long)k * lda + m : (long long)m * lda + k) : 0;
      if constexpr (VEC) ra[i] = *(const dbl2*)(A + off);
      else ra[i].x = A[off];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int u = tid + i * NTH;
      int col, kk;
      if constexpr (BKN) {
        kk = u / (BN / W);
        col = (u % (BN / W)) * W;
      } else {
        col = u / (QBK / W);
        kk = (u % (QBK / W)) * W;
      }
      const int n = n0 + col, k = k0 + kk;
      ob[i] = u < UB && n < g.N && k < Ks;
      const long long off = ob[i] ? (BKN ? (long long)k * ldb + n : (long long)n * ldb + k) : 0;
      if constexpr (VEC) rb[i] = *(const dbl2*)(B + off);
      else rb[i].x = B[off];
    }
  };
  auto store = [&](double* as, double* bs) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int u = tid + i * NTH;
      if (u >= UA) continue;
      if constexpr (AKM) {
        const int kk = u / (BM / W), row = (u % (BM / W)) * W;
        as[kk * LA + row] = oa[i] ? ra[i].x : 0.0;
        if constexpr (VEC) as[kk * LA + row + 1] = oa[i] ? ra[i].y : 0.0;
      } else {
        const int row = u / (QBK / W), kk = (u % (QBK / W)) * W;
        as[kk * LA + row] = oa[i] ? ra[i].x : 0.0;
        if constexpr (VEC) as[(kk + 1) * LA + row] = oa[i] ? ra[i].y : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int u = tid + i * NTH;
      if (u >= UB) continue;
      if constexpr (BKN) {
        const int kk = u / (BN / W), col = (u % (BN / W)) * W;
        bs[kk * LB + col] = ob[i] ? rb[i].x : 0.0;
        if constexpr (VEC) bs[kk * LB + col + 1] = ob[i] ? rb[i].y : 0.0;
      } else {
        const int col = u / (QBK / W), kk = (u % (QBK / W)) * W;
        bs[kk * LB + col] = ob[i] ? rb[i].x : 0.0;
        if constexpr (VEC) bs[(kk + 1) * LB + col] = ob[i] ? rb[i].y : 0.0;
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
  if (ntile > 0) {
    load(0);
    store(As[0], Bs[0]);
  }
  __syncthreads();
  for (int t = 0; t < ntile; ++t) {
    const int cur = t & 1;
    if (t + 1 < ntile) load(t + 1);
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
    if (t + 1 < ntile) store(As[cur ^ 1], Bs[cur ^ 1]);
    __syncthreads();
  }
  // accumulator register r of lane l: row 4r + l/16, column l%16
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm0 + i * 16 + 4 * r + lane / 16;
      if (m >= g.M) continue;
      const long long mo = coff + map4(g.cm, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = n0 + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        double* p = g.C + mo + map4(g.cn, n);
        const double x = g.alpha * acc[i][j][r];
        *p = g.accumulate ? *p + x : x;
      }
    }
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
    case 0: return qlaunch<4, 4, 2, 2, AKM, BKN, VEC>(g, batch, s);   // 128 x 128
    case 1: return qlaunch<5, 4, 1, 4, AKM, BKN, VEC>(g, batch, s);   // 80 x 256
    case 2: return qlaunch<4, 5, 4, 1, AKM, BKN, VEC>(g, batch, s);   // 256 x 80
    case 3: return qlaunch<2, 5, 4, 1, AKM, BKN, VEC>(g, batch, s);   // 128 x 80
    case 4: return qlaunch<5, 2, 1, 4, AKM, BKN, VEC>(g, batch, s);   // 80 x 128
    case 5: return qlaunch<5, 5, 1, 2, AKM, BKN, VEC>(g, batch, s);   // 80 x 160
    case 6: return qlaunch<5, 5, 2, 1, AKM, BKN, VEC>(g, batch, s);   // 160 x 80
    default: return qlaunch<2, 2, 2, 2, AKM, BKN, VEC>(g, batch, s);  // 64 x 64
  }
}

constexpr int QCFG_BM[8] = {128, 80, 256, 128, 80, 80, 160, 64};
constexpr int QCFG_BN[8] = {128, 256, 80, 80, 128, 160, 80, 64};

// Tile choice: the largest operand reuse (BM BN / (BM + BN)) among the
// shapes that waste at most 15 % of the padded output, else the best
// product of reuse and useful fraction.
int qpick(int M, int N) {
  int best = 7;
  double best_score = -1.0;
  for (int c = 0; c < 8; ++c) {
    const double bm = QCFG_BM[c], bn = QCFG_BN[c];
    const double padded = std::ceil(M / bm) * bm * std::ceil(N / bn) * bn;
    const double useful = (double)M * N / padded;
    const double reuse = bm * bn / (bm + bn);
    const double score = (useful >= 0.85 ? 1.0 : useful) * reuse;
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

__global__ __launch_bounds__(256) void t3v_gather_kernel(const double* __restrict__ T3v, double* __restrict__ out,
                                                         T3Gather g, long long total) {
  const long long o3 = (long long)g.o * g.o * g.o;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long q = idx % o3;
    long long r = idx / o3;
    const int e = (int)(r % g.ne);
    r /= g.ne;
    int dig[3] = {0, 0, 0};
    for (int d = g.nd - 1; d >= 0; --d) {
      dig[d] = (int)(r % g.rad[d]);
      r /= g.rad[d];
    }
    const int y[3] = {(int)(q / (g.o * g.o)), (int)((q / g.o) % g.o), (int)(q % g.o)};
    int lab[3], occ[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lab[c] = g.lab[c] == 3 ? e : g.st[g.lab[c]] + dig[g.lab[c]];
      occ[c] = y[g.ax[c]];
    }
    // order the column pairs by virtual label (ties: equal values by column symmetry)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2 - i; ++j)
        if (lab[j] > lab[j + 1]) {
          const int tl = lab[j], to = occ[j];
          lab[j] = lab[j + 1];
          occ[j] = occ[j + 1];
          lab[j + 1] = tl;
          occ[j + 1] = to;
        }
    out[idx] = T3v[vtri(lab[0], lab[1], lab[2], g.v) * o3 + ((long long)occ[0] * g.o + occ[1]) * g.o + occ[2]];
  }
}

// Wbar_{ijk}^{xym} (alternative form) = -1/2 sum_n (v^{mn}_{ki} t_{nj}^{xy} + v^{mn}_{kj} t_{ni}^{yx})
// for x = x0 + lx, y = y0 + ly; element [lx][ly][rows][m] with the row index
// holding i, j, k at the positions rowpos[0..2].
__global__ __launch_bounds__(256) void q_wo_kernel(double* __restrict__ out, const double* __restrict__ Voooo,
                                                   const double* __restrict__ t2, int o, int v, int x0, int nx,
                                                   int y0, int ny, int p0, int p1, int p2, long long total) {
  const long long o2 = (long long)o * o, vv = (long long)v * v;
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
      const double* vr = Voooo + ((long long)m * o + n) * o2 + (long long)k * o;
      s += vr[i] * t2[((long long)n * o + j) * vv + (long long)x * v + y] +
           vr[j] * t2[((long long)n * o + i) * vv + (long long)y * v + x];
    }
    out[idx] = -0.5 * s;
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

__global__ __launch_bounds__(256) void q_add_kernel(double* __restrict__ Y, const double* __restrict__ X,
                                                    long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    Y[i] += X[i];
}

// The spin summation 2 (2 - P_cd)(2 - P_bc - P_bd)(2 - P_ab - P_ac - P_ad),
// multiplied out, is a class function of the permutation group: 16 on the
// identity, -8 on transpositions, 4 on three-cycles and on double
// transpositions, -2 on four-cycles.
struct QPerms {
  int p[24][4];
  double c[24];
};

constexpr int QE_CHUNK = 2048;  // occupied quadruples per workgroup

__global__ __launch_bounds__(256) void q_abc_energy_kernel(const double* __restrict__ X, const double* __restrict__ R,
                                                           const double* __restrict__ Vvvoo,
                                                           const double* __restrict__ t2,
                                                           const double* __restrict__ eps, QSlots sl, QPerms P, int o,
                                                           int v, int nchunk, double* __restrict__ part) {
  __shared__ double red[256];
  const int chunk = blockIdx.x % nchunk;
  const int tau = blockIdx.x / nchunk;
  int l[4], lab[4];
  {
    int r = tau;
    for (int s = 3; s >= 0; --s) {
      l[s] = r % sl.n[s];
      r /= sl.n[s];
    }
    for (int s = 0; s < 4; ++s) lab[s] = sl.st[s] + l[s];
  }
  const bool canon = lab[0] <= lab[1] && lab[1] <= lab[2] && lab[2] <= lab[3] &&
                     !(lab[0] == lab[1] && lab[1] == lab[2]) && !(lab[1] == lab[2] && lab[2] == lab[3]);
  double acc = 0.0;
  if (canon) {
    const long long o2 = (long long)o * o, o4 = o2 * o2, vv = (long long)v * v;
    const double* x = X + (long long)tau * o4;
    const double* rr = R + (long long)tau * o4;
    const double ev = eps[o + lab[0]] + eps[o + lab[1]] + eps[o + lab[2]] + eps[o + lab[3]];
    const long long st[4] = {o2 * o, o2, (long long)o, 1};
    const long long q0 = (long long)chunk * QE_CHUNK;
    const long long q1 = min(q0 + (long long)QE_CHUNK, o4);
    for (long long q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
      const int i[4] = {(int)(q / (o2 * o)), (int)((q / o2) % o), (int)((q / o) % o), (int)(q % o)};
      double u = 0.0;
#pragma unroll 4
      for (int p = 0; p < 24; ++p)
        u += P.c[p] * rr[i[P.p[p][0]] * st[0] + i[P.p[p][1]] * st[1] + i[P.p[p][2]] * st[2] + i[P.p[p][3]]];
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
                t2[((long long)i[s2] * o + i[s3]) * vv + (long long)lab[s2] * v + lab[s3]];
        }
      acc += (x[q] + vs) * (u / den);
    }
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
  const int cfg = qpick(g.M, g.N);
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
  long long total = (long long)g.o * g.o * g.o * g.ne;
  for (int d = 0; d < g.nd; ++d) total *= g.rad[d];
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(t3v_gather_kernel, dim3(grid_for(total)), dim3(256), 0, s, T3v, out, g, total);
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
  hipLaunchKernelGGL(q_wv_kernel, dim3(grid_for(total)), dim3(256), 0, s, out, Zxy, Zxz, Vmyje, Vmxje, t2, o, v, x0,
                     nx, y0, ny, z0, nz, total);
  return hipGetLastError();
}

hipError_t q_add(double* Y, const double* X, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(q_add_kernel, dim3(grid_for(n)), dim3(256), 0, s, Y, X, n);
  return hipGetLastError();
}

hipError_t gather_idx(const double* src, const long long* idx, long long n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_idx_kernel, dim3(grid_for(n)), dim3(256), 0, s, src, idx, n, out);
  return hipGetLastError();
}

hipError_t q_abc_energy(const double* X, const double* R, const double* Vvvoo, const double* t2, const double* eps,
                        const QSlots& sl, int o, int v, double* part, double* etup, double* etask, hipStream_t s) {
  const long long o4 = (long long)o * o * o * o;
  const int nchunk = (int)((o4 + QE_CHUNK - 1) / QE_CHUNK);
  const long long ntau = (long long)sl.n[0] * sl.n[1] * sl.n[2] * sl.n[3];
  if (ntau <= 0) return hipSuccess;
  if (ntau * nchunk > INT_MAX) return hipErrorInvalidValue;
  QPerms P{};
  int np = 0;
  int p[4] = {0, 1, 2, 3};
  do {
    // cycle type from the number of fixed points and the cycle structure
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
    P.c[np] = c;
    ++np;
  } while (std::next_permutation(p, p + 4));
  hipLaunchKernelGGL(q_abc_energy_kernel, dim3((unsigned)(ntau * nchunk)), dim3(256), 0, s, X, R, Vvvoo, t2, eps, sl, P,
                     o, v, nchunk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(q_abc_reduce_kernel, dim3(1), dim3(256), 0, s, part, sl, (int)ntau, nchunk, etup, etask);
  return hipGetLastError();
}

}  // namespace cct
