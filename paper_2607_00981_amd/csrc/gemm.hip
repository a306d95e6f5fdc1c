// Strided, batched GEMM on CDNA4 matrix cores with two-level index maps.
//
// C[b](m,n) = alpha * sum_k A[b](m,k) B[b](k,n) + beta * C[b](m,n), where every
// index of every operand goes through an Idx2 map, so permuted views of packed
// T3 blocks (the three relabelled operands of the particle-particle ladder)
// and of the dressed integrals are read in place without transposed copies.
//
// Tiling: 256 threads = 4 waves of 64 lanes, BM x BN output tile, BK = 16.
// Operand tiles are staged through LDS (double buffered); each wave owns a
// (BM/2) x (BN/2) sub-tile of 16x16 MFMA blocks.  Global loads of the next K
// tile are issued before the MFMAs of the current one, so their latency hides
// behind the matrix-core work.  Loads follow the operand's unit-stride axis
// (k-fast or m/n-fast mapping) so that a wave reads contiguous 128-byte runs.
//
// FP64:   v_mfma_f64_16x16x4_f64.  A lane l holds A(row l%16, k l/16) and
//         B(k l/16, col l%16); the accumulator register r of lane l holds
//         D(row 4r + l/16, col l%16).
// FP32:   operands rounded to FP32 in LDS, v_mfma_f32_16x16x4_f32; the FP32
//         accumulators are flushed into FP64 registers every K tile.
// BF16X3: each operand x is split into hi = bf16(x), lo = bf16(x - hi); the
//         product uses hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x32_bf16
//         (A(row l%16, k 8*(l/16)+e), D(row 4*(l/16)+r, col l%16)); FP32
//         accumulators are flushed into FP64 every K tile.
#include "internal.h"

#include <climits>
#include <numeric>

namespace cct {
namespace {

constexpr int NT = 256;
constexpr int BK = 16;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ long long map2(const Idx2& d, int i) {
  if (d.inner == 0) return (long long)i * d.s_lo;
  int hi = (int)((unsigned)i / (unsigned)d.inner);
  int lo = i - hi * d.inner;
  return (long long)hi * d.s_hi + (long long)lo * d.s_lo;
}

// One 16-byte-per-lane copy from global memory into LDS (the 64 lanes fill
// 1 KB from LDS byte address lds, lane i at lds + 16 i).  Written out rather
// than through the compiler builtin: the builtin makes the compiler wait for
// every such copy in flight before any later LDS read, including the reads of
// the other buffer that the copies are meant to overlap.  The instruction has
// no register results; its completion is counted by vmcnt, and the kernels
// that use it wait for it (s_waitcnt vmcnt(0)) before the barrier that ends
// each K step, i.e. before anything reads the copied tile.
__device__ __forceinline__ void lds_copy16(const void* src, unsigned lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" : : "v"(src), "s"(lds) : "memory", "m0");
}
__device__ __forceinline__ unsigned lds_addr(const __bf16* p) {
  return (unsigned)(size_t)(__attribute__((address_space(3))) const void*)p;
}

// Position of the tile handled by this workgroup.  Consecutive workgroup ids
// land on different XCDs (round robin over 8); remap so that each XCD gets a
// contiguous range of the tile order, and order tiles in groups of GM tile
// rows so that concurrently running workgroups on one XCD share A and B
// panels in that XCD's L2.
__device__ __forceinline__ bool tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
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

template <int BM, int BN>
struct Tiles {
  static constexpr int TM = BM / 32;  // 16x16 blocks per wave along M
  static constexpr int TN = BN / 32;
  static constexpr int PADA = 2, PADB = 2;
  static constexpr int LA = BM + PADA, LB = BN + PADB;
  static constexpr int EA = BM * BK / NT;  // A elements loaded per thread per K tile
  static constexpr int EB = BN * BK / NT;
};

// ---------------------------------------------------------------------------
// operand staging: global (any Idx2 layout) -> registers -> LDS
// ---------------------------------------------------------------------------
template <int BM, int BN>
struct Loader {
  // Row (A) and column (B) parts of the operand addresses, one per tile row /
  // column, kept in LDS (-1 marks rows/columns outside the matrix).
  const long long* a_row;
  const long long* b_col;
  int a_k0, a_m0;
  bool a_kfast;
  int b_k0, b_n0;
  bool b_nfast;
};

template <int BM, int BN>
__device__ __forceinline__ void load_tile(const GemmArgs& g, const double* __restrict__ A, const double* __restrict__ B,
                                          const Loader<BM, BN>& L, int k0, double (&ra)[Tiles<BM, BN>::EA],
                                          double (&rb)[Tiles<BM, BN>::EB]) {
  using T = Tiles<BM, BN>;
  if (L.a_kfast) {
    const int k = k0 + L.a_k0;
    const bool kok = k < g.K;
    const long long ko = kok ? map2(g.ak, k) : 0;
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      const long long r = L.a_row[L.a_m0 + e * (NT / BK)];
      ra[e] = (kok && r >= 0) ? A[r + ko] : 0.0;
    }
  } else {
    constexpr int step = NT / BM;
    const long long r = L.a_row[L.a_m0];
#pragma unroll
    for (int e = 0; e < T::EA; ++e) {
      const int k = k0 + L.a_k0 + e * step;
      ra[e] = (k < g.K && r >= 0) ? A[r + map2(g.ak, k)] : 0.0;
    }
  }
  if (L.b_nfast) {
    constexpr int step = NT / BN;
    const long long c = L.b_col[L.b_n0];
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const int k = k0 + L.b_k0 + e * step;
      rb[e] = (k < g.K && c >= 0) ? B[c + map2(g.bk, k)] : 0.0;
    }
  } else {
    const int k = k0 + L.b_k0;
    const bool kok = k < g.K;
    const long long ko = kok ? map2(g.bk, k) : 0;
#pragma unroll
    for (int e = 0; e < T::EB; ++e) {
      const long long c = L.b_col[L.b_n0 + e * (NT / BK)];
      rb[e] = (kok && c >= 0) ? B[c + ko] : 0.0;
    }
  }
}

template <int BM, int BN, typename S>
__device__ __forceinline__ void store_tile(const Loader<BM, BN>& L, const double (&ra)[Tiles<BM, BN>::EA],
                                           const double (&rb)[Tiles<BM, BN>::EB], S* As, S* Bs) {
  using T = Tiles<BM, BN>;
  if (L.a_kfast) {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) As[L.a_k0 * T::LA + L.a_m0 + e * (NT / BK)] = (S)ra[e];
  } else {
#pragma unroll
    for (int e = 0; e < T::EA; ++e) As[(L.a_k0 + e * (NT / BM)) * T::LA + L.a_m0] = (S)ra[e];
  }
  if (L.b_nfast) {
#pragma unroll
    for (int e = 0; e < T::EB; ++e) Bs[(L.b_k0 + e * (NT / BN)) * T::LB + L.b_n0] = (S)rb[e];
  } else {
#pragma unroll
    for (int e = 0; e < T::EB; ++e) Bs[L.b_k0 * T::LB + L.b_n0 + e * (NT / BK)] = (S)rb[e];
  }
}

// Fill the LDS offset tables (rows of A, columns of B) and choose the load
// mappings.  Ends with a barrier.
template <int BM, int BN>
__device__ __forceinline__ void init_loader(const GemmArgs& g, int tm, int tn, long long a_off, long long b_off,
                                            long long* rowA, long long* colB, Loader<BM, BN>& L) {
  const int tid = threadIdx.x;
  const int m_base = tm * BM, n_base = tn * BN;
  for (int i = tid; i < BM; i += NT) {
    const int m = m_base + i;
    rowA[i] = (m < g.M) ? a_off + map2(g.am, m) : -1;
  }
  for (int i = tid; i < BN; i += NT) {
    const int n = n_base + i;
    colB[i] = (n < g.N) ? b_off + map2(g.bn, n) : -1;
  }
  L.a_row = rowA;
  L.b_col = colB;
  L.a_kfast = (g.ak.s_lo == 1);
  if (L.a_kfast) { L.a_k0 = tid % BK; L.a_m0 = tid / BK; }
  else { L.a_m0 = tid % BM; L.a_k0 = tid / BM; }
  L.b_nfast = (g.bn.s_lo == 1);
  if (L.b_nfast) { L.b_n0 = tid % BN; L.b_k0 = tid / BN; }
  else { L.b_k0 = tid % BK; L.b_n0 = tid / BK; }
  __syncthreads();
}

template <int BM, int BN>
__device__ __forceinline__ void store_c(const GemmArgs& g, int tm, int tn, long long c_off,
                                        const double (&acc)[Tiles<BM, BN>::TM][Tiles<BM, BN>::TN][4],
                                        int wm0, int wn0, bool f64_layout) {
  using T = Tiles<BM, BN>;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < T::TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = f64_layout ? (4 * r + lane / 16) : (4 * (lane / 16) + r);
      const int m = tm * BM + wm0 + i * 16 + row;
      if (m >= g.M) continue;
      const long long mo = c_off + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < T::TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        double* p = g.C + mo + map2(g.cn, n);
        const double x = g.alpha * acc[i][j][r];
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 kernel
// ---------------------------------------------------------------------------
// kchunk > 0: this workgroup covers K range [blockIdx.y * kchunk, + kchunk)
// (absolute K indices through the operands' index maps, so a range may start
// anywhere) and writes its raw partial sums to part[((b * splits + y) * M + m) * N + n].
template <int BM, int BN>
__global__ __launch_bounds__(NT, 2) void gemm_f64_kernel(GemmArgs g, int tiles_m, int tiles_n, int kchunk,
                                                         double* __restrict__ part) {
  using T = Tiles<BM, BN>;
  __shared__ double As[2][BK * T::LA];
  __shared__ double Bs[2][BK * T::LB];
  __shared__ long long rowA[BM], colB[BN];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int b = blockIdx.z;
  constexpr bool can_split = (BM == 64);  // the split path exists for the small-tile kernel only
  int kb = 0;  // first K index of this workgroup; g.K becomes the end of its range
  if (can_split && kchunk > 0) {
    kb = blockIdx.y * kchunk;
    g.K = min(g.K, kb + kchunk);
  }
  const double* A = (const double*)g.A;
  const double* B = (const double*)g.B;
  Loader<BM, BN> L;
  init_loader<BM, BN>(g, tm, tn, (long long)b * g.a_batch, (long long)b * g.b_batch, rowA, colB, L);

  const int wave = threadIdx.x / 64, lane = threadIdx.x & 63;
  const int wm0 = (wave >> 1) * (BM / 2), wn0 = (wave & 1) * (BN / 2);
  d4 acc[T::TM][T::TN];
#pragma unroll
  for (int i = 0; i < T::TM; ++i)
#pragma unroll
    for (int j = 0; j < T::TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[T::EA], rb[T::EB];
  const int nk = (g.K - kb + BK - 1) / BK;
  load_tile<BM, BN>(g, A, B, L, kb, ra, rb);
  store_tile<BM, BN, double>(L, ra, rb, As[0], Bs[0]);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load_tile<BM, BN>(g, A, B, L, kb + (kt + 1) * BK, ra, rb);
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      double af[T::TM], bf[T::TN];
#pragma unroll
      for (int i = 0; i < T::TM; ++i) af[i] = as[kr * T::LA + wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < T::TN; ++j) bf[j] = bs[kr * T::LB + wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < T::TM; ++i)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile<BM, BN, double>(L, ra, rb, As[cur ^ 1], Bs[cur ^ 1]);
    __syncthreads();
  }
  double out[T::TM][T::TN][4];
#pragma unroll
  for (int i = 0; i < T::TM; ++i)
#pragma unroll
    for (int j = 0; j < T::TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[i][j][r] = acc[i][j][r];
  if (can_split && kchunk > 0) {
    const int lane_ = threadIdx.x & 63;
    double* P = part + ((long long)b * gridDim.y + blockIdx.y) * (long long)g.M * g.N;
#pragma unroll
    for (int i = 0; i < T::TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = tm * BM + wm0 + i * 16 + 4 * r + lane_ / 16;
        if (m >= g.M) continue;
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
          const int n = tn * BN + wn0 + j * 16 + (lane_ & 15);
          if (n < g.N) P[(long long)m * g.N + n] = out[i][j][r];
        }
      }
    return;
  }
  store_c<BM, BN>(g, tm, tn, (long long)b * g.c_batch, out, wm0, wn0, true);
}

// C(m,n) = alpha * sum_y part[b][y][m][n] + beta * C(m,n), splits added in order.
__global__ void splitk_reduce_kernel(const double* __restrict__ part, int splits, GemmArgs g) {
  const long long mn = (long long)g.M * g.N;
  const long long total = mn * g.batch;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long b = e / mn, r = e - b * mn;
    const int m = (int)(r / g.N), n = (int)(r - (long long)m * g.N);
    const double* p = part + b * splits * mn + r;
    double acc = 0.0;
    for (int y = 0; y < splits; ++y) acc += p[y * mn];
    double* c = g.C + b * g.c_batch + map2(g.cm, m) + map2(g.cn, n);
    const double x = g.alpha * acc;
    *c = (g.beta == 0.0) ? x : x + g.beta * *c;
  }
}

template <int BM, int BN>
hipError_t launch(const GemmArgs& g, Prec prec, hipStream_t s) {
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long grid_x = ((nb + 7) / 8) * 8;
  if (grid_x > INT_MAX || g.batch > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid_x, 1, (unsigned)g.batch);
  if (prec == Prec::F64) {
    // few output tiles and a long K: split K so that the chip fills
    int splits = 1;
    const long long tiles = nb * g.batch;
    const long long mn = (long long)g.M * g.N * g.batch;
    if (BM == 64 && g.split_ws && tiles < 128 && g.K >= 8 * BK) {
      splits = (int)std::min<long long>((256 + tiles - 1) / tiles, g.K / (4 * BK));
      splits = (int)std::min<long long>(splits, g.split_cap / std::max<long long>(mn, 1));
      splits = std::min(splits, 64);
    }
    // each split covers whole K tiles
    const long long unit = BK;
    if (splits >= 2 && unit < g.K) {
      const long long per = (g.K + splits - 1) / splits;
      const int kchunk = (int)(((per + unit - 1) / unit) * unit);
      splits = (g.K + kchunk - 1) / kchunk;
    } else {
      splits = 1;
    }
    if (splits >= 2) {
      const long long per = (g.K + splits - 1) / splits;
      const int kchunk = (int)(((per + unit - 1) / unit) * unit);
      grid.y = (unsigned)splits;
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN>), grid, dim3(NT), 0, s, g, tiles_m, tiles_n, kchunk, g.split_ws);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      const long long total = mn;
      const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 4096);
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const double*)g.split_ws, splits, g);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN>), grid, dim3(NT), 0, s, g, tiles_m, tiles_n, 0, (double*)nullptr);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t gemm(const GemmArgs& g, Prec prec, hipStream_t s) {
  if (prec != Prec::F64) return hipErrorInvalidValue;  // low precision: gemm_nt_lp on converted operands
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  const long long nb = g.batch - 1;
  if (g.a_len > 0 && nb * g.a_batch + idx_max(g.am, g.M) + idx_max(g.ak, g.K) >= g.a_len) return hipErrorInvalidValue;
  if (g.b_len > 0 && nb * g.b_batch + idx_max(g.bk, g.K) + idx_max(g.bn, g.N) >= g.b_len) return hipErrorInvalidValue;
  if (g.c_len > 0 && nb * g.c_batch + idx_max(g.cm, g.M) + idx_max(g.cn, g.N) >= g.c_len) return hipErrorInvalidValue;
  if (g.K <= 0) return g.beta == 1.0 ? hipSuccess : hipErrorInvalidValue;
  const long long work = (long long)g.M * g.N * g.batch;
  if (work >= (long long)256 * 128 * 128 * 2) return launch<128, 128>(g, prec, s);
  return launch<64, 64>(g, prec, s);
}

}  // namespace cct

// ===========================================================================
// K-contiguous ("NT") GEMM: both operands are row-major with the contracted
// index fastest, so a K tile of 16 doubles is one 128-byte line per row.
// Loads are 16-byte vectors (two doubles), rows outside the matrix are
// clamped to a valid row and zeroed, and the main loop carries no index
// arithmetic beyond pointer increments.  Tile BM x BN with WM x WN waves.
// ===========================================================================
namespace cct {
namespace {

typedef double dbl2 __attribute__((ext_vector_type(2)));

template <int BM, int BN, int WM, int WN>
struct NtCfg {
  static constexpr int NTH = 64 * WM * WN;
  static constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  static constexpr int LA = BM + 2, LB = BN + 2;
  static constexpr int SA = BM * (BK / 2) / NTH;  // 16-byte segments of A per thread per K tile
  static constexpr int SB = BN * (BK / 2) / NTH;
};

template <int BM, int BN, int WM, int WN, int OCC, bool BKN>
__global__ __launch_bounds__(64 * WM * WN, OCC) void gemm_nt_f64_kernel(NtArgs g, int tiles_m, int tiles_n) {
  using C = NtCfg<BM, BN, WM, WN>;
  __shared__ double As[2][BK * C::LA];
  __shared__ double Bs[2][BK * C::LB];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x;
  const int b = blockIdx.z;
  const double* A = g.A + (long long)b * g.a_batch;
  const double* B = g.B + (long long)b * g.b_batch;
  // per-thread source rows (clamped) and validity
  const double* pa[C::SA];
  const double* pb[C::SB];
  int ka[C::SA], kb[C::SB];
  bool va[C::SA], vb[C::SB];
#pragma unroll
  for (int i = 0; i < C::SA; ++i) {
    const int seg = tid + i * C::NTH;
    const int row = seg / (BK / 2);
    ka[i] = 2 * (seg % (BK / 2));
    const int m = tm * BM + row;
    va[i] = m < g.M;
    pa[i] = A + (long long)(va[i] ? m : 0) * g.lda + ka[i];
  }
#pragma unroll
  for (int i = 0; i < C::SB; ++i) {
    const int seg = tid + i * C::NTH;
    if constexpr (BKN) {
      // B[k][n]: segments of two consecutive n in one k row
      kb[i] = seg / (BN / 2);
      const int n = tn * BN + 2 * (seg % (BN / 2));
      vb[i] = n < g.N;
      pb[i] = B + (long long)kb[i] * g.ldb + (vb[i] ? (g.b_map ? map2(g.bnm, n) : (long long)n) : 0);
    } else {
      const int row = seg / (BK / 2);
      kb[i] = 2 * (seg % (BK / 2));
      const int n = tn * BN + row;
      vb[i] = n < g.N;
      pb[i] = B + (long long)(vb[i] ? n : 0) * g.ldb + kb[i];
    }
  }
  const int wave = tid / 64, lane = tid & 63;
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  d4 acc[C::TM][C::TN];
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // Raw loads go to registers; masking is applied when they are written to
  // LDS after the matrix-core work, so the wait for the loads lands there
  // and not right after the loads are issued.
  dbl2 ra[C::SA], rb[C::SB];
  bool oa[C::SA], ob[C::SB];
  const int nk = (g.K + BK - 1) / BK;
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < C::SA; ++i) {
      oa[i] = va[i] && (k0 + ka[i] < g.K);
      ra[i] = *(const dbl2*)(pa[i] + (oa[i] ? k0 : 0));
    }
#pragma unroll
    for (int i = 0; i < C::SB; ++i) {
      ob[i] = vb[i] && (k0 + kb[i] < g.K);
      if constexpr (BKN) rb[i] = *(const dbl2*)(pb[i] + (ob[i] ? (long long)k0 * g.ldb : 0));
      else rb[i] = *(const dbl2*)(pb[i] + (ob[i] ? k0 : 0));
    }
  };
  auto store = [&](double* as, double* bs) {
#pragma unroll
    for (int i = 0; i < C::SA; ++i) {
      const int row = (tid + i * C::NTH) / (BK / 2);
      as[ka[i] * C::LA + row] = oa[i] ? ra[i].x : 0.0;
      as[(ka[i] + 1) * C::LA + row] = oa[i] ? ra[i].y : 0.0;
    }
#pragma unroll
    for (int i = 0; i < C::SB; ++i) {
      if constexpr (BKN) {
        const int col = 2 * ((tid + i * C::NTH) % (BN / 2));
        bs[kb[i] * C::LB + col] = ob[i] ? rb[i].x : 0.0;
        bs[kb[i] * C::LB + col + 1] = ob[i] ? rb[i].y : 0.0;
      } else {
        const int row = (tid + i * C::NTH) / (BK / 2);
        bs[kb[i] * C::LB + row] = ob[i] ? rb[i].x : 0.0;
        bs[(kb[i] + 1) * C::LB + row] = ob[i] ? rb[i].y : 0.0;
      }
    }
  };
  load(0);
  store(As[0], Bs[0]);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      double af[C::TM], bf[C::TN];
#pragma unroll
      for (int i = 0; i < C::TM; ++i) af[i] = as[kr * C::LA + wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < C::TN; ++j) bf[j] = bs[kr * C::LB + wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int j = 0; j < C::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store(As[cur ^ 1], Bs[cur ^ 1]);
    __syncthreads();
  }
  // epilogue: accumulator register r of lane l holds row 4r + l/16, column l%16
  const long long coff = (long long)b * g.c_batch;
#pragma unroll
  for (int i = 0; i < C::TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = tm * BM + wm0 + i * 16 + 4 * r + lane / 16;
      if (m >= g.M) continue;
      const long long mo = coff + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        double* p = g.C + mo + map2(g.cn, n);
        const double x = g.alpha * acc[i][j][r];
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
  }
}

template <int BM, int BN, int WM, int WN, int OCC>
hipError_t launch_nt(const NtArgs& g, hipStream_t s) {
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long grid_x = ((nb + 7) / 8) * 8;
  if (grid_x > INT_MAX || g.batch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)grid_x, 1, (unsigned)g.batch);
  if (g.b_kn)
    hipLaunchKernelGGL((gemm_nt_f64_kernel<BM, BN, WM, WN, OCC, true>), grid, dim3(64 * WM * WN), 0, s, g, tiles_m,
                       tiles_n);
  else
    hipLaunchKernelGGL((gemm_nt_f64_kernel<BM, BN, WM, WN, OCC, false>), grid, dim3(64 * WM * WN), 0, s, g, tiles_m,
                       tiles_n);
  return hipGetLastError();
}

// The NT kernel with the operand tiles copied from global memory straight
// into LDS (no register staging, no LDS stores), for K a multiple of BK = 16
// and both operands K-contiguous.  An LDS row holds one K tile of one matrix
// row: 16 doubles as eight 16-byte pairs, pair p at slot p ^ ((row >> 1) & 7).
// The 16 x 16 x 4 fragment reads (16 consecutive rows at one k per 16 lanes)
// then fall on distinct banks.  Each wave copies whole 1 KB chunks (8 rows);
// lane s of a chunk lands in row s / 8 at slot s % 8 and fetches the pair that
// the swizzle keeps there.  Rows past the matrix are read from row 0 (finite
// values whose products go to outputs that are not stored).  Two buffers; the
// copies of step t + 1 fly while step t is multiplied.
__device__ __forceinline__ int nt_swz(int row, int k) { return row * BK + 2 * ((k >> 1) ^ ((row >> 1) & 7)) + (k & 1); }

template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, 1) void gemm_nt_f64_dl_kernel(NtArgs g, int tiles_m, int tiles_n) {
  constexpr int NW = WM * WN, TM = BM / WM / 16, TN = BN / WN / 16;
  constexpr int CA = BM / 8, CB = BN / 8;  // 1 KB chunks per K tile
  static_assert(CA % NW == 0 && CB % NW == 0, "whole chunks per wave");
  constexpr int PA = CA / NW, PB = CB / NW;
  constexpr int ABUF = BM * BK, BBUF = BN * BK;  // doubles per buffer
  __shared__ __attribute__((aligned(1024))) double As[2 * ABUF];
  __shared__ __attribute__((aligned(1024))) double Bs[2 * BBUF];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x, b = blockIdx.z;
  const int wave = tid / 64, lane = tid & 63;
  const double* A = g.A + (long long)b * g.a_batch;
  const double* B = g.B + (long long)b * g.b_batch;
  const double* sa[PA];
  const double* sb[PB];
  unsigned la[PA], lb[PB];
  const unsigned as0 = (unsigned)(size_t)(__attribute__((address_space(3))) const void*)As;
  const unsigned bs0 = (unsigned)(size_t)(__attribute__((address_space(3))) const void*)Bs;
#pragma unroll
  for (int j = 0; j < PA; ++j) {
    const int c = wave + NW * j, row = c * 8 + lane / 8, kp = (lane % 8) ^ ((row >> 1) & 7);
    const int m = tm * BM + row;
    sa[j] = A + (long long)(m < g.M ? m : 0) * g.lda + 2 * kp;
    la[j] = __builtin_amdgcn_readfirstlane(as0 + 8u * (unsigned)(c * 8 * BK));
  }
#pragma unroll
  for (int j = 0; j < PB; ++j) {
    const int c = wave + NW * j, row = c * 8 + lane / 8, kp = (lane % 8) ^ ((row >> 1) & 7);
    const int n = tn * BN + row;
    sb[j] = B + (long long)(n < g.N ? n : 0) * g.ldb + 2 * kp;
    lb[j] = __builtin_amdgcn_readfirstlane(bs0 + 8u * (unsigned)(c * 8 * BK));
  }
  auto issue = [&](int kt, int buf) {
    const long long k0 = (long long)kt * BK;
    const unsigned da = buf * (8u * ABUF), db = buf * (8u * BBUF);  // bytes
#pragma unroll
    for (int j = 0; j < PA; ++j) lds_copy16(sa[j] + k0, la[j] + da);
#pragma unroll
    for (int j = 0; j < PB; ++j) lds_copy16(sb[j] + k0, lb[j] + db);
  };
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = g.K / BK;
  issue(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) issue(kt + 1, cur ^ 1);
    const double* as = As + cur * ABUF;
    const double* bs = Bs + cur * BBUF;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = as[nt_swz(wm0 + i * 16 + (lane & 15), kr)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = bs[nt_swz(wn0 + j * 16 + (lane & 15), kr)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  // epilogue: accumulator register r of lane l holds row 4r + l/16, column l%16
  const long long coff = (long long)b * g.c_batch;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = tm * BM + wm0 + i * 16 + 4 * r + lane / 16;
      if (m >= g.M) continue;
      const long long mo = coff + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        double* p = g.C + mo + map2(g.cn, n);
        const double x = g.alpha * acc[i][j][r];
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
  }
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_nt_dl(const NtArgs& g, hipStream_t s) {
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long grid_x = ((nb + 7) / 8) * 8;
  if (grid_x > INT_MAX || g.batch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)grid_x, 1, (unsigned)g.batch);
  hipLaunchKernelGGL((gemm_nt_f64_dl_kernel<BM, BN, WM, WN>), grid, dim3(64 * WM * WN), 0, s, g, tiles_m, tiles_n);
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_nt(const NtArgs& g, Prec prec, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (prec != Prec::F64) return hipErrorInvalidValue;
  // 16-byte loads: A rows (and B rows, or B's N for [K][N] storage) in pairs, 16-byte aligned
  if (g.K <= 0 || (g.K & 1) || (g.lda & 1) || (g.ldb & 1) || (g.a_batch & 1) || (g.b_batch & 1) ||
      ((uintptr_t)g.A & 15) || ((uintptr_t)g.B & 15) || (g.b_kn && (g.N & 1)))
    return hipErrorInvalidValue;
  if (g.b_map && (!g.b_kn || g.bnm.s_lo != 1 || (g.bnm.inner != 0 && (g.bnm.inner & 1)) || (g.bnm.s_hi & 1)))
    return hipErrorInvalidValue;
  const long long nb = g.batch - 1;
  if (g.a_len > 0 && nb * g.a_batch + (long long)(g.M - 1) * g.lda + g.K > g.a_len) return hipErrorInvalidValue;
  if (g.b_len > 0 && !g.b_kn && nb * g.b_batch + (long long)(g.N - 1) * g.ldb + g.K > g.b_len)
    return hipErrorInvalidValue;
  if (g.b_len > 0 && g.b_kn && nb * g.b_batch + (long long)(g.K - 1) * g.ldb + (g.b_map ? idx_max(g.bnm, g.N) + 1 : g.N) >
                                   g.b_len)
    return hipErrorInvalidValue;
  if (g.c_len > 0 && nb * g.c_batch + idx_max(g.cm, g.M) + idx_max(g.cn, g.N) >= g.c_len) return hipErrorInvalidValue;
  // variants 9, 10 and 11: the 128 x 256, 192 x 256 and 128 x 192 tiles with
  // the operands copied straight into LDS (both operands K-contiguous, K a
  // multiple of 16)
  const bool dl_ok = !g.b_kn && g.K % BK == 0;
  int variant = g.variant;
  if (variant == 0) {
    // score each tile shape by the fraction of its MFMA work that lands inside
    // the matrix (skinny M or N wastes most of a large tile), by how well its
    // tile count fills the chip (two workgroups on each of 256 CUs), and by
    // the measured relative speed of the shape on full tiles (an M or N of
    // v = 180 virtual labels fills 94 % of 192, 70 % of 256)
    struct Cand { int var, bm, bn; double speed; };
    const Cand cands[9] = {{9, 128, 256, 1.10}, {10, 192, 256, 1.10}, {11, 128, 192, 1.10},
                           {1, 128, 256, 1.00}, {2, 256, 128, 1.00},  {4, 128, 128, 0.96},
                           {3, 64, 64, 0.86},   {5, 256, 32, 0.80},   {6, 32, 256, 0.80}};
    double best = -1.0;
    for (const Cand& c : cands) {
      if (c.var >= 9 && !dl_ok) continue;
      const long long tm = (g.M + c.bm - 1) / c.bm, tn = (g.N + c.bn - 1) / c.bn;
      const double used = ((double)g.M / (double)(tm * c.bm)) * ((double)g.N / (double)(tn * c.bn));
      const double tiles = (double)(tm * tn * g.batch);
      const double fill = tiles >= 512.0 ? 1.0 : tiles / 512.0;
      const double score = used * fill * c.speed;
      if (score > best) { best = score; variant = c.var; }
    }
  }
  if (variant >= 9 && variant <= 11 && !dl_ok) variant = 1;
  switch (variant) {
    case 9: return launch_nt_dl<128, 256, 2, 4>(g, s);
    case 10: return launch_nt_dl<192, 256, 2, 4>(g, s);
    case 11: return launch_nt_dl<128, 192, 2, 4>(g, s);
    case 1: return launch_nt<128, 256, 2, 4, 2>(g, s);
    case 2: return launch_nt<256, 128, 4, 2, 2>(g, s);
    case 3: return launch_nt<64, 64, 2, 2, 2>(g, s);
    case 5: return launch_nt<256, 32, 4, 1, 2>(g, s);  // N of a few tens: 64 x 32 per wave
    case 6: return launch_nt<32, 256, 1, 4, 2>(g, s);  // M of a few tens: 32 x 64 per wave
    default: return launch_nt<128, 128, 2, 2, 2>(g, s);
  }
}

}  // namespace cct

// ===========================================================================
// K-contiguous kernels on low-precision operands stored in memory.
//   FP32 operands: 16-byte loads of 4 floats, K tile of 32, FP32 MFMA with
//   FP32 accumulation over LP_FLUSH K tiles and an FP64 flush after them.
//   Split-BF16 operands: hi and lo planes, 16-byte loads of 8 bf16 per plane,
//   K tile of 32 (one bf16 MFMA step), three products per tile, FP32
//   accumulation over the whole K (the kernel keeps an FP64 flush as an
//   option, unused by the library).
// ===========================================================================
namespace cct {
namespace {

// K tiles accumulated in FP32 before the FP64 flush (K = 4 x 32 = 128 products)
constexpr int LP_FLUSH = 4;

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int BM, int BN, int WM, int WN, int OCC, bool VEC>
__global__ __launch_bounds__(64 * WM * WN, OCC) void gemm_lp_f32_kernel(NtLpArgs g, int tiles_m, int tiles_n) {
  constexpr int NTH = 64 * WM * WN, TM = BM / WM / 16, TN = BN / WN / 16, KB = 32, LA = BM + 4, LB = BN + 4;
  constexpr int SA = BM * (KB / 4) / NTH, SB = BN * (KB / 4) / NTH;  // 16-byte segments per thread
  __shared__ float As[2][KB * LA];
  __shared__ float Bs[2][KB * LB];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x, b = blockIdx.z;
  const float* A = (const float*)g.A + (long long)b * g.a_batch;
  const float* B = (const float*)g.B + (long long)b * g.b_batch;
  const float* pa[SA];
  const float* pb[SB];
  int ka[SA], kb[SB];
  bool va[SA], vb[SB];
#pragma unroll
  for (int i = 0; i < SA; ++i) {
    const int seg = tid + i * NTH, row = seg / (KB / 4);
    ka[i] = 4 * (seg % (KB / 4));
    const int m = tm * BM + row;
    va[i] = m < g.M;
    pa[i] = A + (long long)(va[i] ? m : 0) * g.lda + ka[i];
  }
#pragma unroll
  for (int i = 0; i < SB; ++i) {
    const int seg = tid + i * NTH, row = seg / (KB / 4);
    kb[i] = 4 * (seg % (KB / 4));
    const int n = tn * BN + row;
    vb[i] = n < g.N;
    pb[i] = B + (long long)(vb[i] ? n : 0) * g.ldb + kb[i];
  }
  const int wave = tid / 64, lane = tid & 63;
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  double out[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[i][j][r] = 0.0;
  flt4 ra[SA], rb[SB];
  bool oa[SA], ob[SB];
  const int nk = (g.K + KB - 1) / KB;
  auto load = [&](int k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < SA; ++i) { oa[i] = va[i] && (k0 + ka[i] < g.K); ra[i] = *(const flt4*)(pa[i] + (oa[i] ? k0 : 0)); }
#pragma unroll
      for (int i = 0; i < SB; ++i) { ob[i] = vb[i] && (k0 + kb[i] < g.K); rb[i] = *(const flt4*)(pb[i] + (ob[i] ? k0 : 0)); }
    } else {
      // any K, leading dimension and alignment: element loads, masked per element
#pragma unroll
      for (int i = 0; i < SA; ++i) {
        oa[i] = true;
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[i][q] = (va[i] && k0 + ka[i] + q < g.K) ? pa[i][k0 + q] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        ob[i] = true;
#pragma unroll
        for (int q = 0; q < 4; ++q) rb[i][q] = (vb[i] && k0 + kb[i] + q < g.K) ? pb[i][k0 + q] : 0.f;
      }
    }
  };
  auto store = [&](float* as, float* bs) {
#pragma unroll
    for (int i = 0; i < SA; ++i) {
      const int row = (tid + i * NTH) / (KB / 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) as[(ka[i] + q) * LA + row] = oa[i] ? ra[i][q] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < SB; ++i) {
      const int row = (tid + i * NTH) / (KB / 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) bs[(kb[i] + q) * LB + row] = ob[i] ? rb[i][q] : 0.f;
    }
  };
  load(0);
  store(As[0], Bs[0]);
  __syncthreads();
  f4 acc[TM][TN];
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * KB);
    const float* as = As[cur];
    const float* bs = Bs[cur];
    if (kt % LP_FLUSH == 0) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int ks = 0; ks < KB / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      float af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = as[kr * LA + wm0 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = bs[kr * LB + wn0 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt % LP_FLUSH == LP_FLUSH - 1 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[i][j][r] += (double)acc[i][j][r];
    }
    if (kt + 1 < nk) store(As[cur ^ 1], Bs[cur ^ 1]);
    __syncthreads();
  }
  const long long coff = (long long)b * g.c_batch;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = tm * BM + wm0 + i * 16 + 4 * (lane / 16) + r;
      if (m >= g.M) continue;
      const long long mo = coff + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        double* p = g.C + mo + map2(g.cn, n);
        const double x = g.alpha * out[i][j][r];
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
}

// The FP32 kernel with the operand tiles copied from global memory straight
// into LDS (no register staging, no LDS stores), for K a multiple of 32.  An
// LDS row holds one K tile of one matrix row: 32 floats as eight 16-byte
// slots, slot p at position p ^ ((row >> 1) & 7); the 16 x 16 x 4 fragment
// reads (16 consecutive rows per 16 lanes, k = lane / 16 within a group of 4)
// then fall on 64 distinct banks.  Each wave copies whole 1 KB chunks (8 rows);
// lane s of a chunk lands in row s / 8 at position s % 8 and fetches the slot
// that the swizzle keeps there.  Rows past the matrix are read from row 0
// (their outputs are not stored).  FP32 accumulation over LP_FLUSH K tiles,
// then FP64, as in the register-staged kernel.
__device__ __forceinline__ int f32_swz(int row, int k) { return row * 32 + 4 * ((k >> 2) ^ ((row >> 1) & 7)) + (k & 3); }

template <int BM, int BN, int WM, int WN, int OCC>
__global__ __launch_bounds__(64 * WM * WN, OCC) void gemm_lp_f32_dl_kernel(NtLpArgs g, int tiles_m, int tiles_n) {
  constexpr int NW = WM * WN, TM = BM / WM / 16, TN = BN / WN / 16, KB = 32;
  constexpr int CA = BM / 8, CB = BN / 8;  // 1 KB chunks per K tile
  static_assert(CA % NW == 0 && CB % NW == 0, "whole chunks per wave");
  constexpr int PA = CA / NW, PB = CB / NW;
  constexpr int ABUF = BM * KB, BBUF = BN * KB;  // floats per buffer
  __shared__ __attribute__((aligned(1024))) float As[2 * ABUF];
  __shared__ __attribute__((aligned(1024))) float Bs[2 * BBUF];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x, b = blockIdx.z;
  const int wave = tid / 64, lane = tid & 63;
  const float* A = (const float*)g.A + (long long)b * g.a_batch;
  const float* B = (const float*)g.B + (long long)b * g.b_batch;
  const float* sa[PA];
  const float* sb[PB];
  unsigned la[PA], lb[PB];
  const unsigned as0 = (unsigned)(size_t)(__attribute__((address_space(3))) const void*)As;
  const unsigned bs0 = (unsigned)(size_t)(__attribute__((address_space(3))) const void*)Bs;
#pragma unroll
  for (int j = 0; j < PA; ++j) {
    const int c = wave + NW * j, row = c * 8 + lane / 8, kp = (lane % 8) ^ ((row >> 1) & 7);
    const int m = tm * BM + row;
    sa[j] = A + (long long)(m < g.M ? m : 0) * g.lda + 4 * kp;
    la[j] = __builtin_amdgcn_readfirstlane(as0 + 4u * (unsigned)(c * 8 * KB));
  }
#pragma unroll
  for (int j = 0; j < PB; ++j) {
    const int c = wave + NW * j, row = c * 8 + lane / 8, kp = (lane % 8) ^ ((row >> 1) & 7);
    const int n = tn * BN + row;
    sb[j] = B + (long long)(n < g.N ? n : 0) * g.ldb + 4 * kp;
    lb[j] = __builtin_amdgcn_readfirstlane(bs0 + 4u * (unsigned)(c * 8 * KB));
  }
  auto issue = [&](int kt, int buf) {
    const long long k0 = (long long)kt * KB;
    const unsigned da = buf * (4u * ABUF), db = buf * (4u * BBUF);  // bytes
#pragma unroll
    for (int j = 0; j < PA; ++j) lds_copy16(sa[j] + k0, la[j] + da);
#pragma unroll
    for (int j = 0; j < PB; ++j) lds_copy16(sb[j] + k0, lb[j] + db);
  };
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  double out[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) out[i][j][r] = 0.0;
  f4 acc[TM][TN];
  const int nk = g.K / KB;
  issue(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) issue(kt + 1, cur ^ 1);
    const float* as = As + cur * ABUF;
    const float* bs = Bs + cur * BBUF;
    if (kt % LP_FLUSH == 0) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int ks = 0; ks < KB / 4; ++ks) {
      const int kr = ks * 4 + lane / 16;
      float af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = as[f32_swz(wm0 + i * 16 + (lane & 15), kr)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = bs[f32_swz(wn0 + j * 16 + (lane & 15), kr)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt % LP_FLUSH == LP_FLUSH - 1 || kt + 1 == nk) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) out[i][j][r] += (double)acc[i][j][r];
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  const long long coff = (long long)b * g.c_batch;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = tm * BM + wm0 + i * 16 + 4 * (lane / 16) + r;
      if (m >= g.M) continue;
      const long long mo = coff + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        double* p = g.C + mo + map2(g.cn, n);
        const double x = g.alpha * out[i][j][r];
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
}

template <int BM, int BN, int WM, int WN, int OCC>
hipError_t launch_lp_f32_dl(const NtLpArgs& g, hipStream_t s) {
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long grid_x = ((nb + 7) / 8) * 8;
  if (grid_x > INT_MAX || g.batch > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid_x, 1, (unsigned)g.batch);
  hipLaunchKernelGGL((gemm_lp_f32_dl_kernel<BM, BN, WM, WN, OCC>), grid, dim3(64 * WM * WN), 0, s, g, tiles_m, tiles_n);
  return hipGetLastError();
}

// LDS rows of the split-BF16 kernel hold one K tile (32 values, four 16-byte
// segments) unpadded; segment q of row r sits at position q ^ ((r >> 1) & 3).
// On gfx950 this is free of bank conflicts for both 16-byte accesses the
// kernel makes: the fragment reads (16 consecutive rows, one segment per 16
// lanes) and the tile stores (4 rows x 4 segments per 16 lanes).  Rows padded
// to 40 values conflict on both (2x the LDS cycles per instruction).
__device__ __forceinline__ int lp_swz(int row, int q) { return row * 32 + 8 * (q ^ ((row >> 1) & 3)); }

template <int BM, int BN, int WM, int WN, int OCC, bool VEC, bool ACC64, int PF>
__global__ __launch_bounds__(64 * WM * WN, OCC) void gemm_lp_bf16x3_kernel(NtLpArgs g, int tiles_m, int tiles_n) {
  static_assert(PF == 1 || PF == 2, "one or two load stages");
  constexpr int NTH = 64 * WM * WN, TM = BM / WM / 16, TN = BN / WN / 16, KB = 32, LK = KB;
  constexpr int SA = BM * (KB / 8) / NTH, SB = BN * (KB / 8) / NTH;  // 16-byte segments per plane per thread
  __shared__ __attribute__((aligned(16))) __bf16 As[2][2][BM * LK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][2][BN * LK];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x, b = blockIdx.z;
  const __bf16* A = (const __bf16*)g.A + (long long)b * g.a_batch;
  const __bf16* B = (const __bf16*)g.B + (long long)b * g.b_batch;
  const __bf16* pa[SA];
  const __bf16* pb[SB];
  int ka[SA], kb[SB], rowa[SA], rowb[SB];
  bool va[SA], vb[SB];
#pragma unroll
  for (int i = 0; i < SA; ++i) {
    const int seg = tid + i * NTH;
    rowa[i] = seg / (KB / 8);
    ka[i] = 8 * (seg % (KB / 8));
    const int m = tm * BM + rowa[i];
    va[i] = m < g.M;
    pa[i] = A + (long long)(va[i] ? m : 0) * g.lda + ka[i];
  }
#pragma unroll
  for (int i = 0; i < SB; ++i) {
    const int seg = tid + i * NTH;
    rowb[i] = seg / (KB / 8);
    kb[i] = 8 * (seg % (KB / 8));
    const int n = tn * BN + rowb[i];
    vb[i] = n < g.N;
    pb[i] = B + (long long)(vb[i] ? n : 0) * g.ldb + kb[i];
  }
  const int wave = tid / 64, lane = tid & 63;
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  // ACC64: FP32 accumulators flushed into FP64 every LP_FLUSH K tiles;
  // otherwise FP32 accumulation over the whole K (no FP64 registers)
  double out[ACC64 ? TM : 1][ACC64 ? TN : 1][4];
  if constexpr (ACC64) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) out[i][j][r] = 0.0;
  }
  // PF register stages of global loads.  With two, the tile of K step t + 1
  // waits in one while the loads of step t + 2 are in flight into the other,
  // so each global load has two K steps of matrix-core work to arrive in.
  struct Stage {
    u32x4 ah[SA], al[SA], bh[SB], bl[SB];
    bool oa[SA], ob[SB];
  };
  Stage S0, S1;
  const int nk = (g.K + KB - 1) / KB;
  // planar operands: K tile t starts t * 32 elements into the row; blocked
  // (hi 32, lo 32) operands: t * 64, with the lo values 32 further on
  const int kmul = g.il ? 2 : 1;
  auto load = [&](Stage& st, int k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int i = 0; i < SA; ++i) {
        st.oa[i] = va[i] && (k0 + ka[i] < g.K);
        const __bf16* p = pa[i] + (st.oa[i] ? kmul * k0 : 0);
        st.ah[i] = *(const u32x4*)p;
        st.al[i] = *(const u32x4*)(p + g.a_plane);
      }
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        st.ob[i] = vb[i] && (k0 + kb[i] < g.K);
        const __bf16* p = pb[i] + (st.ob[i] ? kmul * k0 : 0);
        st.bh[i] = *(const u32x4*)p;
        st.bl[i] = *(const u32x4*)(p + g.b_plane);
      }
    } else {
      // any K, leading dimension and alignment: element loads, masked per element
      const __bf16 z = (__bf16)0.f;
#pragma unroll
      for (int i = 0; i < SA; ++i) {
        st.oa[i] = true;
        __bf16 h[8], l[8];
        const __bf16* p = pa[i] + kmul * k0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool ok = va[i] && k0 + ka[i] + q < g.K;
          h[q] = ok ? p[q] : z;
          l[q] = ok ? p[q + g.a_plane] : z;
        }
        __builtin_memcpy(&st.ah[i], h, 16);
        __builtin_memcpy(&st.al[i], l, 16);
      }
#pragma unroll
      for (int i = 0; i < SB; ++i) {
        st.ob[i] = true;
        __bf16 h[8], l[8];
        const __bf16* p = pb[i] + kmul * k0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const bool ok = vb[i] && k0 + kb[i] + q < g.K;
          h[q] = ok ? p[q] : z;
          l[q] = ok ? p[q + g.b_plane] : z;
        }
        __builtin_memcpy(&st.bh[i], h, 16);
        __builtin_memcpy(&st.bl[i], l, 16);
      }
    }
  };
  const u32x4 zero4 = {0u, 0u, 0u, 0u};
  auto store = [&](const Stage& st, int buf) {
#pragma unroll
    for (int i = 0; i < SA; ++i) {
      const int at = lp_swz(rowa[i], ka[i] / 8);
      *(u32x4*)&As[buf][0][at] = st.oa[i] ? st.ah[i] : zero4;
      *(u32x4*)&As[buf][1][at] = st.oa[i] ? st.al[i] : zero4;
    }
#pragma unroll
    for (int i = 0; i < SB; ++i) {
      const int at = lp_swz(rowb[i], kb[i] / 8);
      *(u32x4*)&Bs[buf][0][at] = st.ob[i] ? st.bh[i] : zero4;
      *(u32x4*)&Bs[buf][1][at] = st.ob[i] ? st.bl[i] : zero4;
    }
  };
  const int kq = lane / 16;  // the lane's 16-byte segment of the K tile
  f4 acc[TM][TN];
  // one K step out of LDS buffer cur: all B fragments of the wave, then one A
  // fragment at a time; each accumulator takes its three products (lo*hi,
  // hi*lo, hi*hi, in that order) TN launches apart
  auto compute = [&](int kt, int cur) {
    if (kt == 0 || (ACC64 && kt % LP_FLUSH == 0)) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
    bf8 bh[TN], bl[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = wn0 + j * 16 + (lane & 15);
      bh[j] = *(const bf8*)&Bs[cur][0][lp_swz(col, kq)];
      bl[j] = *(const bf8*)&Bs[cur][1][lp_swz(col, kq)];
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int row = wm0 + i * 16 + (lane & 15);
      const bf8 ah = *(const bf8*)&As[cur][0][lp_swz(row, kq)];
      const bf8 al = *(const bf8*)&As[cur][1][lp_swz(row, kq)];
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
    }
    if constexpr (ACC64) {
      if (kt % LP_FLUSH == LP_FLUSH - 1 || kt + 1 == nk) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[i][j][r] += (double)acc[i][j][r];
      }
    }
  };
  // K step t sits in LDS buffer t & 1.
  if constexpr (PF == 1) {
    // one stage: the loads of step t + 1 fly during step t's products
    load(S0, 0);
    store(S0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) load(S0, (kt + 1) * KB);
      compute(kt, kt & 1);
      if (kt + 1 < nk) store(S0, (kt + 1) & 1);
      __syncthreads();
    }
  } else {
    // two stages: on entry to step t the tile of step t + 1 is in S1 (t even)
    // or S0 (t odd) and the loads of step t + 2 are in flight into the other;
    // after step t's products the waiting stage goes to LDS and is refilled
    // with step t + 3
    load(S0, 0);
    if (nk > 1) load(S1, KB);
    store(S0, 0);
    if (nk > 2) load(S0, 2 * KB);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
      compute(kt, 0);
      if (kt + 1 < nk) {
        store(S1, 1);
        if (kt + 3 < nk) load(S1, (kt + 3) * KB);
      }
      __syncthreads();
      if (kt + 1 >= nk) break;
      compute(kt + 1, 1);
      if (kt + 2 < nk) {
        store(S0, 0);
        if (kt + 4 < nk) load(S0, (kt + 4) * KB);
      }
      __syncthreads();
    }
  }
  const long long coff = (long long)b * g.c_batch;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = tm * BM + wm0 + i * 16 + 4 * (lane / 16) + r;
      if (m >= g.M) continue;
      const long long mo = coff + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        const double x = g.alpha * (ACC64 ? out[ACC64 ? i : 0][ACC64 ? j : 0][r] : (double)acc[i][j][r]);
        if (!ACC64 && g.C32) {
          g.C32[mo + map2(g.cn, n)] = (float)x;
          continue;
        }
        double* p = g.C + mo + map2(g.cn, n);
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
}

// The split-BF16 kernel with the operand tiles copied from global memory
// straight into LDS (16 bytes per lane, no register staging and no LDS store
// instructions), for K a multiple of 32, two tile buffers.  Each wave copies
// whole 1 KB chunks of a tile (16 rows of one plane); lane s of a chunk lands
// at byte 16 s of it, i.e. in row s / 4 at segment position s % 4, so the lane
// fetches the logical segment (s % 4) ^ ((row >> 1) & 3) that the swizzled
// layout keeps there.  Rows past the matrix are read from row 0 (finite
// values whose products go to outputs that are not stored).  FP32
// accumulation over the whole K.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, 1) void gemm_lp_bf16x3_dl_kernel(NtLpArgs g, int tiles_m, int tiles_n) {
  constexpr int NW = WM * WN, TM = BM / WM / 16, TN = BN / WN / 16, KB = 32;
  constexpr int CA = 2 * BM / 16, CB = 2 * BN / 16;  // 1 KB chunks per K tile (both planes)
  static_assert(CA % NW == 0 && CB % NW == 0, "whole chunks per wave");
  constexpr int PA = CA / NW, PB = CB / NW;  // chunks per wave per step
  constexpr int ABUF = 2 * BM * KB, BBUF = 2 * BN * KB;  // elements per buffer (planes hi, lo)
  __shared__ __attribute__((aligned(1024))) __bf16 As[2 * ABUF];
  __shared__ __attribute__((aligned(1024))) __bf16 Bs[2 * BBUF];
  int tm, tn;
  if (!tile_coords(tiles_m, tiles_n, tm, tn)) return;
  const int tid = threadIdx.x, b = blockIdx.z;
  const int wave = tid / 64, lane = tid & 63;
  const __bf16* A = (const __bf16*)g.A + (long long)b * g.a_batch;
  const __bf16* B = (const __bf16*)g.B + (long long)b * g.b_batch;
  const int kmul = g.il ? 2 : 1;
  // per chunk: the lane's source (K step 0) and the chunk's LDS byte address
  // in buffer 0 (wave-uniform)
  const __bf16* sa[PA];
  const __bf16* sb[PB];
  unsigned la[PA], lb[PB];
  const unsigned as0 = lds_addr(As), bs0 = lds_addr(Bs);
#pragma unroll
  for (int j = 0; j < PA; ++j) {
    const int c = wave + NW * j, pl = c / (BM / 16), cc = c % (BM / 16);
    const int row = cc * 16 + lane / 4, q = (lane % 4) ^ ((row >> 1) & 3);
    const int m = tm * BM + row;
    sa[j] = A + (long long)(m < g.M ? m : 0) * g.lda + 8 * q + (pl ? g.a_plane : 0);
    la[j] = __builtin_amdgcn_readfirstlane(as0 + 2u * (unsigned)(pl * BM * KB + cc * 16 * KB));
  }
#pragma unroll
  for (int j = 0; j < PB; ++j) {
    const int c = wave + NW * j, pl = c / (BN / 16), cc = c % (BN / 16);
    const int row = cc * 16 + lane / 4, q = (lane % 4) ^ ((row >> 1) & 3);
    const int n = tn * BN + row;
    sb[j] = B + (long long)(n < g.N ? n : 0) * g.ldb + 8 * q + (pl ? g.b_plane : 0);
    lb[j] = __builtin_amdgcn_readfirstlane(bs0 + 2u * (unsigned)(pl * BN * KB + cc * 16 * KB));
  }
  const int nk = g.K / KB;
  auto issue = [&](int kt, int buf) {
    const long long k0 = (long long)kmul * kt * KB;
    const unsigned da = buf * (2u * ABUF), db = buf * (2u * BBUF);  // bytes
#pragma unroll
    for (int j = 0; j < PA; ++j) lds_copy16(sa[j] + k0, la[j] + da);
#pragma unroll
    for (int j = 0; j < PB; ++j) lds_copy16(sb[j] + k0, lb[j] + db);
  };
  const int wm0 = (wave / WN) * (BM / WM), wn0 = (wave % WN) * (BN / WN);
  const int kq = lane / 16;
  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto compute = [&](const __bf16* Ac, const __bf16* Bc) {
    bf8 bh[TN], bl[TN];
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = wn0 + j * 16 + (lane & 15);
      bh[j] = *(const bf8*)&Bc[lp_swz(col, kq)];
      bl[j] = *(const bf8*)&Bc[BN * KB + lp_swz(col, kq)];
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int row = wm0 + i * 16 + (lane & 15);
      const bf8 ah = *(const bf8*)&Ac[lp_swz(row, kq)];
      const bf8 al = *(const bf8*)&Ac[BM * KB + lp_swz(row, kq)];
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
    }
  };
  // Step t multiplies out of buffer t & 1 while the copies of step t + 1 fill
  // the other (last read in step t - 1, before the barrier); each wave then
  // waits for its own copies, and the barrier for everyone's.
  issue(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) issue(kt + 1, cur ^ 1);
    compute(As + cur * ABUF, Bs + cur * BBUF);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  const long long coff = (long long)b * g.c_batch;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = tm * BM + wm0 + i * 16 + 4 * (lane / 16) + r;
      if (m >= g.M) continue;
      const long long mo = coff + map2(g.cm, m);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = tn * BN + wn0 + j * 16 + (lane & 15);
        if (n >= g.N) continue;
        const double x = g.alpha * (double)acc[i][j][r];
        if (g.C32) {
          g.C32[mo + map2(g.cn, n)] = (float)x;
          continue;
        }
        double* p = g.C + mo + map2(g.cn, n);
        *p = (g.beta == 0.0) ? x : x + g.beta * *p;
      }
    }
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_lp_dl(const NtLpArgs& g, hipStream_t s) {
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long grid_x = ((nb + 7) / 8) * 8;
  if (grid_x > INT_MAX || g.batch > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid_x, 1, (unsigned)g.batch);
  hipLaunchKernelGGL((gemm_lp_bf16x3_dl_kernel<BM, BN, WM, WN>), grid, dim3(64 * WM * WN), 0, s, g, tiles_m, tiles_n);
  return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int OCC, bool VEC, bool ACC64 = true, int PF = 2>
hipError_t launch_lp(const NtLpArgs& g, Prec prec, hipStream_t s) {
  const int tiles_m = (g.M + BM - 1) / BM, tiles_n = (g.N + BN - 1) / BN;
  const long long nb = (long long)tiles_m * tiles_n;
  const long long grid_x = ((nb + 7) / 8) * 8;
  if (grid_x > INT_MAX || g.batch > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)grid_x, 1, (unsigned)g.batch);
  if (prec == Prec::F32)
    hipLaunchKernelGGL((gemm_lp_f32_kernel<BM, BN, WM, WN, OCC, VEC>), grid, dim3(64 * WM * WN), 0, s, g, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((gemm_lp_bf16x3_kernel<BM, BN, WM, WN, OCC, VEC, ACC64, PF>), grid, dim3(64 * WM * WN), 0, s, g,
                       tiles_m, tiles_n);
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_nt_lp(const NtLpArgs& g_in, Prec prec, hipStream_t s) {
  if (g_in.M <= 0 || g_in.N <= 0 || g_in.batch <= 0) return hipSuccess;
  if (prec == Prec::F64 || g_in.K <= 0) return hipErrorInvalidValue;
  NtLpArgs g = g_in;
  if (g.il) {
    // blocked split-BF16 operands (OUT_BF16X2I): the caller's strides and
    // lengths count logical elements; rows, batch strides and lengths have to
    // hold whole blocks of 32, and the stored rows are twice as long
    if (prec != Prec::BF16X3 || g.lda % 32 || g.ldb % 32 || g.a_batch % 32 || g.b_batch % 32 || g.a_len % 32 ||
        g.b_len % 32)
      return hipErrorInvalidValue;
  } else if (prec == Prec::BF16X3 && (g.a_plane <= 0 || g.b_plane <= 0)) {
    return hipErrorInvalidValue;
  }
  // FP32 output only where it is exact: FP32 accumulation (split BF16), no read of C
  if (g.C32 && (prec != Prec::BF16X3 || g.beta != 0.0 || g.alpha != 1.0)) return hipErrorInvalidValue;
  const long long nb = g.batch - 1;
  if (g.a_len > 0 && nb * g.a_batch + (long long)(g.M - 1) * g.lda + g.K > g.a_len) return hipErrorInvalidValue;
  if (g.b_len > 0 && nb * g.b_batch + (long long)(g.N - 1) * g.ldb + g.K > g.b_len) return hipErrorInvalidValue;
  if (g.c_len > 0 && nb * g.c_batch + idx_max(g.cm, g.M) + idx_max(g.cn, g.N) >= g.c_len) return hipErrorInvalidValue;
  if (g.il) {
    g.lda *= 2;
    g.ldb *= 2;
    g.a_batch *= 2;
    g.b_batch *= 2;
    g.a_plane = g.b_plane = 32;
  }
  // 16-byte vector loads need K, leading dimensions, batch strides and planes
  // in multiples of the vector width and 16-byte aligned bases
  const int w = prec == Prec::F32 ? 4 : 8;
  const bool vec = !(g.K % w || g.lda % w || g.ldb % w || g.a_batch % w || g.b_batch % w ||
                     ((uintptr_t)g.A & 15) || ((uintptr_t)g.B & 15) ||
                     (prec == Prec::BF16X3 && (g.a_plane % w || g.b_plane % w)));
  // FP32 operands: FP32 accumulation over LP_FLUSH K tiles, then FP64.
  // Split-BF16 operands: FP32 accumulation over the whole K (the three
  // products of the split already carry ~2^-17 relative rounding).
  if (prec == Prec::F32) {
    if (!vec) return launch_lp<64, 64, 2, 2, 2, false, true>(g, prec, s);
    int variant = g.variant;
    if (variant == 0) {
      // 128 x 128 tiles of 8 waves (64 x 32 each, two waves per SIMD) once
      // there are enough of them, with the operands copied straight into LDS
      // where K is a multiple of 32; 64 x 64 below that
      const long long t128 = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch;
      variant = t128 >= 256 ? (g.K % 32 == 0 ? 5 : 2) : 3;
    }
    if (variant == 5 && g.K % 32 != 0) variant = 2;
    switch (variant) {
      case 5: return launch_lp_f32_dl<128, 128, 2, 4, 2>(g, s);
      case 1: return launch_lp<128, 128, 2, 2, 1, true, true>(g, prec, s);
      case 2: return launch_lp<128, 128, 2, 4, 2, true, true>(g, prec, s);
      default: return launch_lp<64, 64, 2, 2, 2, true, true>(g, prec, s);
    }
  }
  if (!vec) return launch_lp<64, 64, 2, 2, 2, false, false>(g, prec, s);
  int variant = g.variant;
  if (variant == 0) {
    // 256 x 256 tiles of 8 waves (128 x 64 each; the two LDS buffers take
    // the whole 160 KB) once there are enough of them, then 256 x 128, ...
    const long long t2x2 = (long long)((g.M + 255) / 256) * ((g.N + 255) / 256) * g.batch;
    const long long t256 = (long long)((g.M + 255) / 256) * ((g.N + 127) / 128) * g.batch;
    const long long t128 = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch;
    variant = t2x2 >= 256 ? (g.K % 32 == 0 ? 5 : 4) : (t256 >= 256 ? 1 : (t128 >= 256 ? 2 : 3));
  }
  // the 256 x 256 tile keeps one load stage (two need more than the 256
  // registers a wave has at two waves per SIMD); variant 5 is the same tile
  // with the operands copied straight into LDS, where K is a multiple of 32
  if (variant == 5 && g.K % 32 != 0) variant = 4;
  switch (variant) {
    case 5: return launch_lp_dl<256, 256, 2, 4>(g, s);
    case 4: return launch_lp<256, 256, 2, 4, 1, true, false, 1>(g, prec, s);
    case 1: return launch_lp<256, 128, 4, 2, 1, true, false, 2>(g, prec, s);
    case 2: return launch_lp<128, 128, 2, 4, 2, true, false, 2>(g, prec, s);
    default: return launch_lp<64, 64, 2, 2, 2, true, false, 2>(g, prec, s);
  }
}

}  // namespace cct
