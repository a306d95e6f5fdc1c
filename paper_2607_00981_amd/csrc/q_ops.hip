// Bandwidth kernels of the perturbative quadruples correction: permuted
// combinations of v^4 virtual blocks.
#include "internal.h"

namespace cct {

namespace {

constexpr int QT = 8;  // tile edge along each of the four virtual axes
// LDS pitches of the padded 8^4 tile (one extra double per level keeps
// permuted reads across lanes off a single bank)
constexpr int QS2 = QT + 1;
constexpr int QS1 = QT * QS2 + 1;
constexpr int QS0 = QT * QS1 + 1;
constexpr int QTPB = 256;
constexpr int QPER = QT * QT * QT * QT / QTPB;  // output elements per thread

template <bool TILED>
__global__ __launch_bounds__(QTPB) void perm_combine_kernel(double* __restrict__ out, double* __restrict__ out2,
                                                            QCombineArgs a, int nt) {
  __shared__ double L[QT * QS0];
  const int v = a.v;
  const long long v1 = v, v2 = v1 * v, v3 = v2 * v;
  int tile = blockIdx.x;
  int org[4];
  for (int d = 3; d >= 0; --d) {
    org[d] = (tile % nt) * QT;
    tile /= nt;
  }
  double acc[QPER], acc2[QPER];
#pragma unroll
  for (int e = 0; e < QPER; ++e) acc[e] = acc2[e] = 0.0;

  // the global loads of term t+1 are issued into registers before term t is
  // computed from LDS, so their latency overlaps that work
  double pre[QPER];
  auto load_term = [&](int t) {
    const QPermTerm& T = a.t[t];
    int sorg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) sorg[k] = org[T.perm[k]];
    if (TILED) {
      // the source tile is one contiguous run of 4096 doubles; its padding
      // positions only reach outputs outside [0, v)^4, which are not stored
      const long long ti = (((long long)(sorg[0] >> 3) * nt + (sorg[1] >> 3)) * nt + (sorg[2] >> 3)) * nt +
                           (sorg[3] >> 3);
      const double* src = T.in + ti * 4096;
#pragma unroll
      for (int e = 0; e < QPER; ++e) pre[e] = src[threadIdx.x + e * QTPB];
      return;
    }
#pragma unroll
    for (int e = 0; e < QPER; ++e) {
      const int lin = threadIdx.x + e * QTPB;
      const int m3 = lin & 7, m2 = (lin >> 3) & 7, m1 = (lin >> 6) & 7, m0 = lin >> 9;
      const int y0 = sorg[0] + m0, y1 = sorg[1] + m1, y2 = sorg[2] + m2, y3 = sorg[3] + m3;
      pre[e] = (y0 < v && y1 < v && y2 < v && y3 < v) ? T.in[y0 * v3 + y1 * v2 + y2 * v1 + y3] : 0.0;
    }
  };
  load_term(0);
  for (int t = 0; t < a.nterms; ++t) {
    const QPermTerm& T = a.t[t];
    // source tile: in-index y_k = w_{perm[k]} runs over org[perm[k]] + [0, QT)
    int sorg[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) sorg[k] = org[T.perm[k]];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < QPER; ++e) {
      const int lin = threadIdx.x + e * QTPB;
      const int m3 = lin & 7, m2 = (lin >> 3) & 7, m1 = (lin >> 6) & 7, m0 = lin >> 9;
      L[m0 * QS0 + m1 * QS1 + m2 * QS2 + m3] = pre[e];
    }
    __syncthreads();
    if (t + 1 < a.nterms) load_term(t + 1);
#pragma unroll
    for (int e = 0; e < QPER; ++e) {
      const int lin = threadIdx.x + e * QTPB;
      const int l[4] = {lin >> 9, (lin >> 6) & 7, (lin >> 3) & 7, lin & 7};
      const int p0 = l[T.perm[0]], p1 = l[T.perm[1]], p2 = l[T.perm[2]], p3 = l[T.perm[3]];
      const double x = L[p0 * QS0 + p1 * QS1 + p2 * QS2 + p3];
      if (T.dst & 1) acc[e] += T.coef * x;
      if (T.dst & 2) {
        double y = x;
        if (T.va) {
          const int y0 = sorg[0] + p0, y1 = sorg[1] + p1, y2 = sorg[2] + p2, y3 = sorg[3] + p3;
          if (y0 < v && y1 < v && y2 < v && y3 < v) y += T.vcoef * T.va[y0 * v + y1] * T.vb[y2 * v + y3];
        }
        acc2[e] += T.coef * y;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < QPER; ++e) {
    const int lin = threadIdx.x + e * QTPB;
    const int w0 = org[0] + (lin >> 9), w1 = org[1] + ((lin >> 6) & 7), w2 = org[2] + ((lin >> 3) & 7),
              w3 = org[3] + (lin & 7);
    if (w0 >= v || w1 >= v || w2 >= v || w3 >= v) continue;
    const long long off = w0 * v3 + w1 * v2 + w2 * v1 + w3;
    double x = acc[e];
    if (a.eps_v) x /= a.eps_occ - (a.eps_v[w0] + a.eps_v[w1] + a.eps_v[w2] + a.eps_v[w3]);
    out[off] = (a.beta == 0.0) ? x : x + a.beta * out[off];
    if (out2) out2[off] = (a.beta == 0.0) ? acc2[e] : acc2[e] + a.beta * out2[off];
  }
}

// C[m][n] += alpha * sum_k A[m*lda + k] * B[k*ldb + n] for a short K: a
// streaming read-modify-write of C.  Each thread owns two adjacent columns
// (16-byte loads and stores, consecutive threads on consecutive pairs) and
// keeps their K values of B in registers; the block walks RM rows, reading
// each row of A once (the same for every thread).
constexpr int RK_MAX = 16;
constexpr int RM = 16;

__global__ __launch_bounds__(256) void rank_k_update_kernel(double* __restrict__ C, long long ldc,
                                                            const double* __restrict__ A, long long lda,
                                                            const double* __restrict__ B, long long ldb, int M,
                                                            long long N, int K, double alpha) {
  const long long n = 2 * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
  const int m0 = blockIdx.y * RM;
  __shared__ double As[RM * RK_MAX];
  for (int i = threadIdx.x; i < RM * K; i += blockDim.x) {
    const int r = i / K, k = i - r * K;
    As[r * RK_MAX + k] = (m0 + r < M) ? A[(long long)(m0 + r) * lda + k] : 0.0;
  }
  __syncthreads();
  if (n >= N) return;
  double2 b[RK_MAX];
#pragma unroll
  for (int k = 0; k < RK_MAX; ++k)
    if (k < K) b[k] = *reinterpret_cast<const double2*>(B + (long long)k * ldb + n);
  const int mend = min(RM, M - m0);
  for (int r = 0; r < mend; ++r) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < RK_MAX; ++k)
      if (k < K) {
        const double a = As[r * RK_MAX + k];
        acc.x += a * b[k].x;
        acc.y += a * b[k].y;
      }
    double2* c = reinterpret_cast<double2*>(C + (long long)(m0 + r) * ldc + n);
    double2 cv = *c;
    cv.x += alpha * acc.x;
    cv.y += alpha * acc.y;
    *c = cv;
  }
}

__global__ __launch_bounds__(256) void rank_k_update_tiled_kernel(const double* __restrict__ C, double* __restrict__ D,
                                                                  int v, int rsplit, long long M, long long N,
                                                                  const double* __restrict__ A, long long lda,
                                                                  const double* __restrict__ B, long long ldb, int K,
                                                                  double alpha, int nt) {
  const long long n = 2 * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
  const long long m0 = (long long)blockIdx.y * RM;
  __shared__ double As[RM * RK_MAX];
  for (int i = threadIdx.x; i < RM * K; i += blockDim.x) {
    const int r = i / K, k = i - r * K;
    As[r * RK_MAX + k] = (m0 + r < M) ? A[(m0 + r) * lda + k] : 0.0;
  }
  __syncthreads();
  if (n >= N) return;
  double2 b[RK_MAX];
#pragma unroll
  for (int k = 0; k < RK_MAX; ++k)
    if (k < K) b[k] = *reinterpret_cast<const double2*>(B + (long long)k * ldb + n);
  // axes of column n: (c, d) when rows cover (a, b); (b, c, d) when rows cover a
  const int d = (int)(n % v);
  const int c = (int)((n / v) % v);
  const int bcol = rsplit == 1 ? (int)(n / ((long long)v * v)) : 0;
  const long long mend = min((long long)RM, M - m0);
  for (long long r = 0; r < mend; ++r) {
    const long long m = m0 + r;
    const int a = rsplit == 1 ? (int)m : (int)(m / v);
    const int bb = rsplit == 1 ? bcol : (int)(m % v);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < RK_MAX; ++k)
      if (k < K) {
        const double x = As[r * RK_MAX + k];
        acc.x += x * b[k].x;
        acc.y += x * b[k].y;
      }
    double2 cv = *reinterpret_cast<const double2*>(C + m * N + n);
    cv.x += alpha * acc.x;
    cv.y += alpha * acc.y;
    const long long ti = (((long long)(a >> 3) * nt + (bb >> 3)) * nt + (c >> 3)) * nt + (d >> 3);
    *reinterpret_cast<double2*>(D + ti * 4096 + (((a & 7) * 8 + (bb & 7)) * 8 + (c & 7)) * 8 + (d & 7)) = cv;
  }
}

}  // namespace

hipError_t perm_combine(double* out, double* out2, const QCombineArgs& a, hipStream_t s) {
  if (a.v <= 0) return hipSuccess;
  if (!out || a.nterms < 1 || a.nterms > QMAXT || out2 == out) return hipErrorInvalidValue;
  for (int t = 0; t < a.nterms; ++t) {
    const QPermTerm& T = a.t[t];
    if (!T.in || T.in == out || (out2 && T.in == out2)) return hipErrorInvalidValue;
    if (T.dst < 1 || T.dst > 3 || ((T.dst & 2) && !out2)) return hipErrorInvalidValue;
    if ((T.va == nullptr) != (T.vb == nullptr)) return hipErrorInvalidValue;
    int seen = 0;
    for (int k = 0; k < 4; ++k) {
      if (T.perm[k] < 0 || T.perm[k] > 3) return hipErrorInvalidValue;
      seen |= 1 << T.perm[k];
    }
    if (seen != 15) return hipErrorInvalidValue;
  }
  const int nt = (a.v + QT - 1) / QT;
  const long long ntiles = (long long)nt * nt * nt * nt;
  if (ntiles > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.tiled)
    hipLaunchKernelGGL(perm_combine_kernel<true>, dim3((unsigned)ntiles), dim3(QTPB), 0, s, out, out2, a, nt);
  else
    hipLaunchKernelGGL(perm_combine_kernel<false>, dim3((unsigned)ntiles), dim3(QTPB), 0, s, out, out2, a, nt);
  return hipGetLastError();
}

hipError_t rank_k_update(double* C, long long ldc, const double* A, long long lda, const double* B, long long ldb,
                         int M, long long N, int K, double alpha, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K > RK_MAX || (N & 1) || (ldc & 1) || (ldb & 1) || ((uintptr_t)C & 15) || ((uintptr_t)B & 15))
    return hipErrorInvalidValue;
  const long long nx = (N / 2 + 255) / 256;
  const long long ny = (M + RM - 1) / RM;
  if (nx > 0x7fffffffLL || ny > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rank_k_update_kernel, dim3((unsigned)nx, (unsigned)ny), dim3(256), 0, s, C, ldc, A, lda, B, ldb,
                     M, N, K, alpha);
  return hipGetLastError();
}

hipError_t rank_k_update_tiled(const double* C, double* D, int v, int rsplit, const double* A, long long lda,
                               const double* B, long long ldb, int K, double alpha, hipStream_t s) {
  if (v <= 0 || K <= 0) return hipSuccess;
  if ((v & 1) || K > RK_MAX || (rsplit != 1 && rsplit != 2) || (ldb & 1) || ((uintptr_t)C & 15) ||
      ((uintptr_t)B & 15) || ((uintptr_t)D & 15))
    return hipErrorInvalidValue;
  const long long v2 = (long long)v * v;
  const long long M = rsplit == 1 ? v : v2;
  const long long N = rsplit == 1 ? v2 * v : v2;
  const long long nx = (N / 2 + 255) / 256;
  const long long ny = (M + RM - 1) / RM;
  if (nx > 0x7fffffffLL || ny > 65535) return hipErrorInvalidValue;
  const int nt = (v + 7) / 8;
  hipLaunchKernelGGL(rank_k_update_tiled_kernel, dim3((unsigned)nx, (unsigned)ny), dim3(256), 0, s, C, D, v, rsplit, M,
                     N, A, lda, B, ldb, K, alpha, nt);
  return hipGetLastError();
}

}  // namespace cct
