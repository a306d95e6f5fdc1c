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
      const int y0 = sorg[0] + m0, y1 = sorg[1] + m1, y2 = sorg[2] + m2, y3 = sorg[3] + m3;
      double val = 0.0;
      if (y0 < v && y1 < v && y2 < v && y3 < v) val = T.in[y0 * v3 + y1 * v2 + y2 * v1 + y3];
      L[m0 * QS0 + m1 * QS1 + m2 * QS2 + m3] = val;
    }
    __syncthreads();
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
  hipLaunchKernelGGL(perm_combine_kernel, dim3((unsigned)ntiles), dim3(QTPB), 0, s, out, out2, a, nt);
  return hipGetLastError();
}

}  // namespace cct
