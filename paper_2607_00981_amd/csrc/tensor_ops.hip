// Bandwidth-bound kernels around the matrix-core contractions: strided
// permute/accumulate, T3 unpacking (the paper's on-the-fly reconstruction of
// off-triangle blocks from stored i<=j<=k blocks, with the spin-summed
// combinations applied in the same pass), output-stationary folding of
// contracted blocks into packed R3, the fused R3 post-processing / Jacobi
// update, and deterministic reductions.
#include "internal.h"

#include <algorithm>
#include <climits>

namespace cct {
namespace {

constexpr int TPB = 256;

inline unsigned blocks_for(long long n, int per_block, unsigned cap = 1u << 20) {
  long long b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

__device__ __forceinline__ void put_out(const OutSpec& o, long long i, double x) {
  if (o.fmt == OUT_F64) {
    ((double*)o.p)[i] = x;
  } else if (o.fmt == OUT_F32) {
    ((float*)o.p)[i] = (float)x;
  } else {
    const __bf16 hi = (__bf16)(float)x;
    const __bf16 lo = (__bf16)(float)(x - (double)(float)hi);
    const long long h = o.fmt == OUT_BF16X2I ? 2 * i - (i & 31) : i;
    ((__bf16*)o.p)[h] = hi;
    ((__bf16*)o.p)[o.fmt == OUT_BF16X2I ? h + 32 : o.plane + i] = lo;
  }
}

// ---------------------------------------------------------------------------
// permute / accumulate
// ---------------------------------------------------------------------------
__global__ void permute_add_kernel(const double* __restrict__ X, double* __restrict__ Y, PermArgs p, long long total) {
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    long long r = idx, ox = 0, oy = 0;
    for (int d = p.nd - 1; d >= 0; --d) {
      const long long c = r % p.dim[d];
      r /= p.dim[d];
      ox += c * p.sx[d];
      oy += c * p.sy[d];
    }
    const double x = p.alpha * X[ox];
    Y[oy] = (p.beta == 0.0) ? x : x + p.beta * Y[oy];
  }
}

// ---------------------------------------------------------------------------
// T3 unpacking
// ---------------------------------------------------------------------------
// grid.y enumerates (slot, free indices); grid.x enumerates tiles of the v^3 virtual block.
// LDS-staged unpack.  One workgroup builds one UT x UT x UT tile of one
// output block.  Each term is gathered with the threads running along the
// axis that is unit-stride in that term's stored block (coalesced 128-byte
// row segments whatever the virtual permutation) and accumulated into the
// LDS tile; the tile is then written with the threads running along the
// output's unit-stride axis.
constexpr int UT = 16;
constexpr int UP_Z = UT + 1;            // pitch of y rows in the LDS tile
constexpr int UP_X = UT * UP_Z + 1;     // pitch of x planes

// Tile of this workgroup.  Workgroups go to the eight XCDs in turn, so tile
// k * per + i runs on XCD k: each XCD takes a contiguous range of tiles, and
// neighbouring tiles, which share the 128-byte lines that a row of v values
// leaves partly used when v is not a multiple of 16, meet in one L2 instead
// of fetching (and writing) the same lines from two.  The grid's x extent is
// 8 per; workgroups past the last tile return at once.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = (ntiles + 7) / 8;
  return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}
inline unsigned xcd_grid(int ntiles) { return (unsigned)(((ntiles + 7) / 8) * 8); }

template <bool DUAL>
__global__ __launch_bounds__(256) void unpack_tiled_kernel(const double* __restrict__ T,
                                                           const BlockRef* __restrict__ tbl,
                                                           const int2* __restrict__ slots, OutSpec out,
                                                           OutSpec out2, UnpackArgs a, int nt) {
  __shared__ double L[UT * UP_X];
  const int o = a.o, v = a.v;
  const int nfc = (a.nfree == 2) ? o * o : o;
  const int sy_ = blockIdx.y;
  const int slot = sy_ / nfc;
  const int fc = sy_ - slot * nfc;
  const int f0 = (a.nfree == 2) ? fc / o : fc;
  const int f1 = (a.nfree == 2) ? fc - f0 * o : 0;
  const int2 fx = slots[slot];
  const int ids[4] = {fx.x, fx.y, f0, f1};
  const int tile = xcd_tile(nt * nt * nt);
  if (tile >= nt * nt * nt) return;
  const int t2 = tile % nt, t1 = (tile / nt) % nt, t0 = tile / (nt * nt);
  // the fastest tile digit runs along the output's unit-stride axis
  const int wf = a.fast == 0 ? 2 : (a.fast == 1 ? 1 : 0);
  int tb[3];
  tb[wf] = t2;
  tb[(wf + 1) % 3] = t1;
  tb[(wf + 2) % 3] = t0;
  const int base[3] = {tb[0] * UT, tb[1] * UT, tb[2] * UT};  // x, y, z origins
  const long long obase = (long long)slot * a.s_slot + (long long)f0 * a.s_free[0] + (long long)f1 * a.s_free[1];
  for (int t = 0; t < a.nterms; ++t) {
    const UnpackTerm& tm = a.terms[t];
    const int p = ids[tm.occ[0]], q = ids[tm.occ[1]], r = ids[tm.occ[2]];
    const BlockRef br = tbl[((long long)p * o + q) * o + r];
    // output axis read by the unit-stride stored axis
    int u = 2;
#pragma unroll
    for (int m = 0; m < 3; ++m)
      if (br.s[m] == 1) u = tm.virt[m];
    const int ua = (u + 1) % 3, ub = (u + 2) % 3;
    // stride of each output axis in the stored block
    long long st[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) st[tm.virt[m]] = br.s[m];
    // all loads of this thread first (independent, in flight together), then the LDS updates
    constexpr int PER = UT * UT * UT / 256;
    double vals[PER];
    int lds[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * 256;
      int c[3];
      c[u] = e % UT;
      c[ua] = (e / UT) % UT;
      c[ub] = e / (UT * UT);
      const int x = base[0] + c[0], y = base[1] + c[1], z = base[2] + c[2];
      const bool ok = x < v && y < v && z < v;
      lds[it] = ok ? c[0] * UP_X + c[1] * UP_Z + c[2] : -1;
      vals[it] = ok ? T[br.off + x * st[0] + y * st[1] + z * st[2]] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      if (lds[it] < 0) continue;
      const double val = tm.coef * vals[it];
      L[lds[it]] = (t == 0) ? val : L[lds[it]] + val;
    }
    __syncthreads();
  }
  // write the tile along the output's unit-stride axis (fast: 0 = z, 1 = y, 2 = x)
  {
    const int w = a.fast == 0 ? 2 : (a.fast == 1 ? 1 : 0);
    const int wa = (w + 1) % 3, wb = (w + 2) % 3;
    const long long so[3] = {a.s_x, a.s_y, a.s_z};
    for (int e = threadIdx.x; e < UT * UT * UT; e += blockDim.x) {
      int c[3];
      c[w] = e % UT;
      c[wa] = (e / UT) % UT;
      c[wb] = e / (UT * UT);
      const int x = base[0] + c[0], y = base[1] + c[1], z = base[2] + c[2];
      if (x >= v || y >= v || z >= v) continue;
      put_out(out, obase + x * so[0] + y * so[1] + z * so[2], L[c[0] * UP_X + c[1] * UP_Z + c[2]]);
    }
  }
  if constexpr (DUAL) {
    const long long obase2 =
        (long long)slot * a.s2_slot + (long long)f0 * a.s2_free[0] + (long long)f1 * a.s2_free[1];
    const int w = a.fast2 == 0 ? 2 : (a.fast2 == 1 ? 1 : 0);
    const int wa = (w + 1) % 3, wb = (w + 2) % 3;
    const long long so[3] = {a.s2_x, a.s2_y, a.s2_z};
    for (int e = threadIdx.x; e < UT * UT * UT; e += blockDim.x) {
      int c[3];
      c[w] = e % UT;
      c[wa] = (e / UT) % UT;
      c[wb] = e / (UT * UT);
      const int x = base[0] + c[0], y = base[1] + c[1], z = base[2] + c[2];
      if (x >= v || y >= v || z >= v) continue;
      put_out(out2, obase2 + x * so[0] + y * so[1] + z * so[2], L[c[0] * UP_X + c[1] * UP_Z + c[2]]);
    }
  }
}

// ---------------------------------------------------------------------------
// fold temporary blocks into packed R3 (one output block per task)
// ---------------------------------------------------------------------------
// One workgroup per UT^3 tile of one output block: the R tile is staged in
// LDS, each contribution is added with the threads running along the axis
// that is unit-stride in Z for that contribution (coalesced reads for any
// virtual permutation), and the tile is written back along c.
template <typename ZT>
__global__ __launch_bounds__(256) void fold_tiled_kernel(double* __restrict__ R, long long bs, int v,
                                                         const ZT* __restrict__ Z,
                                                         const FoldTask* __restrict__ tasks,
                                                         const FoldContrib* __restrict__ contribs, int nt) {
  __shared__ double L[UT * UP_X];
  constexpr int PER = UT * UT * UT / 256;
  const FoldTask tk = tasks[blockIdx.y];
  const long long v2 = (long long)v * v;
  double* Rt = R + (long long)tk.t * bs;
  const int tile = xcd_tile(nt * nt * nt);
  if (tile >= nt * nt * nt) return;
  const int t2 = tile % nt, t1 = (tile / nt) % nt, t0 = tile / (nt * nt);
  const int base[3] = {t0 * UT, t1 * UT, t2 * UT};  // a, b, c origins
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int e = threadIdx.x + it * 256;
    const int c2 = e % UT, c1 = (e / UT) % UT, c0 = e / (UT * UT);
    const int a = base[0] + c0, b = base[1] + c1, c = base[2] + c2;
    if (a < v && b < v && c < v) L[c0 * UP_X + c1 * UP_Z + c2] = Rt[a * v2 + (long long)b * v + c];
  }
  __syncthreads();
  for (int i = 0; i < tk.nc; ++i) {
    const FoldContrib fc = contribs[tk.c0 + i];
    const long long st[3] = {fc.sa, fc.sb, fc.sc};
    const int u = fc.sa == 1 ? 0 : (fc.sb == 1 ? 1 : 2);
    const int ua = (u + 1) % 3, ub = (u + 2) % 3;
    double vals[PER];
    int lds[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int e = threadIdx.x + it * 256;
      int cc[3];
      cc[u] = e % UT;
      cc[ua] = (e / UT) % UT;
      cc[ub] = e / (UT * UT);
      const int a = base[0] + cc[0], b = base[1] + cc[1], c = base[2] + cc[2];
      const bool ok = a < v && b < v && c < v;
      lds[it] = ok ? cc[0] * UP_X + cc[1] * UP_Z + cc[2] : -1;
      vals[it] = ok ? (double)Z[fc.base + a * st[0] + b * st[1] + c * st[2]] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < PER; ++it)
      if (lds[it] >= 0) L[lds[it]] += fc.coef * vals[it];
    __syncthreads();
  }
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int e = threadIdx.x + it * 256;
    const int c2 = e % UT, c1 = (e / UT) % UT, c0 = e / (UT * UT);
    const int a = base[0] + c0, b = base[1] + c1, c = base[2] + c2;
    if (a < v && b < v && c < v) Rt[a * v2 + (long long)b * v + c] = L[c0 * UP_X + c1 * UP_Z + c2];
  }
}

// ---------------------------------------------------------------------------
// R3 post-processing + norm + Jacobi update.  The virtual block is cut into
// PT^3 tiles; a workgroup takes an orbit of tiles {(A,B,C) and its
// permutations}, A <= B <= C, stages those (at most six) R tiles in LDS with
// row-contiguous loads, post-processes every element orbit
// {(a,b,c) and its permutations} inside LDS, and writes R back and updates T
// with row-contiguous accesses.  Each element is read and written once.
// ---------------------------------------------------------------------------
constexpr int PT = 8;
constexpr int PT3 = PT * PT * PT;

__device__ __forceinline__ void decode_tile_orbit(int idx, int nt, int& A, int& B, int& C) {
  A = 0;
  while (true) {
    const int cnt = (nt - A) * (nt - A + 1) / 2;
    if (idx < cnt) break;
    idx -= cnt;
    ++A;
  }
  B = A;
  while (idx >= nt - B) {
    idx -= nt - B;
    ++B;
  }
  C = B + idx;
}

__global__ __launch_bounds__(256) void post_update_kernel(double* __restrict__ R, double* __restrict__ T,
                                                          const int4* __restrict__ tri,
                                                          const double* __restrict__ eps,
                                                          double* __restrict__ partial, PostArgs pa, int nt,
                                                          int norbit) {
  __shared__ double L[6 * PT3];
  __shared__ double red[TPB];
  const int t = blockIdx.y;
  const int4 ijk = tri[t];
  const int o = pa.o, v = pa.v;
  const long long v2 = (long long)v * v;
  double* Rt = R + (long long)t * pa.bs;
  double* Tt = T + (long long)t * pa.bs;
  const bool ij = (ijk.x == ijk.y), jk = (ijk.y == ijk.z);
  const double eocc = eps[ijk.x] + eps[ijk.y] + eps[ijk.z];
  // placements p of (x,y,z): 0:(x,y,z) 1:(x,z,y) 2:(y,x,z) 3:(y,z,x) 4:(z,x,y) 5:(z,y,x)
  const int sw12[6] = {2, 4, 0, 5, 1, 3};
  const int sw23[6] = {1, 0, 3, 2, 5, 4};
  double nrm = 0.0;
  for (int orb = blockIdx.x; orb < norbit; orb += gridDim.x) {
    int A, B, C;
    decode_tile_orbit(orb, nt, A, B, C);
    const int TP[6][3] = {{A, B, C}, {A, C, B}, {B, A, C}, {B, C, A}, {C, A, B}, {C, B, A}};
    int slot[6];
    int nslot = 0;
    int slot_tile[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      slot[p] = -1;
      for (int q = 0; q < p; ++q)
        if (TP[q][0] == TP[p][0] && TP[q][1] == TP[p][1] && TP[q][2] == TP[p][2]) { slot[p] = slot[q]; break; }
      if (slot[p] < 0) { slot[p] = nslot; slot_tile[nslot] = p; ++nslot; }
    }
    // stage the distinct R tiles (rows of PT contiguous elements)
    for (int sl = 0; sl < nslot; ++sl) {
      const int* tp = TP[slot_tile[sl]];
      for (int e = threadIdx.x; e < PT3; e += blockDim.x) {
        const int x = tp[0] * PT + e / (PT * PT), y = tp[1] * PT + (e / PT) % PT, z = tp[2] * PT + e % PT;
        if (x < v && y < v && z < v) L[sl * PT3 + e] = Rt[x * v2 + (long long)y * v + z];
      }
    }
    __syncthreads();
    // element orbits with a representative in tile (A,B,C)
    for (int e = threadIdx.x; e < PT3; e += blockDim.x) {
      const int a = A * PT + e / (PT * PT), b = B * PT + (e / PT) % PT, c = C * PT + e % PT;
      if (a >= v || b >= v || c >= v) continue;
      if ((A == B && a > b) || (B == C && b > c)) continue;
      const int P[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
      int li[6];
      double r[6];
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        const int* tp = TP[p];
        li[p] = slot[p] * PT3 + (P[p][0] - tp[0] * PT) * PT * PT + (P[p][1] - tp[1] * PT) * PT + (P[p][2] - tp[2] * PT);
        r[p] = L[li[p]];
      }
      double sv[6];
      if (ij && jk) {
#pragma unroll
        for (int p = 0; p < 6; ++p) sv[p] = 0.0;
      } else if (ij) {
#pragma unroll
        for (int p = 0; p < 6; ++p) sv[p] = 0.5 * (r[p] + r[sw12[p]]);
      } else if (jk) {
#pragma unroll
        for (int p = 0; p < 6; ++p) sv[p] = 0.5 * (r[p] + r[sw23[p]]);
      } else {
#pragma unroll
        for (int p = 0; p < 6; ++p) sv[p] = r[p];
      }
      const double mean = (sv[0] + sv[1] + sv[2] + sv[3] + sv[4] + sv[5]) * (1.0 / 6.0);
#pragma unroll
      for (int p = 0; p < 6; ++p) {
        bool dup = false;
#pragma unroll
        for (int q = 0; q < p; ++q) dup = dup || (li[q] == li[p]);
        if (dup) continue;
        const double x = sv[p] - mean;
        nrm += x * x;
        L[li[p]] = x;
      }
    }
    __syncthreads();
    // write R, update T (rows of PT contiguous elements)
    for (int sl = 0; sl < nslot; ++sl) {
      const int* tp = TP[slot_tile[sl]];
      for (int e = threadIdx.x; e < PT3; e += blockDim.x) {
        const int x = tp[0] * PT + e / (PT * PT), y = tp[1] * PT + (e / PT) % PT, z = tp[2] * PT + e % PT;
        if (x >= v || y >= v || z >= v) continue;
        const long long off = x * v2 + (long long)y * v + z;
        const double val = L[sl * PT3 + e];
        if (pa.keep_r) Rt[off] = val;
        if (pa.do_update) Tt[off] += val / (eocc - eps[o + x] - eps[o + y] - eps[o + z]);
      }
    }
    __syncthreads();
  }
  red[threadIdx.x] = nrm * (double)ijk.w;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// reductions (fixed grid, fixed order: bitwise reproducible)
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 512;

__device__ __forceinline__ double block_sum(double x, double* red) {
  red[threadIdx.x] = x;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

__global__ void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y, long long n,
                                   double* __restrict__ part) {
  __shared__ double red[TPB];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < n; i += (long long)gridDim.x * TPB)
    acc += x[i] * (y ? y[i] : 1.0);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void sum_kernel(const double* __restrict__ part, long long n, double* __restrict__ out) {
  __shared__ double red[TPB];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += TPB) acc += part[i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[0] = s;
}

__global__ void dot_t3_partial_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                      const int4* __restrict__ tri, long long bs, long long v3, double* __restrict__ part) {
  __shared__ double red[TPB];
  const int t = blockIdx.y;
  const double* xt = x + (long long)t * bs;
  const double* yt = y + (long long)t * bs;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < v3; i += (long long)gridDim.x * TPB)
    acc += xt[i] * yt[i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[(long long)t * gridDim.x + blockIdx.x] = s * (double)tri[t].w;
}

__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, double* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}

__global__ void fill_kernel(double* __restrict__ y, double val, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = val;
}

// 32 x 32 tiles through LDS: reads and writes both coalesced.
__global__ void transpose_kernel(const double* __restrict__ in, OutSpec out, long long b0, int R, int C) {
  __shared__ double tile[32][33];
  const long long b = blockIdx.z + b0;
  const double* src = in + b * (long long)R * C;
  const long long dbase = b * (long long)R * C;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < R && c < C) tile[k][tx] = src[(long long)r * C + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < R && c < C) put_out(out, dbase + (long long)c * R + r, tile[tx][k]);
  }
}

__global__ void swap01_kernel(const double* __restrict__ in, OutSpec out, long long rows, int n0, int n1, int n2) {
  // one (b, i, j) row of n2 elements per (y, z) block index
  const long long row = blockIdx.y + (long long)blockIdx.z * 65535;
  if (row >= rows) return;
  const long long per = (long long)n0 * n1;
  const long long b = row / per;
  const int ij = (int)(row - b * per);
  const int i = ij / n1, j = ij - i * n1;  // out[b][i][j][:] = in[b][j][i][:]
  const double* src = in + ((b * n1 + j) * n0 + i) * (long long)n2;
  const long long dst = ((b * n0 + i) * n1 + j) * (long long)n2;
  for (int k = threadIdx.x; k < n2; k += blockDim.x) put_out(out, dst + k, src[k]);
}

__global__ void convert_kernel(const double* __restrict__ in, OutSpec out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    put_out(out, i, in[i]);
}

__global__ void add_rows_kernel(const double* __restrict__ in, int rows, long long n, double* __restrict__ out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double acc = out[i];
    for (int r = 0; r < rows; ++r) acc += in[(long long)r * n + i];
    out[i] = acc;
  }
}

__global__ void jacobi_kernel(double* __restrict__ t1, const double* __restrict__ r1, double* __restrict__ t2,
                              const double* __restrict__ r2, const double* __restrict__ eps, int o, int v) {
  const long long n1 = (long long)o * v, n2 = n1 * n1;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n1 + n2;
       idx += (long long)gridDim.x * blockDim.x) {
    if (idx < n1) {
      const int i = (int)(idx / v), a = (int)(idx % v);
      t1[idx] += r1[idx] / (eps[i] - eps[o + a]);
    } else {
      const long long k = idx - n1;
      const int b = (int)(k % v);
      const int a = (int)((k / v) % v);
      const int j = (int)((k / ((long long)v * v)) % o);
      const int i = (int)(k / ((long long)v * v * o));
      t2[k] += r2[k] / (eps[i] + eps[j] - eps[o + a] - eps[o + b]);
    }
  }
}

// W[x][y][x'][y'] += c F[x][x'] (y == y')   (pass 0)   or   += c F[y][y'] (x == x')   (pass 1)
__global__ void pair_diag_kernel(double* __restrict__ W, const double* __restrict__ F, long long ldF, int nx, double c,
                                 int pass) {
  const long long n3 = (long long)nx * nx * nx;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n3;
       idx += (long long)gridDim.x * blockDim.x) {
    const int u = (int)(idx / ((long long)nx * nx));
    const int w = (int)((idx / nx) % nx);
    const int d = (int)(idx % nx);
    const long long nx2 = (long long)nx * nx;
    if (pass == 0) {
      // x = u, x' = w, y = y' = d
      W[((long long)u * nx + d) * nx2 + (long long)w * nx + d] += c * F[(long long)u * ldF + w];
    } else {
      // y = u, y' = w, x = x' = d
      W[((long long)d * nx + u) * nx2 + (long long)d * nx + w] += c * F[(long long)u * ldF + w];
    }
  }
}

}  // namespace

hipError_t permute_add(const double* X, double* Y, const PermArgs& p, hipStream_t s) {
  long long total = 1;
  for (int d = 0; d < p.nd; ++d) total *= p.dim[d];
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(permute_add_kernel, dim3(blocks_for(total, TPB * 4)), dim3(TPB), 0, s, X, Y, p, total);
  return hipGetLastError();
}

hipError_t unpack_t3_fmt(const double* T, const BlockRef* tbl, const int2* slots, OutSpec out, const UnpackArgs& a,
                         hipStream_t s) {
  const long long v3 = (long long)a.v * a.v * a.v;
  const long long ny = (long long)a.nslots * (a.nfree == 2 ? (long long)a.o * a.o : a.o);
  if (ny <= 0 || v3 <= 0) return hipSuccess;
  if (ny > 65535) return hipErrorInvalidValue;
  if (a.nterms < 1 || a.nterms > 6) return hipErrorInvalidValue;
  const int nt = (a.v + UT - 1) / UT;
  dim3 grid(xcd_grid(nt * nt * nt), (unsigned)ny);
  hipLaunchKernelGGL(unpack_tiled_kernel<false>, grid, dim3(TPB), 0, s, T, tbl, slots, out, out, a, nt);
  return hipGetLastError();
}

hipError_t unpack_t3_dual(const double* T, const BlockRef* tbl, const int2* slots, OutSpec out, OutSpec out2,
                          const UnpackArgs& a, hipStream_t s) {
  const long long v3 = (long long)a.v * a.v * a.v;
  const long long ny = (long long)a.nslots * (a.nfree == 2 ? (long long)a.o * a.o : a.o);
  if (ny <= 0 || v3 <= 0) return hipSuccess;
  if (ny > 65535) return hipErrorInvalidValue;
  if (a.nterms < 1 || a.nterms > 6) return hipErrorInvalidValue;
  const int nt = (a.v + UT - 1) / UT;
  dim3 grid(xcd_grid(nt * nt * nt), (unsigned)ny);
  hipLaunchKernelGGL(unpack_tiled_kernel<true>, grid, dim3(TPB), 0, s, T, tbl, slots, out, out2, a, nt);
  return hipGetLastError();
}

hipError_t unpack_t3(const double* T, const BlockRef* tbl, const int2* slots, double* out, const UnpackArgs& a,
                     hipStream_t s) {
  return unpack_t3_fmt(T, tbl, slots, OutSpec{out, OUT_F64, 0}, a, s);
}

hipError_t fold_r3(double* R, long long bs, int v, const double* Z, const FoldTask* tasks, int ntasks,
                   const FoldContrib* contribs, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (ntasks > 65535) return hipErrorInvalidValue;
  const int nt = (v + UT - 1) / UT;
  dim3 grid(xcd_grid(nt * nt * nt), (unsigned)ntasks);
  hipLaunchKernelGGL(fold_tiled_kernel<double>, grid, dim3(TPB), 0, s, R, bs, v, Z, tasks, contribs, nt);
  return hipGetLastError();
}

hipError_t fold_r3(double* R, long long bs, int v, const float* Z, const FoldTask* tasks, int ntasks,
                   const FoldContrib* contribs, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  if (ntasks > 65535) return hipErrorInvalidValue;
  const int nt = (v + UT - 1) / UT;
  dim3 grid(xcd_grid(nt * nt * nt), (unsigned)ntasks);
  hipLaunchKernelGGL(fold_tiled_kernel<float>, grid, dim3(TPB), 0, s, R, bs, v, Z, tasks, contribs, nt);
  return hipGetLastError();
}

hipError_t post_update(double* R, double* T, const int4* tri, const double* eps, double* partial, int* npartial,
                       const PostArgs& a, hipStream_t s) {
  if (a.ntri > 65535) return hipErrorInvalidValue;
  const int nt = (a.v + PT - 1) / PT;
  const int norbit = nt * (nt + 1) * (nt + 2) / 6;
  const unsigned gx = (unsigned)std::min(norbit, 64);
  dim3 grid(gx, (unsigned)a.ntri);
  hipLaunchKernelGGL(post_update_kernel, grid, dim3(TPB), 0, s, R, T, tri, eps, partial, a, nt, norbit);
  *npartial = (int)(gx * a.ntri);
  return hipGetLastError();
}

hipError_t reduce_sum(const double* x, long long n, double* out, double* scratch, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(RED_BLOCKS), dim3(TPB), 0, s, x, (const double*)nullptr, n, scratch);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(TPB), 0, s, (const double*)scratch, (long long)RED_BLOCKS, out);
  return hipGetLastError();
}

hipError_t dot(const double* x, const double* y, long long n, double* out, double* scratch, hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(RED_BLOCKS), dim3(TPB), 0, s, x, y, n, scratch);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(TPB), 0, s, (const double*)scratch, (long long)RED_BLOCKS, out);
  return hipGetLastError();
}

hipError_t weighted_dot_t3(const double* x, const double* y, const int4* tri, int ntri, long long bs, long long v3,
                           double* out, double* scratch, hipStream_t s) {
  const unsigned gx = blocks_for(v3, TPB * 16, 16);
  if (ntri > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dot_t3_partial_kernel, dim3(gx, (unsigned)ntri), dim3(TPB), 0, s, x, y, tri, bs, v3, scratch);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(TPB), 0, s, (const double*)scratch, (long long)gx * ntri, out);
  return hipGetLastError();
}

namespace {
__global__ void t3_subcube_kernel(double* __restrict__ T, double* __restrict__ sub, int v, int sv, long long total,
                                  bool gather) {
  const long long s3 = (long long)sv * sv * sv, v2 = (long long)v * v, v3 = v2 * v;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long t = i / s3;
    const long long r = i - t * s3;
    const int a = (int)(r / ((long long)sv * sv)), b = (int)((r / sv) % sv), c = (int)(r % sv);
    const long long off = t * v3 + a * v2 + (long long)b * v + c;
    if (gather) sub[i] = T[off];
    else T[off] = sub[i];
  }
}
}  // namespace

namespace {
__global__ void copy_pad_rows_kernel(const double* __restrict__ in, long long rows, long long cols, OutSpec out,
                                     long long ld, long long total) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / ld, c = i - r * ld;
    put_out(out, i, c < cols ? in[r * cols + c] : 0.0);
  }
}
__global__ void zero_cols_kernel(OutSpec out, long long ld, long long c0, long long total) {
  const long long w = ld - c0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long r = i / w;
    put_out(out, r * ld + c0 + (i - r * w), 0.0);
  }
}
}  // namespace

hipError_t copy_pad_rows(const double* in, long long rows, long long cols, OutSpec out, long long ld_out,
                         hipStream_t s) {
  const long long total = rows * ld_out;
  if (total <= 0) return hipSuccess;
  if (ld_out < cols) return hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_pad_rows_kernel, dim3(blocks_for(total, TPB * 4)), dim3(TPB), 0, s, in, rows, cols, out,
                     ld_out, total);
  return hipGetLastError();
}

hipError_t zero_cols(OutSpec out, long long rows, long long ld, long long c0, hipStream_t s) {
  const long long total = rows * (ld - c0);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_cols_kernel, dim3(blocks_for(total, TPB * 4)), dim3(TPB), 0, s, out, ld, c0, total);
  return hipGetLastError();
}

hipError_t t3_subcube(double* T, double* sub, long long ntri, int v, int sv, bool gather, hipStream_t s) {
  const long long total = ntri * (long long)sv * sv * sv;
  if (total <= 0) return hipSuccess;
  if (sv > v) return hipErrorInvalidValue;
  hipLaunchKernelGGL(t3_subcube_kernel, dim3(blocks_for(total, TPB * 4)), dim3(TPB), 0, s, T, sub, v, sv, total,
                     gather);
  return hipGetLastError();
}

hipError_t axpby(double a, const double* x, double b, double* y, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n, TPB * 4)), dim3(TPB), 0, s, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t fill(double* y, double val, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n, TPB * 4)), dim3(TPB), 0, s, y, val, n);
  return hipGetLastError();
}

hipError_t transpose_batched(const double* in, OutSpec out, long long batch, int R, int C, hipStream_t s) {
  if (batch <= 0 || R <= 0 || C <= 0) return hipSuccess;
  if ((R + 31) / 32 > 65535) return hipErrorInvalidValue;
  for (long long b0 = 0; b0 < batch; b0 += 65535) {
    const long long nb = batch - b0 < 65535 ? batch - b0 : 65535;
    dim3 grid((C + 31) / 32, (R + 31) / 32, (unsigned)nb);
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, in, out, b0, R, C);
  }
  return hipGetLastError();
}

hipError_t swap01_batched(const double* in, OutSpec out, long long batch, int n0, int n1, int n2, hipStream_t s) {
  const long long rows = batch * n0 * n1;
  if (rows <= 0 || n2 <= 0) return hipSuccess;
  const long long gz = (rows + 65534) / 65535;
  if (gz > 65535) return hipErrorInvalidValue;
  const unsigned gy = (unsigned)(rows < 65535 ? rows : 65535);
  hipLaunchKernelGGL(swap01_kernel, dim3(1, gy, (unsigned)gz), dim3(256), 0, s, in, out, rows, n0, n1, n2);
  return hipGetLastError();
}

hipError_t convert(const double* in, OutSpec out, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_kernel, dim3(blocks_for(n, TPB * 4)), dim3(TPB), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t add_rows(const double* in, int rows, long long n, double* out, hipStream_t s) {
  if (n <= 0 || rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_rows_kernel, dim3(blocks_for(n, TPB)), dim3(TPB), 0, s, in, rows, n, out);
  return hipGetLastError();
}

hipError_t jacobi_t1t2(double* t1, const double* r1, double* t2, const double* r2, const double* eps, int o, int v,
                       hipStream_t s) {
  const long long n = (long long)o * v + (long long)o * o * v * v;
  hipLaunchKernelGGL(jacobi_kernel, dim3(blocks_for(n, TPB * 4)), dim3(TPB), 0, s, t1, r1, t2, r2, eps, o, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Symmetric / antisymmetric pair split of the ladder operands and the
// rebuild of both output orders (the split ladder of r3_pp_split)
// ---------------------------------------------------------------------------
namespace {

constexpr int PS = 32;  // tile edge of the pair kernels

__device__ __forceinline__ long long imap(const Idx2& d, long long i) {
  if (d.inner == 0) return i * d.s_lo;
  const long long hi = i / d.inner;
  return hi * d.s_hi + (i - hi * d.inner) * d.s_lo;
}

__device__ __forceinline__ long long pidx(int d, int e, int v) {  // d <= e
  return (long long)d * v - (long long)d * (d - 1) / 2 + (e - d);
}
__device__ __forceinline__ long long qidx(int d, int e, int v) {  // d < e
  return (long long)d * (v - 1) - (long long)d * (d - 1) / 2 + (e - d - 1);
}
// Row and tile pair of this workgroup.  The grid's x extent is rows x P with
// P = 8 ceil(npair / 8) workgroups per row; workgroups go to the eight XCDs
// in turn, and the tile pairs of a row are dealt to them in contiguous
// ranges (pair k per + i on XCD k), so tiles next to each other in a row,
// which share the 128-byte lines that rows of v values leave partly used,
// run on one XCD at about the same time.  tp < 0: no tile.
__device__ __forceinline__ long long pair_row_tile(int nt, int& tp) {
  const int npair = nt * (nt + 1) / 2, per = (npair + 7) / 8, P = 8 * per;
  const long long r = blockIdx.x / P;
  const int t = (int)(blockIdx.x - r * P);
  tp = (t % 8) * per + t / 8;
  if (tp >= npair) tp = -1;
  return r;
}
__device__ __forceinline__ void tile_pair(int idx, int nt, int& Dt, int& Et) {  // Dt <= Et
  Dt = 0;
  while (idx >= nt - Dt) {
    idx -= nt - Dt;
    ++Dt;
  }
  Et = Dt + idx;
}

__global__ __launch_bounds__(256) void pair_split_kernel(const double* __restrict__ in, Idx2 rmap,
                                                         const long long* __restrict__ src, long long sd, int v,
                                                         OutSpec plus, long long pitch_p, OutSpec minus,
                                                         long long pitch_m, double diag_scale, int nt) {
  __shared__ double T1[PS][PS + 1], T2[PS][PS + 1];
  int tp;
  const long long r = pair_row_tile(nt, tp);
  if (tp < 0) return;
  const double* M = in + (src ? src[r] : imap(rmap, r));
  int Dt, Et;
  tile_pair(tp, nt, Dt, Et);
  for (int e = threadIdx.x; e < PS * PS; e += blockDim.x) {
    const int i = e / PS, j = e % PS;
    const int d1 = Dt * PS + i, e1 = Et * PS + j;
    if (d1 < v && e1 < v) T1[i][j] = M[d1 * sd + e1];
    const int d2 = Et * PS + i, e2 = Dt * PS + j;
    if (d2 < v && e2 < v) T2[i][j] = M[d2 * sd + e2];
  }
  __syncthreads();
  const long long P = (long long)v * (v + 1) / 2, Q = (long long)v * (v - 1) / 2;
  for (int e = threadIdx.x; e < PS * PS; e += blockDim.x) {
    const int i = e / PS, j = e % PS;
    const int d = Dt * PS + i, f = Et * PS + j;
    if (d >= v || f >= v || d > f) continue;
    const double a = T1[i][j], b = T2[j][i];  // M[d][f], M[f][d]
    put_out(plus, r * pitch_p + pidx(d, f, v), d == f ? diag_scale * (a + b) : a + b);
    if (d < f) put_out(minus, r * pitch_m + qidx(d, f, v), a - b);
  }
  // zero the padding columns of this row once
  if (tp == 0) {
    for (long long c = P + threadIdx.x; c < pitch_p; c += blockDim.x) put_out(plus, r * pitch_p + c, 0.0);
    for (long long c = Q + threadIdx.x; c < pitch_m; c += blockDim.x) put_out(minus, r * pitch_m + c, 0.0);
  }
}

// Rows form: C+[r][p], C-[r][q] -> R[cmap(r) + y*sy + z*sz] += C^{yz}
template <typename CT>
__global__ __launch_bounds__(256) void pair_combine_rows_kernel(const CT* __restrict__ Cp,
                                                                const CT* __restrict__ Cm, long long pitch_p,
                                                                long long pitch_m, int v, double* __restrict__ R,
                                                                Idx2 cmap, long long sy, long long sz, int nt) {
  __shared__ double U[PS][PS + 1];
  int tp;
  const long long r = pair_row_tile(nt, tp);
  if (tp < 0) return;
  double* Rr = R + imap(cmap, r);
  const CT* cp = Cp + r * pitch_p;
  const CT* cq = Cm + r * pitch_m;
  int Yt, Zt;
  tile_pair(tp, nt, Yt, Zt);
  for (int e = threadIdx.x; e < PS * PS; e += blockDim.x) {
    const int i = e / PS, j = e % PS;
    const int y = Yt * PS + i, z = Zt * PS + j;
    if (y >= v || z >= v || y > z) continue;
    const double p = (double)cp[pidx(y, z, v)];
    if (y == z) {
      Rr[y * sy + z * sz] += 0.5 * p;
    } else {
      const double m = (double)cq[pidx(y, z, v)];
      Rr[y * sy + z * sz] += 0.5 * (p + m);
      U[j][i] = 0.5 * (p - m);  // C^{zy}
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < PS * PS; e += blockDim.x) {
    const int i = e / PS, j = e % PS;  // row z = Zt*PS + i, column y = Yt*PS + j
    const int z = Zt * PS + i, y = Yt * PS + j;
    if (y >= v || z >= v || y >= z) continue;
    Rr[z * sy + y * sz] += U[i][j];
  }
}

// Columns form: C+T[p][c], C-T[q][c] (c = column, contiguous) ->
// R[ccol(c) + y*sy + z*sz] and R[ccol(c) + z*sy + y*sz]
template <typename CT>
__global__ __launch_bounds__(256) void pair_combine_cols_kernel(const CT* __restrict__ CpT,
                                                                const CT* __restrict__ CmT, long long ncol,
                                                                const int2* __restrict__ yz, int v,
                                                                double* __restrict__ R, Idx2 ccol, long long sy,
                                                                long long sz) {
  const long long p = blockIdx.x;
  const int2 t = yz[p];
  const int y = t.x, z = t.y;
  for (long long c = (long long)blockIdx.y * blockDim.x + threadIdx.x; c < ncol; c += (long long)gridDim.y * blockDim.x) {
    const double cp = (double)CpT[p * ncol + c];
    double* base = R + imap(ccol, c);
    if (y == z) {
      base[y * sy + z * sz] += 0.5 * cp;
    } else {
      const double cm = (double)CmT[p * ncol + c];
      base[y * sy + z * sz] += 0.5 * (cp + cm);
      base[z * sy + y * sz] += 0.5 * (cp - cm);
    }
  }
}

}  // namespace

hipError_t pair_split(const double* in, Idx2 rmap, const long long* src, long long rows, long long sd, int v,
                      OutSpec plus, long long pitch_p, OutSpec minus, long long pitch_m, double diag_scale,
                      hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int nt = (v + PS - 1) / PS;
  const long long P = 8LL * ((nt * (nt + 1) / 2 + 7) / 8);
  if (rows * P > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pair_split_kernel, dim3((unsigned)(rows * P)), dim3(TPB), 0, s, in, rmap, src, sd, v,
                     plus, pitch_p, minus, pitch_m, diag_scale, nt);
  return hipGetLastError();
}

template <typename CT>
hipError_t combine_rows_t(const CT* Cp, const CT* Cm, long long pitch_p, long long pitch_m, long long rows, int v,
                          double* R, Idx2 cmap, long long sy, long long sz, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int nt = (v + PS - 1) / PS;
  const long long P = 8LL * ((nt * (nt + 1) / 2 + 7) / 8);
  if (rows * P > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pair_combine_rows_kernel<CT>, dim3((unsigned)(rows * P)), dim3(TPB), 0, s, Cp, Cm,
                     pitch_p, pitch_m, v, R, cmap, sy, sz, nt);
  return hipGetLastError();
}

template <typename CT>
hipError_t combine_cols_t(const CT* CpT, const CT* CmT, long long ncol, const int2* yz, int v, double* R, Idx2 ccol,
                          long long sy, long long sz, hipStream_t s) {
  const long long P = (long long)v * (v + 1) / 2;
  if (ncol <= 0) return hipSuccess;
  if (P > INT_MAX) return hipErrorInvalidValue;
  const unsigned gy = (unsigned)std::min<long long>((ncol + TPB - 1) / TPB, 64);
  hipLaunchKernelGGL(pair_combine_cols_kernel<CT>, dim3((unsigned)P, gy), dim3(TPB), 0, s, CpT, CmT, ncol, yz, v, R,
                     ccol, sy, sz);
  return hipGetLastError();
}

hipError_t pair_combine_rows(const double* Cp, const double* Cm, long long pitch_p, long long pitch_m, long long rows,
                             int v, double* R, Idx2 cmap, long long sy, long long sz, hipStream_t s) {
  return combine_rows_t(Cp, Cm, pitch_p, pitch_m, rows, v, R, cmap, sy, sz, s);
}
hipError_t pair_combine_rows(const float* Cp, const float* Cm, long long pitch_p, long long pitch_m, long long rows,
                             int v, double* R, Idx2 cmap, long long sy, long long sz, hipStream_t s) {
  return combine_rows_t(Cp, Cm, pitch_p, pitch_m, rows, v, R, cmap, sy, sz, s);
}
hipError_t pair_combine_cols(const double* CpT, const double* CmT, long long ncol, const int2* yz, int v, double* R,
                             Idx2 ccol, long long sy, long long sz, hipStream_t s) {
  return combine_cols_t(CpT, CmT, ncol, yz, v, R, ccol, sy, sz, s);
}
hipError_t pair_combine_cols(const float* CpT, const float* CmT, long long ncol, const int2* yz, int v, double* R,
                             Idx2 ccol, long long sy, long long sz, hipStream_t s) {
  return combine_cols_t(CpT, CmT, ncol, yz, v, R, ccol, sy, sz, s);
}

// ---------------------------------------------------------------------------
// T3 -> R1 feedback from one batch of spin-summed slabs (see feedback_r1)
// ---------------------------------------------------------------------------
namespace {

__global__ void r1_feedback_kernel(const double* __restrict__ U, const double* __restrict__ vvT,
                                   double* __restrict__ r1, int o, int v, int S, int f0) {
  __shared__ double red[TPB];
  const int ia = blockIdx.x;
  const int i = ia / v, a = ia - (ia / v) * v;
  const long long v2 = (long long)v * v, rowS = (long long)S * v2;
  double acc = 0.0;
  for (int jj = 0; jj < S; ++jj) {
    for (int k = 0; k < o; ++k) {
      const double* M = vvT + ((long long)(f0 + jj) * o + k) * v2;            // [c][b]
      const double* U1 = U + ((long long)(k * o + i) * v) * rowS + jj * v2 + (long long)a * v;  // + c rowS + b
      const double* U2 = U + ((long long)(k * o + i) * v + a) * rowS + jj * v2;              // + c v + b
      for (long long e = threadIdx.x; e < v2; e += TPB) {
        const int c = (int)(e / v), b = (int)(e - (long long)c * v);
        acc += M[e] * (2.0 * U1[(long long)c * rowS + b] - U2[e]);
      }
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) r1[ia] += 0.5 * red[0];
}

// Y[b*sb + f*sf + b*sp + q*sq] += alpha * X[f*xf + q] for b < nb, f < nf, q < nq.
__global__ void gather_rows_kernel(const double* __restrict__ in, long long ld_in, const int* __restrict__ rows,
                                   int nrows, long long ncols, double* __restrict__ out, long long ld_out) {
  const long long total = (long long)nrows * ncols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / ncols, c = e - r * ncols;
    out[r * ld_out + c] = in[(long long)rows[r] * ld_in + c];
  }
}

__global__ void add_diag_rows_kernel(double* __restrict__ Y, const double* __restrict__ X, int nb, int nf, int nq,
                                     long long sb, long long sf, long long sp, long long sq, long long xf,
                                     double alpha) {
  const long long total = (long long)nb * nf * nq;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int q = (int)(e % nq);
    const long long r = e / nq;
    const int f = (int)(r % nf);
    const int b = (int)(r / nf);
    Y[b * (sb + sp) + f * sf + q * sq] += alpha * X[f * xf + q];
  }
}

}  // namespace

hipError_t feedback_r1(const double* U, const double* vvT, double* r1, int o, int v, int S, int f0,
                       hipStream_t s) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(r1_feedback_kernel, dim3((unsigned)(o * v)), dim3(TPB), 0, s, U, vvT, r1, o, v, S, f0);
  return hipGetLastError();
}

hipError_t gather_rows(const double* in, long long ld_in, const int* rows, int nrows, long long ncols, double* out,
                       long long ld_out, hipStream_t s) {
  const long long total = (long long)nrows * ncols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(total, TPB * 4)), dim3(TPB), 0, s, in, ld_in, rows, nrows,
                     ncols, out, ld_out);
  return hipGetLastError();
}

hipError_t add_diag_rows(double* Y, const double* X, int nb, int nf, int nq, long long sb, long long sf, long long sp,
                         long long sq, long long xf, double alpha, hipStream_t s) {
  const long long total = (long long)nb * nf * nq;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_diag_rows_kernel, dim3(blocks_for(total, TPB * 4)), dim3(TPB), 0, s, Y, X, nb, nf, nq, sb,
                     sf, sp, sq, xf, alpha);
  return hipGetLastError();
}

hipError_t add_pair_diag(double* W, const double* F, long long ldF, int nx, double c, hipStream_t s) {
  const long long n3 = (long long)nx * nx * nx;
  hipLaunchKernelGGL(pair_diag_kernel, dim3(blocks_for(n3, TPB * 4)), dim3(TPB), 0, s, W, F, ldF, nx, c, 0);
  hipLaunchKernelGGL(pair_diag_kernel, dim3(blocks_for(n3, TPB * 4)), dim3(TPB), 0, s, W, F, ldF, nx, c, 1);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// DIIS on the device (Sec. "Distributed DIIS"): the history, its overlap
// matrix and its bookkeeping stay in device memory, so that one iteration
// (residual, Jacobi step, extrapolation, energy) runs without the host and
// can be recorded into a graph and replayed.
// ---------------------------------------------------------------------------
namespace {

constexpr int DIIS_CH = TPB * 16;  // elements per overlap chunk

__device__ __forceinline__ void diis_chunk(const DiisArgs& a, long long c, long long& lo, long long& hi, double& w) {
  const long long nc12 = (a.n12 + DIIS_CH - 1) / DIIS_CH;
  if (c < nc12) {
    lo = c * DIIS_CH;
    hi = lo + DIIS_CH < a.n12 ? lo + DIIS_CH : a.n12;
    w = 1.0;
    return;
  }
  const long long nct = (a.bs + DIIS_CH - 1) / DIIS_CH;
  const long long t = (c - nc12) / nct, q = (c - nc12) - t * nct;
  lo = a.n12 + t * a.bs + q * DIIS_CH;
  const long long end = a.n12 + (t + 1) * a.bs;
  hi = lo + DIIS_CH < end ? lo + DIIS_CH : end;
  w = (double)a.tri[t].w;
}

// part[j][c] = w_c sum over chunk c of e_new * errs[j] (j < M), or e_new^2 (j = M),
// with e_new = vnew - old.
__global__ void diis_overlap_kernel(const double* __restrict__ vnew, const double* __restrict__ old,
                                    const double* __restrict__ errs, DiisArgs a, long long nchunk,
                                    double* __restrict__ part) {
  __shared__ double red[TPB];
  const long long c = blockIdx.x;
  const int j = blockIdx.y;
  long long lo, hi;
  double w;
  diis_chunk(a, c, lo, hi, w);
  const double* ej = errs + (long long)j * a.L;
  double acc = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += TPB) {
    const double e = vnew[i] - old[i];
    acc += e * (j < a.M ? ej[i] : e);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[(long long)j * nchunk + c] = w * s;
}

__global__ void diis_finalize_kernel(const double* __restrict__ part, long long nchunk, double* __restrict__ d) {
  __shared__ double red[TPB];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < nchunk; i += TPB) acc += part[(long long)j * nchunk + i];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) d[j] = s;
}

// One thread: enter the new overlaps into B, advance the ring, solve the
// bordered system over the vectors held (oldest first) by LU with partial
// pivoting; a singular system drops the oldest vector for good and retries.
__global__ void diis_solve_kernel(const double* __restrict__ d, double* __restrict__ B, int* __restrict__ st,
                                  double* __restrict__ coef, int M, int start) {
  __shared__ double A[(DIIS_MAX + 1) * (DIIS_MAX + 1)];
  __shared__ double rhs[DIIS_MAX + 1], x[DIIS_MAX + 1];
  __shared__ int order[DIIS_MAX];
  if (threadIdx.x != 0) return;
  const int k = st[0];
  const int n_new = st[1] + 1 < M ? st[1] + 1 : M;
  for (int idx = 0; idx < n_new; ++idx) order[idx] = (k - n_new + 1 + idx + M) % M;
  for (int idx = 0; idx < n_new; ++idx) {
    const int j = order[idx];
    const double b = (j == k) ? d[M] : d[j];
    B[k * M + j] = b;
    B[j * M + k] = b;
  }
  st[0] = (k + 1) % M;
  st[1] = n_new;
  st[2] = k;
  st[3] = 0;
  st[4] = 0;
  if (n_new < start) return;
  int first = 0;
  while (true) {
    const int m = n_new - first, N = m + 1;
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) A[r * N + c] = B[order[first + r] * M + order[first + c]];
    for (int r = 0; r < m; ++r) {
      A[r * N + m] = -1.0;
      A[m * N + r] = -1.0;
      rhs[r] = 0.0;
    }
    A[m * N + m] = 0.0;
    rhs[m] = -1.0;
    double amax = 0.0;
    for (int i = 0; i < N * N; ++i) amax = fmax(amax, fabs(A[i]));
    bool singular = false;
    for (int c = 0; c < N && !singular; ++c) {
      int pr = c;
      for (int r = c + 1; r < N; ++r)
        if (fabs(A[r * N + c]) > fabs(A[pr * N + c])) pr = r;
      const double pv = fabs(A[pr * N + c]);
      if (pv <= 1e-300 || pv < 1e-25 * amax) {
        singular = true;
        break;
      }
      if (pr != c) {
        for (int q = 0; q < N; ++q) {
          const double t = A[pr * N + q];
          A[pr * N + q] = A[c * N + q];
          A[c * N + q] = t;
        }
        const double t = rhs[pr];
        rhs[pr] = rhs[c];
        rhs[c] = t;
      }
      for (int r = c + 1; r < N; ++r) {
        const double f = A[r * N + c] / A[c * N + c];
        for (int q = c; q < N; ++q) A[r * N + q] -= f * A[c * N + q];
        rhs[r] -= f * rhs[c];
      }
    }
    if (!singular) {
      for (int r = N - 1; r >= 0; --r) {
        double acc = rhs[r];
        for (int q = r + 1; q < N; ++q) acc -= A[r * N + q] * x[q];
        x[r] = acc / A[r * N + r];
        if (!isfinite(x[r])) singular = true;
      }
    }
    if (!singular) {
      for (int idx = 0; idx < m; ++idx) {
        coef[idx] = x[idx];
        st[5 + idx] = order[first + idx];
      }
      st[4] = m;
      st[3] = 1;
      return;
    }
    if (m <= 1) return;
    ++first;
    st[1] -= 1;
  }
}

// The new vector and its error enter the slot the solve assigned.
__global__ void diis_push_kernel(const double* __restrict__ vnew, const double* __restrict__ old,
                                 double* __restrict__ vecs, double* __restrict__ errs, long long L,
                                 const int* __restrict__ st) {
  const long long base = (long long)st[2] * L;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < L; i += (long long)gridDim.x * blockDim.x) {
    const double vn = vnew[i];
    vecs[base + i] = vn;
    errs[base + i] = vn - old[i];
  }
}

// vnew = sum_idx coef[idx] vecs[slot idx] (oldest first) when the solve
// succeeded; otherwise vnew keeps the Jacobi vector.
__global__ void diis_extrapolate_kernel(double* __restrict__ vnew, const double* __restrict__ vecs, long long L,
                                        const int* __restrict__ st, const double* __restrict__ coef) {
  if (st[3] == 0) return;
  const int m = st[4];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < L; i += (long long)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int idx = 0; idx < m; ++idx) acc = fma(coef[idx], vecs[(long long)st[5 + idx] * L + i], acc);
    vnew[i] = acc;
  }
}

__global__ void diis_reset_kernel(int* __restrict__ st, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) st[i] = 0;
}

// scal[6] = scal[4] + 2 scal[5] (the energy); out[0..3] = scal[0..2], scal[6].
__global__ void energy_scalars_kernel(double* __restrict__ scal, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double e = scal[4] + 2.0 * scal[5];
  scal[6] = e;
  if (out) {
    out[0] = scal[0];
    out[1] = scal[1];
    out[2] = scal[2];
    out[3] = e;
  }
}

}  // namespace

long long diis_chunks(const DiisArgs& a) {
  const long long nc12 = (a.n12 + DIIS_CH - 1) / DIIS_CH;
  if (a.L <= a.n12 || a.bs <= 0) return nc12;
  return nc12 + (long long)a.ntri * ((a.bs + DIIS_CH - 1) / DIIS_CH);
}

hipError_t diis_device_step(double* vnew, const double* old, double* vecs, double* errs, double* part, double* d,
                            double* B, int* st, double* coef, const DiisArgs& a, hipStream_t s) {
  if (a.M < 1 || a.M > DIIS_MAX || a.L <= 0) return hipErrorInvalidValue;
  const long long nc = diis_chunks(a);
  if (nc > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(diis_overlap_kernel, dim3((unsigned)nc, (unsigned)(a.M + 1)), dim3(TPB), 0, s,
                     (const double*)vnew, old, (const double*)errs, a, nc, part);
  hipLaunchKernelGGL(diis_finalize_kernel, dim3((unsigned)(a.M + 1)), dim3(TPB), 0, s, (const double*)part, nc, d);
  hipLaunchKernelGGL(diis_solve_kernel, dim3(1), dim3(64), 0, s, (const double*)d, B, st, coef, a.M, a.start);
  hipLaunchKernelGGL(diis_push_kernel, dim3(blocks_for(a.L, TPB * 4)), dim3(TPB), 0, s, (const double*)vnew, old,
                     vecs, errs, a.L, (const int*)st);
  hipLaunchKernelGGL(diis_extrapolate_kernel, dim3(blocks_for(a.L, TPB * 4)), dim3(TPB), 0, s, vnew,
                     (const double*)vecs, a.L, (const int*)st, (const double*)coef);
  return hipGetLastError();
}

hipError_t diis_device_reset(int* st, hipStream_t s) {
  hipLaunchKernelGGL(diis_reset_kernel, dim3(1), dim3(64), 0, s, st, DIIS_STATE);
  return hipGetLastError();
}

hipError_t energy_scalars(double* scal, double* out, hipStream_t s) {
  hipLaunchKernelGGL(energy_scalars_kernel, dim3(1), dim3(64), 0, s, scal, out);
  return hipGetLastError();
}

}  // namespace cct
