// Internal declarations shared by the kernels and the host runtime of libcct.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace cct {

// Two-level index map: i -> (i / inner) * s_hi + (i % inner) * s_lo.
// inner == 0 means one level: i -> i * s_lo.
struct Idx2 {
  int inner;
  long long s_hi, s_lo;
};

static inline Idx2 idx1(long long s) { return Idx2{0, 0, s}; }
static inline Idx2 idx2(int inner, long long s_hi, long long s_lo) { return Idx2{inner, s_hi, s_lo}; }

// C[b](m,n) = alpha * sum_k A[b](m,k) B[b](k,n) + beta * C[b](m,n)
struct GemmArgs {
  int M, N, K, batch;
  const void* A; Idx2 am, ak; long long a_batch;
  const void* B; Idx2 bk, bn; long long b_batch;
  double* C; Idx2 cm, cn; long long c_batch;
  double alpha, beta;
  // Elements addressable from A, B, C (0 = unchecked).  When set, the host
  // verifies before launch that every index map stays inside the operand.
  long long a_len, b_len, c_len;
  // Optional scratch for splitting a long K over workgroups when the output
  // has few tiles (FP64 only): partial products go to split_ws (split_cap
  // doubles) and a fixed-order reduction adds them into C.  nullptr: no split.
  double* split_ws;
  long long split_cap;
};

// Largest offset reached by an index map over [0, n) (non-negative strides).
static inline long long idx_max(const Idx2& d, long long n) {
  if (n <= 0) return 0;
  if (d.inner == 0) return (n - 1) * d.s_lo;
  const long long hi = (n - 1) / d.inner;
  long long best = hi * d.s_hi + ((n - 1) % d.inner) * d.s_lo;
  if (hi >= 1) {
    const long long alt = (hi - 1) * d.s_hi + (long long)(d.inner - 1) * d.s_lo;
    if (alt > best) best = alt;
  }
  return best;
}

enum class Prec { F64 = 0, F32 = 1, BF16X3 = 2 };

// Strided FP64 product (prec must be Prec::F64; the low-precision modes run
// on converted K-contiguous operands through gemm_nt_lp).
hipError_t gemm(const GemmArgs& g, Prec prec, hipStream_t s);

// C[b](m,n) = alpha * sum_k A[b][m*lda + k] * B[b][n*ldb + k] + beta * C[b](m,n):
// both operands K-contiguous (row-major M x K and N x K), the output through
// two-level index maps.  Requires K, lda, ldb even and 16-byte aligned A, B
// (checked; hipErrorInvalidValue otherwise).
struct NtArgs {
  int M, N, K, batch;
  const double* A; long long lda, a_batch;
  const double* B; long long ldb, b_batch;
  double* C; Idx2 cm, cn; long long c_batch;
  double alpha, beta;
  long long a_len, b_len, c_len;  // bounds for the host check (0 = unchecked)
  int variant;                    // tile variant (0 = default)
  int b_kn;                       // 1: B is stored [K][N] (row stride ldb, N contiguous) instead of [N][K]
  int b_map;                      // with b_kn: column n of a B row sits at map2(bnm, n) (pairs n, n+1
  Idx2 bnm;                       // adjacent: bnm.inner even, bnm.s_lo == 1) instead of at n
};
hipError_t gemm_nt(const NtArgs& g, Prec prec, hipStream_t s);

// Y = alpha * X + beta * Y over an index space of up to 6 dimensions.
struct PermArgs {
  int nd;
  long long dim[6];
  long long sx[6], sy[6];
  double alpha, beta;
};
hipError_t permute_add(const double* X, double* Y, const PermArgs& p, hipStream_t s);

// Location of an unpacked T3 block: t_{pqr}^{u0 u1 u2} = T[off + u0*s0 + u1*s1 + u2*s2].
struct BlockRef {
  long long off;
  int s[3];
  int pad;
};

// Element formats of operands written by the bandwidth kernels:
//   OUT_F64: double; OUT_F32: float; OUT_BF16X2: two bf16 planes (hi at
//   out[i], lo at out[plane + i], hi = bf16(x), lo = bf16(x - hi));
//   OUT_BF16X2I: the same pair stored by blocks of 32 consecutive elements,
//   the block's 32 hi values then its 32 lo values (hi of element i at
//   out[2i - i % 32], lo 32 further on), so that one 128-byte line holds both
//   halves of 32 values of a row whose length is a multiple of 32.
enum OutFmt { OUT_F64 = 0, OUT_F32 = 1, OUT_BF16X2 = 2, OUT_BF16X2I = 3 };
struct OutSpec {
  void* p;
  int fmt;
  long long plane;  // element offset of the lo plane (OUT_BF16X2)
};

// One term of an unpacked element: coef * t_{occ}^{virt} where occ[m] selects
// the occupied index at position m (0,1: the slot's fixed indices; 2,3: the
// free indices) and virt[m] selects which of (x,y,z) sits at position m.
struct UnpackTerm {
  double coef;
  int occ[3];
  int virt[3];
};

struct UnpackArgs {
  int o, v, nslots, nfree;
  int fast;  // axis running fastest across threads: 0 = z, 1 = y, 2 = x (the output's unit-stride axis)
  int nterms;
  UnpackTerm terms[6];
  long long s_free[2], s_x, s_y, s_z, s_slot;
  // optional second copy of the same unpacked values in another layout
  // (unpack_t3_dual): its strides and unit-stride axis
  int fast2;
  long long s2_free[2], s2_x, s2_y, s2_z, s2_slot;
};
// slots: device array of int2 (fixed occupied indices) per slot.
hipError_t unpack_t3(const double* T, const BlockRef* tbl, const int2* slots, double* out,
                     const UnpackArgs& a, hipStream_t s);
hipError_t unpack_t3_fmt(const double* T, const BlockRef* tbl, const int2* slots, OutSpec out, const UnpackArgs& a,
                         hipStream_t s);
// The same values written twice: to out with the s_* strides and to out2
// with the s2_* strides (one gather pass for two layouts).
hipError_t unpack_t3_dual(const double* T, const BlockRef* tbl, const int2* slots, OutSpec out, OutSpec out2,
                          const UnpackArgs& a, hipStream_t s);

// out[b][j][i] = in[b][i][j] for a batch of R x C matrices (row-major).
hipError_t transpose_batched(const double* in, OutSpec out, long long batch, int R, int C, hipStream_t s);
// out[b][i][j][k] = in[b][j][i][k] for a batch of n0 x n1 x n2 tensors (swap of the two outer axes).
hipError_t swap01_batched(const double* in, OutSpec out, long long batch, int n0, int n1, int n2, hipStream_t s);
// out[i] = in[i] in the requested format.
hipError_t convert(const double* in, OutSpec out, long long n, hipStream_t s);

// K-contiguous GEMM on low-precision operands (FP32, or split BF16 planes),
// FP64 output through two-level maps.  lda/ldb/batch strides in elements of
// the operand format; a_plane/b_plane: offset of the lo plane (BF16X3).
struct NtLpArgs {
  int M, N, K, batch;
  const void* A; long long lda, a_batch, a_plane;
  const void* B; long long ldb, b_batch, b_plane;
  double* C; Idx2 cm, cn; long long c_batch;
  double alpha, beta;
  long long a_len, b_len, c_len;
  int variant;  // tile variant (0 = size-based default)
  float* C32;   // split BF16 only: FP32 output here instead of C (exact: the accumulation is FP32; beta 0)
  int il;       // split BF16 only: A and B stored as OUT_BF16X2I (planes unused; logical strides and lengths,
                // multiples of 32)
};
hipError_t gemm_nt_lp(const NtLpArgs& g, Prec prec, hipStream_t s);

// Output-stationary accumulation of temporary Y blocks into packed R3:
// R[t] (a,b,c) += sum_c coef * Z[base + a*sa + b*sb + c*sc].
struct FoldContrib {
  long long base, sa, sb, sc;
  double coef;
};
struct FoldTask {
  int t, nc, c0, pad;
};
hipError_t fold_r3(double* R, long long bs, int v, const double* Z, const FoldTask* tasks, int ntasks,
                   const FoldContrib* contribs, hipStream_t s);
// The same with FP32 contracted blocks (accumulated into FP64 R3).
hipError_t fold_r3(double* R, long long bs, int v, const float* Z, const FoldTask* tasks, int ntasks,
                   const FoldContrib* contribs, hipStream_t s);

// R3 post-processing, norms and Jacobi update on packed blocks.
struct PostArgs {
  int o, v, ntri;
  long long bs;
  int do_update;   // 1: T += R / eps
  int keep_r;      // 1: write post-processed R back
};
// tri: device int4 (i,j,k,mult) per packed triple; eps: device [n] orbital energies.
// partial: device array of per-block partial sums (size >= gridDim used), filled with
// weighted squared norms; returns the number of partials in *npartial.
hipError_t post_update(double* R, double* T, const int4* tri, const double* eps, double* partial,
                       int* npartial, const PostArgs& a, hipStream_t s);

// Deterministic fixed-order sum of n doubles into out[0].
hipError_t reduce_sum(const double* x, long long n, double* out, double* scratch, hipStream_t s);
// Deterministic dot product sum_i w(i) x_i y_i with an optional packed-T3 weight.
hipError_t dot(const double* x, const double* y, long long n, double* out, double* scratch, hipStream_t s);
hipError_t weighted_dot_t3(const double* x, const double* y, const int4* tri, int ntri, long long bs, long long v3,
                           double* out, double* scratch, hipStream_t s);
// out[r][c] = in[r*cols + c] for c < cols, 0 for cols <= c < ld_out, in the
// output's format (rows padded with zeros to a vector-load multiple).
hipError_t copy_pad_rows(const double* in, long long rows, long long cols, OutSpec out, long long ld_out,
                         hipStream_t s);
// out[r*ld + c] = 0 for c0 <= c < ld, every row r < rows (the padding columns).
hipError_t zero_cols(OutSpec out, long long rows, long long ld, long long c0, hipStream_t s);
// Low-energy virtual sub-cube of every packed block (a, b, c < sv):
// gather: sub[t][a][b][c] = T[t][a][b][c]; otherwise the reverse copy.
hipError_t t3_subcube(double* T, double* sub, long long ntri, int v, int sv, bool gather, hipStream_t s);
// y = a*x + b*y (elementwise, n elements)
hipError_t axpby(double a, const double* x, double b, double* y, long long n, hipStream_t s);
hipError_t fill(double* y, double val, long long n, hipStream_t s);
// R1[i][a] += 1/2 sum_{j in [f0, f0+S), k, b, c} vvT[j][k][c][b] (2 U[(k,i,c)][j-f0][a][b] - U[(k,i,a)][j-f0][c][b])
// with U[(k,i,x)][j'][p][q] the single-check spin-summed slab t~_{j k i}^{q x p} (one block per (i,a)).
hipError_t feedback_r1(const double* U, const double* vvT, double* r1, int o, int v, int S, int f0, hipStream_t s);
// Symmetric / antisymmetric pair split of one v x v matrix per row r (element
// (d,e) at in + off(r) + d*sd + e, off(r) = src[r] if src else map2(rmap, r)):
//   plus [r*pitch_p + p(d,e)] = M[d][e] + M[e][d] (d < e), diag_scale*2*M[d][d] (d = e)
//   minus[r*pitch_m + q(d,e)] = M[d][e] - M[e][d] (d < e)
// with p(d,e) = d v - d(d-1)/2 + e - d and q(d,e) = d(v-1) - d(d-1)/2 + e - d - 1;
// columns beyond v(v+1)/2 (plus) and v(v-1)/2 (minus) up to the pitch are zeroed.
hipError_t pair_split(const double* in, Idx2 rmap, const long long* src, long long rows, long long sd, int v,
                      OutSpec plus, long long pitch_p, OutSpec minus, long long pitch_m, double diag_scale,
                      hipStream_t s);
// R[cmap(r) + y*sy + z*sz] += C^{yz} from the pair products of row r (both
// indexed by the output pair p(min(y,z), max(y,z))):
// C^{yz} = (C+[p(y,z)] + C-[p(y,z)])/2 (y < z), (C+[p(z,y)] - C-[p(z,y)])/2 (y > z), C+[p(y,y)]/2.
hipError_t pair_combine_rows(const double* Cp, const double* Cm, long long pitch_p, long long pitch_m, long long rows,
                             int v, double* R, Idx2 cmap, long long sy, long long sz, hipStream_t s);
hipError_t pair_combine_rows(const float* Cp, const float* Cm, long long pitch_p, long long pitch_m, long long rows,
                             int v, double* R, Idx2 cmap, long long sy, long long sz, hipStream_t s);
// The same from transposed products C+T[p][c], C-T[p][c] over ncol columns c, pairs given by yz[p]:
// R[ccol(c) + y*sy + z*sz] += C^{yz}.  (FP32 products: split-BF16 GEMM outputs.)
hipError_t pair_combine_cols(const double* CpT, const double* CmT, long long ncol, const int2* yz, int v, double* R,
                             Idx2 ccol, long long sy, long long sz, hipStream_t s);
hipError_t pair_combine_cols(const float* CpT, const float* CmT, long long ncol, const int2* yz, int v, double* R,
                             Idx2 ccol, long long sy, long long sz, hipStream_t s);
// out[r * ld_out + c] = in[rows[r] * ld_in + c] for r < nrows, c < ncols (rows: device array).
hipError_t gather_rows(const double* in, long long ld_in, const int* rows, int nrows, long long ncols, double* out,
                       long long ld_out, hipStream_t s);
// Y[b*sb + f*sf + b*sp + q*sq] += alpha * X[f*xf + q] for b < nb, f < nf, q < nq.
hipError_t add_diag_rows(double* Y, const double* X, int nb, int nf, int nq, long long sb, long long sf, long long sp,
                         long long sq, long long xf, double alpha, hipStream_t s);
// out[i] += sum_r in[r * n + i] for r = 0..rows-1 (fixed order).
hipError_t add_rows(const double* in, int rows, long long n, double* out, hipStream_t s);
// DIIS on the device.  The history holds M slots of L doubles (vecs, errs);
// the first n12 elements of a vector are T1/T2 (weight 1), the rest packed T3
// blocks of bs elements (weight tri[t].w, the orderings of block t).
// st (DIIS_STATE ints): [0] next slot, [1] vectors held, [2] slot of the newest,
// [3] 1 if the last step extrapolated, [4] vectors in that solve, [5..] their
// slots, oldest first.
constexpr int DIIS_MAX = 64;
constexpr int DIIS_STATE = 5 + DIIS_MAX;
struct DiisArgs {
  long long L, n12, bs;
  const int4* tri;
  int ntri, M, start;
};
// Overlap chunks of one step (size of the partial-sum scratch: (M + 1) x chunks).
long long diis_chunks(const DiisArgs& a);
// One DIIS step on the Jacobi vector vnew (old: the amplitudes before the
// step): overlaps of e = vnew - old with the history, the bordered solve
// (a singular system drops the oldest vector for good), e and vnew enter the
// history, and vnew becomes the extrapolated vector when the solve succeeded.
// part: (M + 1) x diis_chunks doubles, d: M + 1, B: M x M, coef: M.
hipError_t diis_device_step(double* vnew, const double* old, double* vecs, double* errs, double* part, double* d,
                            double* B, int* st, double* coef, const DiisArgs& a, hipStream_t s);
// Empty history (a kernel, so that it may sit in a recorded graph).
hipError_t diis_device_reset(int* st, hipStream_t s);
// scal[6] = scal[4] + 2 scal[5]; out (may be null) receives scal[0..2], scal[6].
hipError_t energy_scalars(double* scal, double* out, hipStream_t s);
// Jacobi update of T1 / T2 with denominators built from eps.
hipError_t jacobi_t1t2(double* t1, const double* r1, double* t2, const double* r2, const double* eps, int o, int v,
                       hipStream_t s);
// W_diag: add c * F[a][d] on the (b == e) diagonal and c * F[b][e] on (a == d) for a [x][y][x][y] tensor.
hipError_t add_pair_diag(double* W, const double* F, long long ldF, int nx, double c, hipStream_t s);

// Permuted combination of v^4 virtual blocks (perturbative quadruples):
//   out[w]  = beta * out[w]  + f(w) * sum_{t: dst_t & 1} coef_t * x_t(w)
//   out2[w] = beta * out2[w] +        sum_{t: dst_t & 2} coef_t * (x_t(w) + vcoef_t * va_t[y0 v + y1] * vb_t[y2 v + y3])
// with y = (w_{perm_t[0]}, .., w_{perm_t[3]}) and x_t(w) = in_t[y0][y1][y2][y3]
// (row-major, w in [0, v)^4); f(w) = 1 / (eps_occ - sum_k eps_v[w_k]) when
// eps_v is set, else 1.  out2 may be null (then no term may have dst & 2);
// no input may be an output.
constexpr int QMAXT = 48;
struct QPermTerm {
  const double* in;
  int perm[4];
  double coef;
  int dst;            // 1: out, 2: out2, 3: both
  const double* va;   // optional rank-one addend of the out2 contribution (nullptr: none)
  const double* vb;
  double vcoef;
};
struct QCombineArgs {
  int v, nterms;
  QPermTerm t[QMAXT];
  double beta;
  const double* eps_v;  // device, v virtual orbital energies (nullptr: no division)
  double eps_occ;       // sum of the four occupied orbital energies
  int tiled;            // 1: every input is tile-major (see rank_k_update_tiled)
};
hipError_t perm_combine(double* out, double* out2, const QCombineArgs& a, hipStream_t s);
// C[m][n] += alpha * sum_{k<K} A[m*lda + k] * B[k*ldb + n], m < M, n < N, C
// row stride ldc: streaming update for K <= 16.  Requires N, ldc, ldb even
// and 16-byte aligned C and B (hipErrorInvalidValue otherwise).
hipError_t rank_k_update(double* C, long long ldc, const double* A, long long lda, const double* B, long long ldb,
                         int M, long long N, int K, double alpha, hipStream_t s);
// The same update of a v^4 block C (row-major [a][b][c][d]; rows m cover the
// first rsplit of the four axes, columns n the rest) written to D in the
// tile-major layout instead of back to C: 8^4 tiles of 4096 consecutive
// doubles, tiles in row-major order over ceil(v/8)^4, elements inside a tile
// row-major; padding positions are not written.  Requires v even.
hipError_t rank_k_update_tiled(const double* C, double* D, int v, int rsplit, const double* A, long long lda,
                               const double* B, long long ldb, int K, double alpha, hipStream_t s);
// Elements of a tile-major v^4 block (padded to whole tiles).
static inline long long tiled_len(int v) {
  const long long nt = (v + 7) / 8;
  return nt * nt * nt * nt * 4096;
}

// --- perturbative quadruples in the virtual-tuple order --------------------
// Four-level index map: i = ((d0 n1 + d1) n2 + d2) n3 + d3 -> sum_k d_k s_k
// (n1, n2, n3 >= 1).
struct Idx4 {
  int n1, n2, n3;
  long long s0, s1, s2, s3;
};

// Segmented, digit-batched FP64 product on the matrix cores:
//   C[z](m, n) (+)= alpha * sum_s sum_{k < K_s} A_s[z](m, k) B_s[z](k, n)
// The batch index z (gridDim.z) is split into nd digits of radices rad (the
// last fastest); each operand of each K segment s sits at base + sum_d
// digit_d * sd[d].  A_s is K-contiguous ([m][k] at m*ld + k) or, with AKM,
// M-contiguous ([k][m] at k*ld + m); B_s is N-contiguous ([k][n] at
// k*ld + n) or, without BKN, K-contiguous ([n][k] at n*ld + k).  C through
// the four-level maps cm, cn plus sum_d digit_d * sc[d].
constexpr int QG_MAXSEG = 3, QG_MAXD = 4;
struct QgOperand {
  const double* p;
  long long ld;
  long long sd[QG_MAXD];
  long long len;  // elements addressable from p (for the host bounds check)
};
struct QGemmArgs {
  int M, N, nseg, nd;
  int K[QG_MAXSEG];
  int rad[QG_MAXD];
  QgOperand a[QG_MAXSEG], b[QG_MAXSEG];
  bool akm, bkn;
  double* C;
  Idx4 cm, cn;
  long long sc[QG_MAXD];
  long long c_len;
  double alpha;
  int accumulate;  // 1: C += alpha A B, 0: C = alpha A B
};
hipError_t qgemm(const QGemmArgs& g, hipStream_t s);

// T3 in the virtual-triangular layout: block vb(a <= b <= c) (lexicographic)
// holds t_{ijk}^{abc} for all i, j, k at vb * o^3 + (i o + j) o + k.  Filled
// from the packed occupied-triangular T3 through the table of ordered
// triples (tbl[(i o + j) o + k]).  cubes: (A, B, C, 0) with A <= B <= C,
// every cube of 16^3 labels that holds a canonical triple; ncubes of them.
hipError_t t3v_transpose(const double* T, const BlockRef* tbl, double* T3v, const int4* cubes, long long ncubes,
                         int o, int v, hipStream_t s);
// Gather of T3v slices: out[blk][e][y0][y1][y2], blk over nd label digits
// (radices rad, first labels st), e over ne values (0..ne-1), y over o^3.
// Column pair c of t3 takes its virtual label from digit lab[c] (lab[c] == 3:
// e) and its occupied index from output axis ax[c].
struct T3Gather {
  int o, v, nd, ne;
  int rad[3], st[3];
  int lab[3], ax[3];
};
hipError_t t3v_gather(const double* T3v, double* out, const T3Gather& g, hipStream_t s);

// Slots of one virtual tile task: first label and size of each of the four
// index ranges.
struct QSlots {
  int st[4], n[4];
};
// Wbar^{vvo}_{ooo} of Eq. q_w_alter for the label pairs (x, y) of slots
// (s0, s1) with the occupied indices of slots (s0, s1, s2) in slot order:
// out[lx][ly][rows][m], rows = the three indices ordered by slot, from
// Voooo[n][k][i][m] = v^{mn}_{ki} and t2[i][j][a][b].
hipError_t q_wo_build(double* out, const double* Voooo, const double* t2, int o, int v, int x0, int nx, int y0, int ny,
                      const int rowpos[3], hipStream_t s);
// Wbar^{vvv}_{voo} of Eq. q_w_alter for x in slot s0 and (y, z) in slots
// (r0, r1): out[lx][ly][lz][j][k][e] = Z_xy[z](j, k, e) + Z_xz[y](k, j, e)
// + the four K = o terms, with Z_ab[c] = 1/2 sum_f v^{ab}_{ef} t_{jk}^{fc}
// laid out [la][lb][lc][j][k][e] (Zxy: slots (s0, r0, r1), Zxz: (s0, r1, r0)),
// Vmyje[m][y][j][e] = v^{my}_{ej}, Vmxje[m][x][j][e] = v^{mx}_{je}.
hipError_t q_wv_build(double* out, const double* Zxy, const double* Zxz, const double* Vmyje, const double* Vmxje,
                      const double* t2, int o, int v, int x0, int nx, int y0, int ny, int z0, int nz, hipStream_t s);
// out[i] = src[idx[i]], i < n.
hipError_t gather_idx(const double* src, const long long* idx, long long n, double* out, hipStream_t s);
// Energy of the tuples of one task (t2R[b][a][i][j] = t_ij^ab): for every
// tuple tau of the dense box
// (slot sizes n[]) with a <= b <= c <= d and no three equal labels,
//   e_tau = 1/|Stab| sum_i (X[tau](i) + Vs(tau, i)) U(tau, i),
//   U = (1/den) sum_pi c_pi R[tau](i o pi),
// R = X + Y (formed in the kernel), Vs the rank-one terms, den the orbital-energy
// denominator; other tuples get 0.  etup[tau] (dense order) and etask (the
// fixed-order sum over the box) are written on the device.
hipError_t q_abc_energy(const double* X, const double* Y, const double* Vvvoo, const double* t2R, const double* eps,
                        const QSlots& sl, int o, int v, const int* orbits, int norb, double* part, double* etup,
                        double* etask, hipStream_t s);
// The block orbits q_abc_energy takes (1 + 24 ints each; size / 25 orbits).
std::vector<int> q_abc_orbits(int o);

}  // namespace cct
