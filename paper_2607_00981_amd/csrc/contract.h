// Device tensor views and a small contraction planner on top of the strided
// GEMM: C(labels) = alpha * A(labels) * B(labels) + beta * C(labels), with
// every index group (rows M, columns N, contracted K) mapped onto at most two
// strided levels so that permuted views are read in place; operands whose
// groups cannot be expressed that way are first copied into contiguous
// scratch.
#pragma once

#include "internal.h"

#include <initializer_list>
#include <string>

namespace cct {

struct DT {
  double* p = nullptr;
  int nd = 0;
  long long dim[6] = {0, 0, 0, 0, 0, 0};
  long long st[6] = {0, 0, 0, 0, 0, 0};
  long long size() const {
    long long s = 1;
    for (int i = 0; i < nd; ++i) s *= dim[i];
    return s;
  }
};

// Contiguous row-major view.
DT dense(double* p, std::initializer_list<long long> dims);
// Arbitrary strided view.
DT strided(double* p, std::initializer_list<long long> dims, std::initializer_list<long long> strides);

// Stack allocator over one device buffer; allocations are released in LIFO
// order by resetting to a mark.  All users share one stream, so reuse after a
// reset is ordered behind earlier kernels.
class Arena {
 public:
  void init(char* base, size_t bytes) { base_ = base; cap_ = bytes; top_ = 0; peak_ = 0; }
  double* alloc(size_t n_doubles);  // nullptr if the arena is exhausted
  size_t mark() const { return top_; }
  void reset(size_t m) { top_ = m; }
  size_t capacity() const { return cap_; }
  size_t peak() const { return peak_; }
  size_t available() const { return cap_ - top_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, top_ = 0, peak_ = 0;
};

struct Status {
  hipError_t err = hipSuccess;
  std::string msg;
  bool ok() const { return err == hipSuccess && msg.empty(); }
};

// Y(ly) = alpha * X(lx) + beta * Y(ly); labels of X are a permutation of ly.
Status accumulate(hipStream_t s, double alpha, const DT& X, const char* lx, double beta, const DT& Y, const char* ly);

// C(lc) = alpha * sum_K A(la) B(lb) + beta * C(lc).  No label may occur in all
// three operands or in only one of them.
Status contract(Arena& ws, hipStream_t s, Prec prec, double alpha, const DT& A, const char* la, const DT& B,
                const char* lb, double beta, const DT& C, const char* lc);

}  // namespace cct
