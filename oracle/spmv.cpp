// Multi-threaded CSR product y = A x for the oracle's assembled matrix --
// TEST INFRASTRUCTURE ONLY (the CPU baseline of the benchmark).
//
// The oracle applies the P1 operator as the sparse matrix it assembles
// element by element (Section 5.2.1); this file only evaluates that product
// on all host cores, the library primitive a CPU code would call.  Rows are
// split into contiguous ranges of about equal nonzero count, one per thread;
// each row is summed in column order.  Built by __graft_entry__.build() as
// oracle/libspmv.so; the GPU library never links or loads it.
#include <stdint.h>

#include <thread>
#include <vector>

extern "C" {

// y[r] = sum_k data[k] * x[indices[k]], k in [indptr[r], indptr[r + 1]),
// for r in [0, nrows), with `threads` worker threads (>= 1).  Pointers are
// host arrays of the CSR matrix (int64 row pointers, int32 column indices,
// FP64 values) and FP64 vectors.  Returns 0, or -1 on invalid arguments.
int oracle_csr_spmv(int64_t nrows, const int64_t* indptr, const int32_t* indices,
                    const double* data, const double* x, double* y, int threads) {
  if (nrows < 0 || !indptr || !indices || !data || !x || !y || threads < 1) return -1;
  const int64_t nnz = indptr[nrows];
  std::vector<int64_t> cut(threads + 1, nrows);
  cut[0] = 0;
  // row ranges of about nnz / threads nonzeros each
  for (int t = 1, r = 0; t < threads; ++t) {
    const int64_t target = nnz * t / threads;
    while (r < nrows && indptr[r] < target) ++r;
    cut[t] = r;
  }
  auto work = [&](int t) {
    for (int64_t r = cut[t]; r < cut[t + 1]; ++r) {
      double s = 0.0;
      for (int64_t k = indptr[r]; k < indptr[r + 1]; ++k) s += data[k] * x[indices[k]];
      y[r] = s;
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  return 0;
}

}  // extern "C"
