// backtrans.hip -- explicit reflector blocks for the back-transformation.
//
// The reductions keep their reflectors in place (v[0] = 1 implicit, v[1:] in
// the annihilated part of a column, or of a row for right reflectors).  To
// apply a block of pb consecutive reflectors as I - V T V^T (compact WY, the
// I + W Y^T of Sec. 2.1 with Y = V, W = -V T), V is first copied out as an
// explicit j x pb unit lower trapezoid.
#include "common.hpp"

namespace br {

// V(t, q), t < j, q < pb: reflector i0 + q, whose vector starts at index
// r0 + q (r0 = i0 + off).  Zero above the diagonal, 1 on it, below it the
// stored entry at index r0 + t: A(r0 + t, i0 + q) for column storage,
// A(i0 + q, r0 + t) for row storage.
__global__ void k_extract_v(const double *A, int64_t lda, int rowstore, int64_t r0, int64_t i0,
                            int pb, int j, double *V, int64_t ldv) {
  const int64_t total = (int64_t)j * pb;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int t, q;
    if (rowstore) {  // consecutive threads read consecutive reflectors of one row
      q = (int)(idx % pb);
      t = (int)(idx / pb);
    } else {         // consecutive threads read down one column
      t = (int)(idx % j);
      q = (int)(idx / j);
    }
    double v = 0.0;
    if (t == q) {
      v = 1.0;
    } else if (t > q) {
      v = rowstore ? A[(i0 + q) + (r0 + t) * lda] : A[(r0 + t) + (i0 + q) * lda];
    }
    V[t + (int64_t)q * ldv] = v;
  }
}

int launch_extract_v(const double *A, int64_t lda, int rowstore, int64_t r0, int64_t i0, int pb,
                     int j, double *V, int64_t ldv, hipStream_t s) {
  const int64_t total = (int64_t)j * pb;
  if (total <= 0) return 0;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_extract_v, dim3(blocks), dim3(256), 0, s, A, lda, rowstore, r0, i0, pb, j,
                     V, ldv);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
