// panel.hip -- FP64 Householder factorisation of a tall-skinny panel and the
// compact-WY T factor (gfx950).
//
// Panel QR (eq. updateA0): the m x nb panel (nb <= 128) is spread over
// gridDim.x workgroups, R rows each, and stays resident in LDS for the whole
// factorisation.  Column i needs one grid-wide reduction: every workgroup sums,
// over its rows r > i, the products a(r,i) a(r,k) for k = i .. nb-1; with the
// pivot row a(i,.) (held by workgroup 0) these sums give, in every workgroup
// and bit-identically,
//     sigma^2 = s_i,  beta = -sign(a_ii) sqrt(a_ii^2 + sigma^2),
//     tau = (beta - a_ii) / beta,  d = a_ii - beta,
//     z_k = v^T a(:,k) = a(i,k) + s_k / d,
// after which each workgroup applies a(r,k) -= tau v_r z_k to its own rows
// with v_r = a(r,i) / d (v_i = 1).  So a column costs one inter-workgroup
// barrier, never a second pass over the panel.  The partial sums are summed in
// a fixed order, so the result does not depend on timing.
//
// The same kernel factors a row panel (LQ of eq. updateC): the element (r,k)
// of the transposed panel is read from P[k + r*ldp] instead of P[r + k*ldp].
//
// Inter-workgroup waits are bounded (wall clock): a workgroup that waits too
// long raises an abort flag that releases every other workgroup, and the
// library reports BANDRED_ERR_TIMEOUT instead of hanging.
#include "common.hpp"

namespace br {

__device__ __forceinline__ long long wall_ticks() { return (long long)wall_clock64(); }

// Arrive at barrier number `target / nwg` and wait for all workgroups.
// Called by one thread.  Returns false when the wait was abandoned.
__device__ bool grid_barrier(const PanelDesc &d, unsigned target) {
  __hip_atomic_fetch_add(d.counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  const long long t0 = wall_ticks();
  while (__hip_atomic_load(d.counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(d.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      return false;
    if (wall_ticks() - t0 > d.timeout_ticks) {
      __hip_atomic_store(d.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(d.status, (int)BANDRED_ERR_TIMEOUT, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

template <bool ROWMAJ>
__global__ __launch_bounds__(kThreads) void k_panel(PanelDesc d) {
  extern __shared__ double L[];  // R x LDW, row-major: L[r*LDW + k] = a(r0 + r, k)
  __shared__ double red[2][kNbMax];
  __shared__ double sv[kNbMax];
  __shared__ double zv[kNbMax];
  __shared__ int go;

  if (d.gate && *d.gate != d.gate_val) return;
  const int nb = d.nb;
  const int LDW = (nb & 1) ? nb : nb + 1;
  const int g = blockIdx.x, nwg = gridDim.x, tid = threadIdx.x;
  const int r0 = g * d.R;
  const int rows = min(d.R, d.m - r0);
  const int k = tid & (kNbMax - 1), h = tid >> 7;

  // load the block
  if (!ROWMAJ) {
    for (int idx = tid; idx < rows * nb; idx += kThreads) {
      const int r = idx % rows, kk = idx / rows;
      L[r * LDW + kk] = d.P[(r0 + r) + (int64_t)kk * d.ldp];
    }
  } else {
    for (int idx = tid; idx < rows * nb; idx += kThreads) {
      const int kk = idx % nb, r = idx / nb;
      L[r * LDW + kk] = d.P[kk + (int64_t)(r0 + r) * d.ldp];
    }
  }
  __syncthreads();

  for (int i = 0; i < nb; ++i) {
    const int rstart = max(0, i + 1 - r0);  // first local row with global index > i
    // (1) partial column dots over this workgroup's rows
    {
      double acc = 0.0;
      if (k >= i && k < nb)
        for (int r = rstart + h; r < rows; r += 2) acc += L[r * LDW + i] * L[r * LDW + k];
      red[h][k] = acc;
    }
    __syncthreads();
    double *pbuf = d.part + (size_t)(i & 1) * nwg * kNbMax;
    if (tid < kNbMax) {
      if (k >= i && k < nb) {
        pbuf[g * kNbMax + k] = red[0][k] + red[1][k];
        if (g == 0) d.piv[i * kNbMax + k] = L[i * LDW + k];
      }
      // make this wave's stores visible device-wide before the arrival below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    // (2) grid barrier
    __syncthreads();
    if (tid == 0) go = grid_barrier(d, (unsigned)(i + 1) * (unsigned)nwg) ? 1 : 0;
    __syncthreads();
    if (!go) return;
    // (3) reduce the partial sums in a fixed order
    {
      double s = 0.0;
      if (k >= i && k < nb)
        for (int q = h; q < nwg; q += 2) s += pbuf[q * kNbMax + k];
      red[h][k] = s;
    }
    __syncthreads();
    if (tid < kNbMax && k >= i && k < nb) {
      sv[k] = red[0][k] + red[1][k];
      zv[k] = d.piv[i * kNbMax + k];
    }
    __syncthreads();
    // (4) the reflector (every thread forms the same scalars)
    const double alpha = zv[i];
    const double sig2 = sv[i];
    double tau = 0.0, dv = 1.0, beta = alpha;
    if (sig2 != 0.0) {
      const double nrm = sqrt(alpha * alpha + sig2);
      beta = (alpha < 0.0) ? nrm : -nrm;
      tau = (beta - alpha) / beta;
      dv = alpha - beta;
    }
    if (tau != 0.0) {
      if (tid < kNbMax && k > i && k < nb) zv[k] = zv[k] + sv[k] / dv;
      for (int r = rstart + tid; r < rows; r += kThreads) L[r * LDW + i] = L[r * LDW + i] / dv;
    }
    __syncthreads();
    // (5) apply H = I - tau v v^T to columns k > i of this workgroup's rows
    if (tau != 0.0 && k > i && k < nb) {
      const double tz = tau * zv[k];
      for (int r = rstart + h; r < rows; r += 2) L[r * LDW + k] -= L[r * LDW + i] * tz;
      if (g == 0 && h == 0) L[i * LDW + k] -= tz;
    }
    if (g == 0 && tid == 0) {
      L[i * LDW + i] = beta;
      d.tau[i] = tau;
    }
    __syncthreads();
  }

  // write back in place and the explicit V (unit diagonal, zeros above)
  if (!ROWMAJ) {
    for (int idx = tid; idx < rows * nb; idx += kThreads) {
      const int r = idx % rows, kk = idx / rows;
      d.P[(r0 + r) + (int64_t)kk * d.ldp] = L[r * LDW + kk];
    }
  } else {
    for (int idx = tid; idx < rows * nb; idx += kThreads) {
      const int kk = idx % nb, r = idx / nb;
      d.P[kk + (int64_t)(r0 + r) * d.ldp] = L[r * LDW + kk];
    }
  }
  for (int idx = tid; idx < rows * nb; idx += kThreads) {
    const int r = idx % rows, kk = idx / rows;
    const int gr = r0 + r;
    const double v = (gr == kk) ? 1.0 : ((gr > kk) ? L[r * LDW + kk] : 0.0);
    d.V[gr + (int64_t)kk * d.ldv] = v;
  }
}

// T factor of the compact WY form (the T of Sec. 4.1's W = Y T):
// T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) S(0:i, i) with S = V^T V.
__global__ __launch_bounds__(kThreads) void k_larft(const double *S, int ldS, const double *tau,
                                                    int nb, double *T, int ldT, const int *gate,
                                                    int gate_val) {
  if (gate && *gate != gate_val) return;
  constexpr int LD = kNbMax + 1;
  __shared__ double Tl[kNbMax * LD];  // column-major: Tl[m*LD + l] = T(l, m)
  __shared__ double s[kNbMax];
  __shared__ double red[2][kNbMax];
  const int tid = threadIdx.x;
  const int l = tid & (kNbMax - 1), h = tid >> 7;
  for (int i = 0; i < nb; ++i) {
    const double ti = tau[i];
    if (tid < nb) s[tid] = S[tid + (int64_t)i * ldS];
    __syncthreads();
    double acc = 0.0;
    if (l < i)
      for (int m = l + h; m < i; m += 2) acc += Tl[m * LD + l] * s[m];
    red[h][l] = acc;
    __syncthreads();
    if (tid < nb) {
      double v = 0.0;
      if (l < i) v = -ti * (red[0][l] + red[1][l]);
      else if (l == i) v = ti;
      Tl[i * LD + l] = v;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += kThreads) {
    const int ll = idx % nb, m = idx / nb;
    T[ll + (int64_t)m * ldT] = Tl[m * LD + ll];
  }
}

int panel_lds_bytes(int R, int nb) {
  const int LDW = (nb & 1) ? nb : nb + 1;
  return R * LDW * (int)sizeof(double);
}

int launch_panel(bool rowmajor, const PanelDesc &d, int nwg, hipStream_t s) {
  const int lds = panel_lds_bytes(d.R, d.nb);
  static bool attr_set = false;
  if (!attr_set) {
    BR_HIP_CHECK(hipFuncSetAttribute((const void *)k_panel<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
    BR_HIP_CHECK(hipFuncSetAttribute((const void *)k_panel<true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
    attr_set = true;
  }
  if (rowmajor)
    hipLaunchKernelGGL(k_panel<true>, dim3(nwg), dim3(kThreads), lds, s, d);
  else
    hipLaunchKernelGGL(k_panel<false>, dim3(nwg), dim3(kThreads), lds, s, d);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

int launch_larft(const double *S, int ldS, const double *tau, int nb, double *T, int ldT,
                 hipStream_t s, const int *gate, int gate_val) {
  hipLaunchKernelGGL(k_larft, dim3(1), dim3(kThreads), 0, s, S, ldS, tau, nb, T, ldT, gate,
                     gate_val);
  BR_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace br
