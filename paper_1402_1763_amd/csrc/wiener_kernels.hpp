// Kernels around the deterministic messenger iteration (the Wiener filter of
// the messenger scheme: the Gibbs sweep with every unit normal set to zero and
// P held fixed) and its adjoint.
//
// One iteration maps s_k to s_{k+1} = C (alpha s_k + beta), with
// C = F^-1 diag(f) F, f_b = P_b / (P_b + tau) per |k| bin, f = 0 at k = 0,
// alpha = 1 - tau R_i^2/N_i and beta = tau R_i d_i / N_i on observed voxels,
// (1, 0) elsewhere (Sec. 3.1: the means of the messenger and signal
// conditionals).  With R = 1 the loss is chi2_K = sum_i w_i d_i (d_i - s_K,i),
// w_i = 1/N_i (0 where unobserved), which tends to d^T (S + N)^-1 d as K
// grows; a response is handled by rescaling d to d / R.
//
// The sweep kernels run the iteration in deterministic modes (kZDet, kXDet,
// kXAdj, kPkGrad).  The kernels here build the iteration's inputs and finish
// its outputs; all of them walk the z-pass coefficient order, entry
// ((tile EPT + e) NT + tid) covering voxels (ix, iya, n) and (ix, iya + 1, n).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sweep_kernels.hpp"

namespace mf {

constexpr int kWienerThreads = 256;

template <typename R, int N>
__device__ __forceinline__ void entry_voxels(size_t idx, size_t& va, size_t& vb) {
  using T = ZTile<R, N>;
  const int tile = static_cast<int>(idx / (static_cast<size_t>(T::EPT) * T::NT));
  const int rem = static_cast<int>(idx % (static_cast<size_t>(T::EPT) * T::NT));
  int ix = 0, iya = 0, n = 0;
  zpass_coef_voxel<R, N>(tile, rem / T::NT, rem % T::NT, ix, iya, n);
  va = (static_cast<size_t>(ix) * N + iya) * N + n;
  vb = va + N;
}

// wcoef = (alpha_a, alpha_b, o_a d_a, o_b d_b): the messenger coefficients
// of the problem's noise model with new data d (FP64, [ix][iy][iz]); beta =
// tau d / N = o d with o = tau / N = 1 - alpha (with R = 1, after the
// rescaling by R).  o comes from the problem's own array (formed in FP64 and
// rounded once), not from 1 - alpha: in FP32, 1 - alpha would lose the
// relative precision 6e-8 N / tau where tau << N.
template <typename R, int N>
__global__ void __launch_bounds__(kWienerThreads)
wiener_coef_kernel(const R* coef, const R* omw, R* wcoef, const double* d, size_t entries) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kWienerThreads + threadIdx.x;
  if (idx >= entries) return;
  size_t va = 0, vb = 0;
  entry_voxels<R, N>(idx, va, vb);
  wcoef[idx * 4] = coef[idx * 4];
  wcoef[idx * 4 + 1] = coef[idx * 4 + 1];
  wcoef[idx * 4 + 2] = static_cast<R>(static_cast<double>(omw[idx * 2]) * d[va]);
  wcoef[idx * 4 + 3] = static_cast<R>(static_cast<double>(omw[idx * 2 + 1]) * d[vb]);
}

// Grid-unit P (P / V_cell) and the filter table (A_b = f_b / M, B_b unused).
template <typename R>
__global__ void wiener_table_kernel(const double* pk, double* pkg, R* table, double tau,
                                    double vcell, double m, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double p = pk[b] / vcell;
  pkg[b] = p;
  const double f = p / (p + tau);
  table[2 * b] = static_cast<R>(f / m);
  table[2 * b + 1] = R(0);
}

// y = x * w element by element (y may be x).  With w = 1 / R (0 where
// unobserved) it maps data d to d / R, and a gradient with respect to d / R
// to one with respect to d.
__global__ void scale_kernel(const double* x, const double* w, double* y, size_t n) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    y[i] = x[i] * w[i];
}

// Probe coefficients of the log-determinant estimator: (alpha, beta_z) with
// beta_z = tau R z / N for the probe z = sgn(R) sqrt(N) xi, i.e.
// beta_z = sqrt(tau o) xi with o = tau R^2 / N = 1 - alpha.  xi = +-1
// of voxel v comes from Philox counter (v div 4, probe, kPhaseProbe, chain),
// word v mod 4, top bit set -> -1.
template <typename R, int N>
__global__ void __launch_bounds__(kWienerThreads)
probe_coef_kernel(const R* coef, const R* omw, R* wcoef, double tau, uint32_t probe,
                  uint32_t chain, uint32_t k0, uint32_t k1, size_t entries) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kWienerThreads + threadIdx.x;
  if (idx >= entries) return;
  size_t va = 0, vb = 0;
  entry_voxels<R, N>(idx, va, vb);
  auto sign = [&](size_t v) {
    const Words4 w = philox4x32_10(static_cast<uint32_t>(v >> 2), probe, kPhaseProbe, chain, k0, k1);
    const uint32_t x = (v & 3) == 0 ? w.x0 : (v & 3) == 1 ? w.x1 : (v & 3) == 2 ? w.x2 : w.x3;
    return (x >> 31) ? -1.0 : 1.0;
  };
  wcoef[idx * 4] = coef[idx * 4];
  wcoef[idx * 4 + 1] = coef[idx * 4 + 1];
  wcoef[idx * 4 + 2] = static_cast<R>(sqrt(tau * static_cast<double>(omw[idx * 2])) * sign(va));
  wcoef[idx * 4 + 3] = static_cast<R>(sqrt(tau * static_cast<double>(omw[idx * 2 + 1])) * sign(vb));
}

// out_b += scale (G1_b - f_b G0_b) / (tau^2 V_cell), f_b = P_b / (P_b + tau):
// one probe's estimate of tr(A^-1 R S_b R) per unit of physical P_b, from the
// bin sums G1 = (1/M) sum Re(conj(t^_K) b^) and G0 = the same with t_{K-1}
// (b^ the transform of beta_z; s^_K = f t^_{K-1}).
__global__ void logdet_combine_kernel(const double* g1, const double* g0, const double* pkg,
                                      double tau, double vcell, double scale, int nb, double* out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double f = pkg[b] / (pkg[b] + tau);
  out[b] += scale * (g1[b] - f * g0[b]) / (tau * tau * vcell);
}

template <typename T>
__global__ void fill_zero_kernel(T* p, size_t n) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

// Fixed-order block sum of kWienerThreads doubles in LDS; returns it on lane 0.
__device__ __forceinline__ double block_sum(double* red, double x) {
  const int tid = threadIdx.x;
  red[tid] = x;
  __syncthreads();
  for (int h = kWienerThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  return red[0];
}

// Per-block partial sums of chi2 = sum_i w_i d_i (d_i - s_i), w = o / tau =
// 1 / N (0 where unobserved); optionally s_out = s (FP64, [ix][iy][iz]).  s
// is the iterate in [ix][iy][iz] order (the z-pass state read-out).
template <typename R, int N>
__global__ void __launch_bounds__(kWienerThreads)
wiener_chi2_kernel(const R* omw, const double* d, const R* s, double tau, double* partial,
                   double* s_out, size_t entries) {
  __shared__ double red[kWienerThreads];
  const size_t idx = static_cast<size_t>(blockIdx.x) * kWienerThreads + threadIdx.x;
  double x = 0.0;
  if (idx < entries) {
    size_t va = 0, vb = 0;
    entry_voxels<R, N>(idx, va, vb);
    const double wa = static_cast<double>(omw[idx * 2]) / tau;
    const double wb = static_cast<double>(omw[idx * 2 + 1]) / tau;
    const double sa = s[va], sb = s[vb];
    if (wa > 0.0) x += wa * d[va] * (d[va] - sa);
    if (wb > 0.0) x += wb * d[vb] * (d[vb] - sb);
    if (s_out) {
      s_out[va] = sa;
      s_out[vb] = sb;
    }
  }
  const double t = block_sum(red, x);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// out[0] = sum of n partials in a fixed order (one workgroup).
__global__ void __launch_bounds__(kWienerThreads)
sum_partials_kernel(const double* partial, int n, double* out) {
  __shared__ double red[kWienerThreads];
  double x = 0.0;
  for (int i = threadIdx.x; i < n; i += kWienerThreads) x += partial[i];
  const double t = block_sum(red, x);
  if (threadIdx.x == 0) out[0] = t;
}

// d chi2 / d d_i = w_i (2 d_i - s_K,i) + o_i sum_k r_k,i (o = 1 - alpha), where
// r_k is the adjoint field; zero on unobserved voxels.  The direct term is
// written once s_K is known, the adjoint sum (acc, z-pass order) added last.
template <typename R, int N>
__global__ void __launch_bounds__(kWienerThreads)
wiener_grad_direct_kernel(const R* omw, const double* d, const R* s, double tau, double* grad_d,
                          size_t entries) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kWienerThreads + threadIdx.x;
  if (idx >= entries) return;
  size_t va = 0, vb = 0;
  entry_voxels<R, N>(idx, va, vb);
  const double oa = static_cast<double>(omw[idx * 2]);
  const double ob = static_cast<double>(omw[idx * 2 + 1]);
  grad_d[va] = oa / tau * (2.0 * d[va] - s[va]);
  grad_d[vb] = ob / tau * (2.0 * d[vb] - s[vb]);
}

template <typename R, int N>
__global__ void __launch_bounds__(kWienerThreads)
wiener_grad_adjoint_kernel(const R* omw, const R* acc, double* grad_d, size_t entries) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kWienerThreads + threadIdx.x;
  if (idx >= entries) return;
  size_t va = 0, vb = 0;
  entry_voxels<R, N>(idx, va, vb);
  grad_d[va] += static_cast<double>(omw[idx * 2]) * static_cast<double>(acc[idx * 2]);
  grad_d[vb] += static_cast<double>(omw[idx * 2 + 1]) * static_cast<double>(acc[idx * 2 + 1]);
}

// d chi2 / d P_b (physical units) = d chi2 / d f_b * tau / (P_b + tau)^2 / V_cell.
__global__ void wiener_grad_pk_kernel(const double* gacc, const double* pkg, double tau,
                                      double vcell, int nb, double* grad_pk) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double den = pkg[b] + tau;
  grad_pk[b] = gacc[b] * tau / (den * den) / vcell;
}

// ---------------------------------------------------------------- diagnostics
// Posterior mean and variance (population form, M2 / K) of a chain's recorded
// samples, from the z-pass-order Welford sums to [ix][iy][iz].
template <typename R, int N>
__global__ void __launch_bounds__(kWienerThreads)
moments_kernel(const double* mom, double count, double* mean_out, double* var_out, size_t entries) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kWienerThreads + threadIdx.x;
  if (idx >= entries) return;
  size_t va = 0, vb = 0;
  entry_voxels<R, N>(idx, va, vb);
  const double* m2 = mom + 2 * entries;
  mean_out[va] = mom[idx * 2];
  mean_out[vb] = mom[idx * 2 + 1];
  var_out[va] = m2[idx * 2] / count;
  var_out[vb] = m2[idx * 2 + 1] / count;
}

// Autocorrelation of a recorded chain (Sec. 5.1, Eq. CORR_COEFF), one
// workgroup per bin b of trace [t][nb]: with mean mu and variance var over the
// t samples, acf[n][b] = sum_{i < t-n} (x_i - mu)(x_{i+n} - mu) / ((t - n) var)
// for n <= max_lag, and nc[b] = the first n with acf < 0.1 (-1 if none).  All
// sums run in a fixed order.
__global__ void __launch_bounds__(kWienerThreads)
acf_kernel(const double* trace, int t, int nb, int max_lag, double* acf, int32_t* nc) {
  __shared__ double red[kWienerThreads];
  const int b = blockIdx.x, tid = threadIdx.x;
  double x = 0.0;
  for (int i = tid; i < t; i += kWienerThreads) x += trace[static_cast<size_t>(i) * nb + b];
  const double mu = block_sum(red, x) / t;
  __syncthreads();
  x = 0.0;
  for (int i = tid; i < t; i += kWienerThreads) {
    const double dv = trace[static_cast<size_t>(i) * nb + b] - mu;
    x += dv * dv;
  }
  const double var = block_sum(red, x) / t;
  for (int n = tid; n <= max_lag; n += kWienerThreads) {
    double sum = 0.0;
    for (int i = 0; i + n < t; ++i)
      sum += (trace[static_cast<size_t>(i) * nb + b] - mu) *
             (trace[static_cast<size_t>(i + n) * nb + b] - mu);
    acf[static_cast<size_t>(n) * nb + b] = sum / ((t - n) * var);
  }
  __syncthreads();
  if (tid == 0) {
    int first = -1;
    for (int n = 0; n <= max_lag && first < 0; ++n)
      if (acf[static_cast<size_t>(n) * nb + b] < 0.1) first = n;
    nc[b] = first;
  }
}

}  // namespace mf
