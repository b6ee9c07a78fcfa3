// Kernels of one Gibbs sweep of the messenger-field sampler (gfx950).
//
// Device layout of a chain (R = float or double):
//   alpha, beta  [ix][iy][iz]  R      messenger coefficients (see z-pass)
//   spec         [kz][ix][iy]  cx<R>  half-complex working field, kz <= N/2
//   table        [b][2]        R      per-bin (A_b, B_b) of the signal draw
//   pk           [b]           double P_b in grid units (variance per voxel)
//   partials     [b][wg]       double per-workgroup shell sums of the x-pass
// Between sweeps `spec` holds s transformed along z only, Y = DFT_z(s) / N
// (a real-to-half-complex DFT of each z pencil), so keeping the state costs
// no extra pass.
//
// One sweep = five launches:
//   z-pass  : inverse z-DFT (-> s), messenger draw t, forward z-DFT of t
//   y-pass  : forward y-DFT
//   x-pass  : forward x-DFT (-> t^), signal draw s^, shell sums, inverse x-DFT
//   pk-draw : per-bin reduction of the shell sums and inverse-gamma draw
//   y-pass  : inverse y-DFT
// The signal draw folds the inverse transform's 1/M into s^, so the stored
// field is s^/M and every DFT is unnormalised.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.hpp"
#include "philox.hpp"

namespace mf {

template <typename R>
struct SweepArgs {
  cx<R>* spec;            // chain c at spec + c * spec_stride
  const R* alpha;         // chain c at alpha + c * m
  const R* beta;
  R* staging;             // M reals, shared by all chains (state in/out)
  const double* tau;      // [chain]
  double* pk;             // [chain][nb]
  R* table;               // [chain][nb][2]
  double* partials;       // [chain][nb][n_wg_x]
  const int32_t* qthr;    // [nb] smallest q of every bin
  const double* counts;   // [nb] full-grid modes per bin
  const cx<R>* tw;        // [N] exp(-2 pi i j / N)
  uint32_t* status;       // [chain] bit 0: non-finite P or shell sum
  size_t spec_stride;
  size_t m;
  int32_t nb;
  int32_t n_wg_x;
  int32_t staging_chain;  // chain whose state the staging buffer exchanges
  int32_t sample_pk;
  uint32_t sweep;
  uint32_t chain0;
  uint32_t key0, key1;
};

enum ZMode : int { kZSweep = 0, kZSetState = 1, kZGetState = 2 };

// ---------------------------------------------------------------- tiles
template <typename R, int N>
struct ZTile {
  static constexpr int EPT = 16;                                   // elements / thread
  static constexpr int P = N >= 32 ? (sizeof(R) == 4 ? 32 : 16) : N;  // z pencils / wg
  static constexpr int NPAIR = P / 2;                              // complex pencils
  static constexpr int PSTR = N + 1;
  static constexpr int NT = NPAIR * N / EPT;
};

template <typename R, int N>
struct YTile {
  static constexpr int EPT = 16;
  static constexpr int CAP = sizeof(R) == 4 ? 4096 : 2048;          // elements / wg
  static constexpr int NPEN = CAP / N < 1 ? 1 : (CAP / N > N ? N : CAP / N);
  static constexpr int PSTR = N + 1;
  static constexpr int NT = NPEN * N / EPT;
};

template <typename R, int N>
struct XTile {
  static constexpr int EPT = 16;
  static constexpr int CAP = sizeof(R) == 4 ? 8192 : 4096;
  static constexpr int P = CAP / N > N ? N : CAP / N;              // x pencils (columns)
  static constexpr int PSTR = N + 1;
  static constexpr int NT = P * N / EPT;
  static constexpr int K = N < 16 ? N : 16;                         // rows per chunk
  static constexpr int NWAVES = (NT + 63) / 64;
};

// ---------------------------------------------------------------- helpers
template <typename R>
__device__ __forceinline__ void load_twiddles(cx<R>* dst, const cx<R>* tw, int n, int nt) {
  for (int i = threadIdx.x; i < n; i += nt) dst[i] = tw[i];
}

__device__ __forceinline__ void ld2(const cx<float>* p, cx<float>& a, cx<float>& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = cx<float>{v.x, v.y};
  b = cx<float>{v.z, v.w};
}
__device__ __forceinline__ void ld2(const cx<double>* p, cx<double>& a, cx<double>& b) {
  const double2 v0 = reinterpret_cast<const double2*>(p)[0];
  const double2 v1 = reinterpret_cast<const double2*>(p)[1];
  a = cx<double>{v0.x, v0.y};
  b = cx<double>{v1.x, v1.y};
}
__device__ __forceinline__ void st2(cx<float>* p, cx<float> a, cx<float> b) {
  *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void st2(cx<double>* p, cx<double> a, cx<double> b) {
  reinterpret_cast<double2*>(p)[0] = make_double2(a.x, a.y);
  reinterpret_cast<double2*>(p)[1] = make_double2(b.x, b.y);
}

__device__ __forceinline__ void ld4(const float* p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&v)[4]) {
  const double2 t0 = reinterpret_cast<const double2*>(p)[0];
  const double2 t1 = reinterpret_cast<const double2*>(p)[1];
  v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
}
__device__ __forceinline__ void st4(float* p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(double* p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2*>(p)[1] = make_double2(v[2], v[3]);
}

// Four unit normals of the messenger draw of voxels (ix, iy, 4g .. 4g+3).
template <typename R>
__device__ __forceinline__ void messenger_normals(uint32_t w0, const SweepArgs<R>& a,
                                                  uint32_t chain, R (&g)[4]) {
  const Words4 w = philox4x32_10(w0, a.sweep, kPhaseMessenger, chain, a.key0, a.key1);
  box_muller(w.x0, w.x1, g[0], g[1]);
  box_muller(w.x2, w.x3, g[2], g[3]);
}

// ---------------------------------------------------------------- z-pass
// Workgroup = one ix and P consecutive iy; the z pencils are processed in
// pairs (a, b) = (iy, iy + 1) packed as one complex pencil a + i b.
//   load   : spec[kz][ix][iy..] half spectra A, B -> Z[k] = A_k + i B_k, k < N,
//            with A_{N-k} = conj(A_k) (imaginary parts of kz = 0, N/2 dropped)
//   c2r    : z = inverse DFT(Z); s_a = Re z, s_b = Im z
//   draw   : t = alpha s + beta + sqrt(tau alpha) G   (messenger conditional)
//   r2c    : W = DFT(t_a + i t_b); A'_k = (W_k + conj W_{N-k}) / 2,
//            B'_k = (W_k - conj W_{N-k}) / (2i), k <= N/2 -> spec
// alpha = 1 - tau/N_i, beta = tau d_i / N_i on observed voxels and (1, 0) on
// unobserved ones, i.e. mean tau/N d + (N - tau)/N s and variance
// tau (N - tau)/N, the messenger conditional with T = tau, R in {0, 1}.
template <typename R, int N, int MODE>
__global__ void __launch_bounds__((ZTile<R, N>::NT))
zpass_kernel(SweepArgs<R> a) {
  using T = ZTile<R, N>;
  constexpr int NPAIR = T::NPAIR, PSTR = T::PSTR, NT = T::NT, H = N / 2;
  __shared__ cx<R> lds[NPAIR * PSTR];
  __shared__ cx<R> tw[N];
  const int tid = threadIdx.x;
  const int iy0 = blockIdx.x * T::P;
  const int ix = blockIdx.y;
  const int c = (MODE == kZSweep) ? static_cast<int>(blockIdx.z) : a.staging_chain;
  cx<R>* spec = a.spec + static_cast<size_t>(c) * a.spec_stride;
  load_twiddles(tw, a.tw, N, NT);

  if (MODE != kZSetState) {
    for (int it = tid; it < (H + 1) * NPAIR; it += NT) {
      const int k = it / NPAIR, p = it % NPAIR;
      cx<R> A, B;
      ld2(spec + (static_cast<size_t>(k) * N + ix) * N + iy0 + 2 * p, A, B);
      cx<R>* z = lds + p * PSTR;
      if (k == 0 || k == H) {
        z[k] = cx<R>{A.x, B.x};
      } else {
        z[k] = cx<R>{A.x - B.y, A.y + B.x};
        z[N - k] = cx<R>{A.x + B.y, B.x - A.y};
      }
    }
    __syncthreads();
    lds_fft<R, N, NPAIR, PSTR, NT, true>(lds, tw);
  } else {
    __syncthreads();
  }

  const R tau = static_cast<R>(a.tau[c]);
  const size_t chain_off = static_cast<size_t>(c) * a.m;
  for (int it = tid; it < NPAIR * (N / 4); it += NT) {
    const int g = it % (N / 4), p = it / (N / 4);
    const int iya = iy0 + 2 * p;
    const size_t ra = (static_cast<size_t>(ix) * N + iya) * N + 4 * g;
    cx<R>* z = lds + p * PSTR + 4 * g;
    if (MODE == kZSetState) {
      // the stored z transform carries the 1/N of the inverse z-DFT
      R sa[4], sb[4];
      ld4(a.staging + ra, sa);
      ld4(a.staging + ra + N, sb);
      constexpr R inv_n = R(1) / R(N);
#pragma unroll
      for (int l = 0; l < 4; ++l) z[l] = cx<R>{sa[l] * inv_n, sb[l] * inv_n};
    } else if (MODE == kZGetState) {
      R sa[4], sb[4];
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        sa[l] = z[l].x;
        sb[l] = z[l].y;
      }
      st4(a.staging + ra, sa);
      st4(a.staging + ra + N, sb);
    } else {
      R al[4], bl[4], ab[4], bb[4], ga[4], gb[4];
      ld4(a.alpha + chain_off + ra, al);
      ld4(a.beta + chain_off + ra, bl);
      ld4(a.alpha + chain_off + ra + N, ab);
      ld4(a.beta + chain_off + ra + N, bb);
      const uint32_t chain = a.chain0 + c;
      const uint32_t w0 = static_cast<uint32_t>((ix * N + iya) * (N / 4) + g);
      messenger_normals(w0, a, chain, ga);
      messenger_normals(w0 + N / 4, a, chain, gb);
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const cx<R> s = z[l];
        const R ta = al[l] * s.x + bl[l] + sqrt(tau * al[l]) * ga[l];
        const R tb = ab[l] * s.y + bb[l] + sqrt(tau * ab[l]) * gb[l];
        z[l] = cx<R>{ta, tb};
      }
    }
  }
  if (MODE == kZGetState) return;
  __syncthreads();
  lds_fft<R, N, NPAIR, PSTR, NT, false>(lds, tw);

  for (int it = tid; it < (H + 1) * NPAIR; it += NT) {
    const int k = it / NPAIR, p = it % NPAIR;
    const cx<R>* z = lds + p * PSTR;
    const cx<R> u = z[k];
    const cx<R> w = z[(N - k) & (N - 1)];
    const cx<R> A{R(0.5) * (u.x + w.x), R(0.5) * (u.y - w.y)};
    const cx<R> B{R(0.5) * (u.y + w.y), R(0.5) * (w.x - u.x)};
    st2(spec + (static_cast<size_t>(k) * N + ix) * N + iy0 + 2 * p, A, B);
  }
}

// ---------------------------------------------------------------- y-pass
// Workgroup = NPEN consecutive contiguous y pencils (index kz * N + ix).
template <typename R, int N, bool INV>
__global__ void __launch_bounds__((YTile<R, N>::NT))
ypass_kernel(SweepArgs<R> a) {
  using T = YTile<R, N>;
  constexpr int NPEN = T::NPEN, PSTR = T::PSTR, NT = T::NT, E = NPEN * N;
  __shared__ cx<R> lds[NPEN * PSTR];
  __shared__ cx<R> tw[N];
  const int tid = threadIdx.x;
  cx<R>* base = a.spec + static_cast<size_t>(blockIdx.z) * a.spec_stride +
                static_cast<size_t>(blockIdx.x) * E;
  load_twiddles(tw, a.tw, N, NT);
  for (int it = tid; it < E / 2; it += NT) {
    const int e = 2 * it, pen = e / N, n = e % N;
    cx<R> u, v;
    ld2(base + e, u, v);
    lds[pen * PSTR + n] = u;
    lds[pen * PSTR + n + 1] = v;
  }
  __syncthreads();
  lds_fft<R, N, NPEN, PSTR, NT, INV>(lds, tw);
  for (int it = tid; it < E / 2; it += NT) {
    const int e = 2 * it, pen = e / N, n = e % N;
    st2(base + e, lds[pen * PSTR + n], lds[pen * PSTR + n + 1]);
  }
}

// ---------------------------------------------------------------- x-pass
__device__ __forceinline__ int wavenumber(int i, int n) { return i <= n / 2 ? i : i - n; }

// Bin of q >= 1: the largest b with Q_b <= q (thresholds Q_b in LDS).
__device__ __forceinline__ int bin_of(int q, const int32_t* qthr, int nb, float qscale) {
  int b = static_cast<int>(sqrtf(static_cast<float>(q) * qscale));
  b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
  if (b + 1 < nb && q >= qthr[b + 1]) ++b;
  if (b > 0 && q < qthr[b]) --b;
  return b;
}

// Workgroup = one kz plane and P consecutive iy columns; x pencils are the
// columns.  After the forward x-DFT the tile holds t^ for modes
// (ix, iy, kz).  Each mode is drawn from the signal conditional
//   s^ = f t^ + sqrt(v/2) (G_re + i G_im),  f = P/(P + tau), v = M tau f
// (stored divided by M: s^/M = A_b t^ + B_b (G_re + i G_im) with
// A_b = f/M, B_b = sqrt(tau f / (2M))).  Self-conjugate modes are real with
// the full variance; on the kz = 0 and kz = N/2 planes the member of a
// conjugate pair with the larger ix*N + iy uses its partner's draws
// conjugated; q = 0 gives 0.  Shell sums of w |s^/M|^2 (w = 1 on kz = 0, N/2,
// else 2) go to per-wave LDS histograms (a wave's atomics land in a fixed
// order), then to one partial per workgroup.
template <typename R, int N>
__global__ void __launch_bounds__((XTile<R, N>::NT))
xpass_kernel(SweepArgs<R> a) {
  using T = XTile<R, N>;
  constexpr int P = T::P, PSTR = T::PSTR, NT = T::NT, K = T::K, H = N / 2;
  __shared__ cx<R> lds[P * PSTR];
  __shared__ cx<R> tw[N];
  extern __shared__ double dyn[];      // hist[NWAVES][nb], then table (2 nb R), qthr
  double* hist = dyn;
  R* tab = reinterpret_cast<R*>(hist + T::NWAVES * a.nb);
  int32_t* qthr = reinterpret_cast<int32_t*>(tab + 2 * a.nb);

  const int tid = threadIdx.x;
  const int iy0 = blockIdx.x * P;
  const int kz = blockIdx.y;
  const int c = blockIdx.z;
  cx<R>* spec = a.spec + static_cast<size_t>(c) * a.spec_stride +
                static_cast<size_t>(kz) * N * N;
  const int nb = a.nb;
  load_twiddles(tw, a.tw, N, NT);
  for (int i = tid; i < T::NWAVES * nb; i += NT) hist[i] = 0.0;
  for (int i = tid; i < 2 * nb; i += NT) tab[i] = a.table[static_cast<size_t>(c) * 2 * nb + i];
  for (int i = tid; i < nb; i += NT) qthr[i] = a.qthr[i];
  for (int it = tid; it < N * P; it += NT) {
    const int col = it % P, ix = it / P;
    lds[col * PSTR + ix] = spec[static_cast<size_t>(ix) * N + iy0 + col];
  }
  __syncthreads();
  lds_fft<R, N, P, PSTR, NT, false>(lds, tw);

  const bool herm = (kz == 0 || kz == H);
  const double wgt = herm ? 1.0 : 2.0;
  const float qscale = static_cast<float>(4.0 * nb * nb / (3.0 * N * N));
  const uint32_t chain = a.chain0 + c;
  const int mz2 = kz * kz;
  double* my_hist = hist + (tid / 64) * nb;
  for (int ci = tid; ci < P * (N / K); ci += NT) {
    const int col = ci % P, row0 = (ci / P) * K;
    const int iy = iy0 + col;
    const int my = wavenumber(iy, N);
    const int r2 = my * my + mz2;
    cx<R>* colp = lds + col * PSTR;
    int cur = -1;
    double acc = 0.0;
#pragma unroll 2
    for (int ix = row0; ix < row0 + K; ix += 2) {
      R g[4];
      {
        const uint32_t w0 = static_cast<uint32_t>((kz * N + iy) * H + ix / 2);
        const Words4 w = philox4x32_10(w0, a.sweep, kPhaseSignal, chain, a.key0, a.key1);
        box_muller(w.x0, w.x1, g[0], g[1]);
        box_muller(w.x2, w.x3, g[2], g[3]);
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int x = ix + e;
        const int mx = wavenumber(x, N);
        const int q = mx * mx + r2;
        cx<R> out{R(0), R(0)};
        int b = -1;
        if (q > 0) {
          b = bin_of(q, qthr, nb, qscale);
          const R A = tab[2 * b], B = tab[2 * b + 1];
          const cx<R> t = colp[x];
          R gre = g[2 * e], gim = g[2 * e + 1];
          bool selfconj = false;
          if (herm) {
            const int px = (N - x) & (N - 1), py = (N - iy) & (N - 1);
            const int lin = x * N + iy, plin = px * N + py;
            if (plin == lin) {
              selfconj = true;
            } else if (plin < lin) {
              const uint32_t w0 = static_cast<uint32_t>((kz * N + py) * H + px / 2);
              const Words4 w = philox4x32_10(w0, a.sweep, kPhaseSignal, chain, a.key0, a.key1);
              R h0, h1;
              if (px & 1) box_muller(w.x2, w.x3, h0, h1);
              else box_muller(w.x0, w.x1, h0, h1);
              gre = h0;
              gim = -h1;
            }
          }
          if (selfconj) {
            out = cx<R>{A * t.x + R(1.4142135623730950488) * B * gre, R(0)};
          } else {
            out = cx<R>{A * t.x + B * gre, A * t.y + B * gim};
          }
        }
        colp[x] = out;
        if (b != cur) {
          if (cur >= 0) atomicAdd(my_hist + cur, acc);
          cur = b;
          acc = 0.0;
        }
        if (b >= 0) {
          const double ox = static_cast<double>(out.x), oy = static_cast<double>(out.y);
          acc += wgt * (ox * ox + oy * oy);
        }
      }
    }
    if (cur >= 0) atomicAdd(my_hist + cur, acc);
  }
  __syncthreads();
  lds_fft<R, N, P, PSTR, NT, true>(lds, tw);
  for (int it = tid; it < N * P; it += NT) {
    const int col = it % P, ix = it / P;
    spec[static_cast<size_t>(ix) * N + iy0 + col] = lds[col * PSTR + ix];
  }
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  double* part = a.partials + static_cast<size_t>(c) * a.n_wg_x * nb + wg;
  for (int b = tid; b < nb; b += NT) {
    double s = 0.0;
    for (int w = 0; w < T::NWAVES; ++w) s += hist[w * nb + b];
    part[static_cast<size_t>(b) * a.n_wg_x] = s;
  }
}

// ---------------------------------------------------------------- P(k)
// Per-bin table of the signal draw from P (grid units), in FP64.
template <typename R>
__device__ __forceinline__ void write_table(R* tab, int b, double p, double tau, double m) {
  const double f = p / (p + tau);
  tab[2 * b] = static_cast<R>(f / m);
  tab[2 * b + 1] = static_cast<R>(sqrt(tau * f / (2.0 * m)));
}

// Workgroup = one (bin, chain).  Sums the x-pass partials in a fixed order
// (strided per thread, then a tree), forms sigma_b = M^2 sum w |s^/M|^2, and
// draws P_b = sigma_b / (2 M g), g ~ Gamma(n_b / 2, 1): the inverse-gamma
// conditional of P_b under Jeffreys' prior.  Then refreshes (A_b, B_b).
constexpr int kPkThreads = 256;

template <typename R>
__global__ void __launch_bounds__(kPkThreads) pk_draw_kernel(SweepArgs<R> a) {
  __shared__ double red[kPkThreads];
  const int b = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const double* part = a.partials + (static_cast<size_t>(c) * a.nb + b) * a.n_wg_x;
  double s = 0.0;
  for (int w = tid; w < a.n_wg_x; w += kPkThreads) s += part[w];
  red[tid] = s;
  __syncthreads();
  for (int h = kPkThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid != 0) return;
  const double m = static_cast<double>(a.m);
  const double sigma = red[0] * m * m;
  const double tau = a.tau[c];
  double* pk = a.pk + static_cast<size_t>(c) * a.nb;
  double p = pk[b];
  if (a.sample_pk && a.counts[b] > 0.0) {
    const double g = gamma_mt(0.5 * a.counts[b], static_cast<uint32_t>(b), a.sweep,
                              a.chain0 + c, a.key0, a.key1);
    p = sigma / (2.0 * m * g);
    if (!(g > 0.0) || !isfinite(p) || !isfinite(sigma)) {
      atomicOr(a.status + c, 1u);
      p = pk[b];
    }
    pk[b] = p;
  }
  write_table(a.table + static_cast<size_t>(c) * 2 * a.nb, b, p, tau, m);
}

// Table from the current P of every chain (set-up and state restore).
template <typename R>
__global__ void pk_table_kernel(SweepArgs<R> a) {
  const int c = blockIdx.y;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < a.nb; b += gridDim.x * blockDim.x)
    write_table(a.table + static_cast<size_t>(c) * 2 * a.nb, b,
                a.pk[static_cast<size_t>(c) * a.nb + b], a.tau[c], static_cast<double>(a.m));
}

}  // namespace mf
