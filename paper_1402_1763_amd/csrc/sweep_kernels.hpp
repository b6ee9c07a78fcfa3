// Kernels of one Gibbs sweep of the messenger-field sampler (gfx950).
//
// Device layout of a chain (R = float or double):
//   coef         z-pass order  R      messenger coefficients (alpha, beta)
//   spec         [kz][ix][iy]  cx<R>  half-complex working field, kz <= N/2
//   table        [b][2]        R      per-bin (A_b, B_b) of the signal draw
//   pk           [b]           double P_b in grid units (variance per voxel)
//   partials     [b][wg]       double per-workgroup shell sums of the x-pass
//                                     (a second set for the mixing sweep)
// Between sweeps `spec` holds s transformed along z only, Y = DFT_z(s) / N
// (a real-to-half-complex DFT of each z pencil), so keeping the state costs
// no extra pass.
//
// One Gibbs sweep = four launches:
//   z-pass  : inverse z-DFT (-> s), messenger draw t, forward z-DFT of t
//   y-pass  : forward y-DFT (and, on the split path, 32 <= N <= 256, the
//             first half of the forward x-DFT, see "x split")
//   x-pass  : forward x-DFT (-> t^), signal draw s^, shell sums, inverse x-DFT
//   y-pass  : inverse y-DFT (and the last half of the inverse x-DFT), plus the
//             per-bin reduction of the shell sums and the inverse-gamma draw of
//             P(k) in extra workgroups
// The signal draw folds the inverse transform's 1/M into s^, so the stored
// field is s^/M and every DFT is unnormalised.  The same kernels serve the
// mixing sweep (kXMix, then mix_pk_kernel and xmixinv_kernel between the
// x-pass and the inverse y-pass), the deterministic Wiener iteration and its
// adjoint (kZDet / kZAccum, kXDet / kXAdj, kPkGrad), and the diagnostics
// (Welford moments in the z-pass, P traces in the P workgroups).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.hpp"
#include "philox.hpp"

namespace mf {

template <typename R>
struct SweepArgs {
  cx<R>* spec;            // chain c at spec + c * spec_stride
  const R* coef;          // chain c at coef + c * 2 m (z-pass thread order)
  const uint32_t* tile_obs;  // [chain][z tile] bit e: element e of the tile holds an observed voxel
  int32_t ztiles;         // z-pass tiles per chain
  R* staging;             // M reals, shared by all chains (state in/out)
  const double* tau;      // [chain]
  double* pk;             // [chain][nb]
  R* table;               // [chain][nb][2]
  double* partials;       // [chain][nb][n_wg_x]
  double* partials2;      // [chain][nb][n_wg_x] second sums (mixing sweep)
  double* ratio;          // [chain][nb] mixing sweep: sqrt(S^'_b / S^_b)
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
  uint32_t* ctr;          // [0] next sweep's index, [1] index of the sweep in flight
  uint32_t chain0;
  uint32_t key0, key1;
  // Deterministic messenger iteration (the Wiener filter) and its adjoint:
  R cs, cb;               // z-pass forms t = cs alpha s + cb beta (no draw)
  int32_t cb_over_tau;    // nonzero: cb / tau of the chain replaces cb
  R* acc;                 // z-pass order [entry][2]: adds s before the messenger step
  cx<R>* aux;             // x-pass layout: t^ of one iteration (stored or read)
  double* gacc;           // [chain][nb] accumulated d chi2 / d f_b
  int32_t advance;        // the forward y-pass advances the sweep counter
  int32_t pk_mode;        // P(k) workgroups of the inverse y-pass (PkMode)
  // Diagnostics: sample n (the state after n sweeps) is recorded as sweep n
  // begins, for n = diag_start + j diag_thin, j >= 0.
  double* trace;          // [chain][trace_cap][nb] P_b of sample n, physical units
  double* mom;            // [chain][2][m] Welford mean and M2 of s, z-pass order
  uint32_t diag_start;
  int32_t diag_thin;
  int32_t trace_cap;
  double vcell;
  // InvGamma(prior_a, prior_b) prior on P_b, prior_b in grid units; (0, 0) is
  // Jeffreys' prior
  double prior_a, prior_b;
};

// Index j of sample `sweep` among the recorded ones, or -1.
template <typename R>
__device__ __forceinline__ int recorded(const SweepArgs<R>& a, uint32_t sweep) {
  if (a.diag_thin <= 0 || sweep < a.diag_start) return -1;
  const uint32_t d = sweep - a.diag_start;
  return d % static_cast<uint32_t>(a.diag_thin) == 0 ? static_cast<int>(d / a.diag_thin) : -1;
}

enum ZMode : int { kZSweep = 0, kZSetState = 1, kZGetState = 2, kZDet = 3, kZAccum = 4 };
enum XMode : int { kXSample = 0, kXDet = 1, kXAdj = 2, kXMix = 3 };
enum PkMode : int { kPkDraw = 0, kPkNone = 1, kPkGrad = 2 };

// ---------------------------------------------------------------- tiles
// Largest power of two d <= cap that divides n (at least 1).
__host__ __device__ constexpr int pow2_divisor(int n, int cap) {
  int d = 1;
  while (d * 2 <= cap && n % (d * 2) == 0) d *= 2;
  return d;
}

// Largest divisor d of n with d <= cap (at least 1).
__host__ __device__ constexpr int divisor_below(int n, int cap) {
  int d = 1;
  for (int k = 1; k <= n && k <= cap; ++k)
    if (n % k == 0) d = k;
  return d;
}

// z-pass: IXB consecutive ix and P consecutive iy (NPAIR complex pencils per
// ix), pencil-fastest; pencil pen = ixb * NPAIR + p.  Small grids take several
// ix per workgroup, up to 256 threads and 40 KB of staging LDS.
template <typename R, int N>
struct ZTile {
  static constexpr int EPT = ept<N>();
  static constexpr int P = N >= 32 ? ((sizeof(R) == 4 && N % 32 == 0) ? 32 : 16) : N;
  static constexpr int NPAIR = P / 2;
  static constexpr int IXCAP_T = 256 / (NPAIR * N / EPT);
  static constexpr int IXCAP_L = 40960 / (NPAIR * (N + 1) * 2 * static_cast<int>(sizeof(R)));
  static constexpr int IXB = pow2_divisor(N, IXCAP_T < IXCAP_L ? IXCAP_T : IXCAP_L);
  static constexpr int NPEN = IXB * NPAIR;
  static constexpr int NT = NPEN * N / EPT;
  static constexpr int PSTR = N + 1;
  using TL = Tile<N, NPEN, NT, true, PSTR, 0>;
  static_assert(EPT <= 32, "one observation bit per element");
  // FP64 at N = 256 would take 256 VGPRs and 8 AGPRs (1 wave per SIMD); held
  // to 256 registers (2 waves, no spill) the FP64 sweep runs 8% faster.
  static constexpr int MIN_WAVES = (sizeof(R) == 8 && N == 256) ? 2 : 1;
};

// y-pass (whole-transform path): NPEN consecutive contiguous pencils of one
// kz plane, q-fastest, padded LDS.
template <typename R, int N>
struct YTile {
  static constexpr int EPT = ept<N>();
  static constexpr int CAP = sizeof(R) == 4 ? 4096 : 2048;
  static constexpr int NPEN = divisor_below(N, CAP / N);
  static constexpr int NT = NPEN * N / EPT;
  static constexpr int PADS = ilog2(Radices<N>::r[0]);
  static constexpr int PSTR = N + (N >> PADS);
  using TL = Tile<N, NPEN, NT, false, PSTR, PADS>;
};

// x-pass (whole-transform path): one kz plane, P consecutive iy columns,
// pencil-fastest.
template <typename R, int N>
struct XTile {
  static constexpr int EPT = ept<N>();
  static constexpr int CAP = 4096;
  static constexpr int P = divisor_below(N, CAP / N);
  static constexpr int NT = P * N / EPT;
  static constexpr int PSTR = N + 1;
  static constexpr int NWAVES = (NT + 63) / 64;
  static constexpr int HG = 2;            // histogram copies per wave (by lane % HG)
  static constexpr int NHIST = NWAVES * HG;
  using TL = Tile<N, P, NT, true, PSTR, 0>;
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

// ---------------------------------------------------------------- z-pass
// Messenger coefficients are stored in the z-pass's thread order so that each
// lane's loads are contiguous: entry ((tile * EPT + e) * NT + tid) holds
// (alpha_a, alpha_b, beta_a, beta_b) of the voxels (ix, iya (+1), n) that
// thread tid holds as element e after the inverse z-DFT, where
// tile = (ix0 / IXB) * (N / P) + iy0 / P.  alpha = 1 - tau/N_i,
// beta = tau d_i / N_i on observed voxels and (1, 0) elsewhere.
template <typename R, int N>
__host__ __device__ inline void zpass_coef_voxel(int tile, int e, int tid, int& ix, int& iya,
                                                 int& n) {
  using T = ZTile<R, N>;
  int pen = 0;
  T::TL::template out_pos<false>(tid, e, pen, n);
  ix = (tile / (N / T::P)) * T::IXB + pen / T::NPAIR;
  iya = (tile % (N / T::P)) * T::P + 2 * (pen % T::NPAIR);
}

// Which elements of z-pass tile `tile` of chain c hold an observed voxel:
// bit e covers element e of every lane (at N = 256, the z range
// [16 e, 16 e + 16) of the tile's pencils).  Elements with none skip their
// coefficient loads: alpha = 1 and beta = 0 there exactly.  The mask is the
// same for the whole workgroup.
template <typename R>
__device__ __forceinline__ uint32_t tile_obs_mask(const SweepArgs<R>& a, int c, int tile) {
  if (a.tile_obs == nullptr) return ~0u;
  const uint32_t f = a.tile_obs[static_cast<size_t>(c) * a.ztiles + tile];
  return __builtin_amdgcn_readfirstlane(f);
}

// Workgroup = IXB consecutive ix and P consecutive iy; z pencils (iy, iy + 1)
// are packed as one complex pencil a + i b.
//   load    : Z_k = A_k + i B_k from the half spectra, Hermitian-extended
//             (A_{N-k} = conj A_k; imaginary parts of kz = 0, N/2 dropped),
//             straight into the registers of the first inverse stage
//   c2r     : z = inverse DFT(Z); s_a = Re z, s_b = Im z
//   draw    : t = alpha s + beta + sqrt(tau alpha) G  -- the messenger
//             conditional with T = tau: alpha = 1 - tau R^2/N and
//             beta = tau R d/N on observed voxels, (1, 0) elsewhere
//   r2c     : W = DFT(t_a + i t_b), A'_k = (W_k + conj W_{N-k}) / 2,
//             B'_k = (W_k - conj W_{N-k}) / (2i), k <= N/2 -> spec
// The unit normals of voxel (ix, iy, n) come from Philox counter
// ((ix N + iy) N/4 + n mod N/4, sweep, 0, chain), normal n div (N/4) of the
// call; a thread's elements n = q + (N/R_L) r cover all four normals of a call.
// kZDet replaces the draw by t = cs alpha s + cb beta (the messenger mean for
// cs = cb = 1) and, if acc is set, first adds s to acc; kZAccum only adds s.
// Messenger noise amplitude sqrt(tau alpha).  FP32 takes the hardware square
// root (within 1 ulp); the correctly rounded expansion costs about 16
// instructions per voxel, some 18% of the pass's vector instructions.
__device__ __forceinline__ float noise_amp(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double noise_amp(double x) { return sqrt(x); }

template <typename R, int N, int MODE>
__global__ void __launch_bounds__((ZTile<R, N>::NT), (ZTile<R, N>::MIN_WAVES))
zpass_kernel(SweepArgs<R> a) {
  using T = ZTile<R, N>;
  using TL = typename T::TL;
  constexpr int NPAIR = T::NPAIR, NPEN = T::NPEN, NT = T::NT, EPT = T::EPT, H = N / 2;
  constexpr int RL = radix_at<N, false>(Radices<N>::n - 1);
  constexpr int NSL = N / RL;
  __shared__ cx<R> lds[NPEN * T::PSTR];
  __shared__ cx<R> tw[N];
  const int tid = threadIdx.x;
  const int blk = blockIdx.x;
  const int iy0 = blk * T::P;
  const int ix0 = blockIdx.y * T::IXB;
  const int c = (MODE == kZSweep || MODE == kZDet || MODE == kZAccum)
                    ? static_cast<int>(blockIdx.z) : a.staging_chain;
  cx<R>* spec = a.spec + static_cast<size_t>(c) * a.spec_stride;
  load_twiddles(tw, a.tw, N, NT);
  cx<R> v[EPT];
  const uint32_t sweep = a.ctr[0];
  // Publish this sweep's index to the later passes (the forward y-pass then
  // advances slot 0 for the next sweep): no other z-pass workgroup reads
  // slot 1, and the later passes start after this kernel has finished.
  if (MODE == kZSweep && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
    a.ctr[1] = sweep;

  if (MODE != kZSetState) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int pen = 0, k = 0;
      TL::template in_pos<false>(tid, e, pen, k);
      const int kk = k <= H ? k : N - k;
      cx<R> A, B;
      ld2(spec + (static_cast<size_t>(kk) * N + ix0 + pen / NPAIR) * N + iy0 + 2 * (pen % NPAIR),
          A, B);
      if (k == 0 || k == H) v[e] = cx<R>{A.x, B.x};
      else if (k < H) v[e] = cx<R>{A.x - B.y, A.y + B.x};
      else v[e] = cx<R>{A.x + B.y, B.x - A.y};
    }
    fft_regs<R, N, TL, NT, true, false>(v, lds, tw);
    if (MODE == kZSweep && a.mom != nullptr) {
      const int j = recorded(a, sweep);
      if (j >= 0) {   // Welford update with the (j + 1)-th sample
        const double inv_k = 1.0 / (j + 1.0);
        double* mean = a.mom + static_cast<size_t>(c) * 2 * a.m +
                       static_cast<size_t>(blockIdx.y * (N / T::P) + blk) * EPT * NT * 2;
        double* m2 = mean + a.m;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const size_t i = (static_cast<size_t>(e) * NT + tid) * 2;
          const double x0 = v[e].x, x1 = v[e].y;
          const double u0 = mean[i], u1 = mean[i + 1];
          const double n0 = u0 + (x0 - u0) * inv_k, n1 = u1 + (x1 - u1) * inv_k;
          mean[i] = n0;
          mean[i + 1] = n1;
          m2[i] += (x0 - u0) * (x0 - n0);
          m2[i + 1] += (x1 - u1) * (x1 - n1);
        }
      }
    }
    if (MODE == kZAccum || (MODE == kZDet && a.acc != nullptr)) {
      R* acc = a.acc + static_cast<size_t>(c) * a.m +
               static_cast<size_t>(blockIdx.y * (N / T::P) + blk) * EPT * NT * 2;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        R* q = acc + (static_cast<size_t>(e) * NT + tid) * 2;
        q[0] += v[e].x;
        q[1] += v[e].y;
      }
      if (MODE == kZAccum) return;
    }
    if (MODE == kZGetState) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        int pen = 0, n = 0;
        TL::template out_pos<false>(tid, e, pen, n);
        const size_t ra =
            (static_cast<size_t>(ix0 + pen / NPAIR) * N + iy0 + 2 * (pen % NPAIR)) * N + n;
        a.staging[ra] = v[e].x;
        a.staging[ra + N] = v[e].y;
      }
      return;
    }
  }

  if (MODE == kZSetState) {
    // the stored z transform carries the 1/N of the inverse z-DFT
    constexpr R inv_n = R(1) / R(N);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int pen = 0, n = 0;
      TL::template out_pos<false>(tid, e, pen, n);
      const size_t ra =
          (static_cast<size_t>(ix0 + pen / NPAIR) * N + iy0 + 2 * (pen % NPAIR)) * N + n;
      v[e] = cx<R>{a.staging[ra] * inv_n, a.staging[ra + N] * inv_n};
    }
  } else if (MODE == kZDet) {
    const int tile = blockIdx.y * (N / T::P) + blk;
    const R* coef = a.coef + static_cast<size_t>(c) * 2 * a.m + static_cast<size_t>(tile) * EPT * NT * 4;
    const uint32_t obs = tile_obs_mask(a, c, tile);
    const R cb = a.cb_over_tau ? static_cast<R>(static_cast<double>(a.cb) / a.tau[c]) : a.cb;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      R cf[4] = {R(1), R(1), R(0), R(0)};
      if ((obs >> e) & 1u) ld4(coef + (static_cast<size_t>(e) * NT + tid) * 4, cf);
      const cx<R> s = v[e];
      v[e] = cx<R>{a.cs * cf[0] * s.x + cb * cf[2], a.cs * cf[1] * s.y + cb * cf[3]};
    }
  } else {
    const R tau = static_cast<R>(a.tau[c]);
    const int tile = blockIdx.y * (N / T::P) + blk;
    const R* coef = a.coef + static_cast<size_t>(c) * 2 * a.m + static_cast<size_t>(tile) * EPT * NT * 4;
    const uint32_t obs = tile_obs_mask(a, c, tile);
    const uint32_t chain = a.chain0 + c;
#pragma unroll
    for (int i = 0; i < EPT / RL; ++i) {
      int pen = 0, q = 0;
      TL::split(tid + i * NT, NSL, pen, q);
      const int ix = ix0 + pen / NPAIR, iya = iy0 + 2 * (pen % NPAIR);
      const uint32_t wa = static_cast<uint32_t>((ix * N + iya) * (N / 4) + q);
#pragma unroll
      for (int cq = 0; cq < RL / 4; ++cq) {
        // three-input XORs in Philox at 256^3 FP32 only (0.4 us there);
        // elsewhere the extra registers cross an occupancy step
        constexpr bool kXor3 = sizeof(R) == 4 && N == 256;
        R ga[4], gb[4];
        {
          const Words4 w = philox4x32_10<kXor3>(wa + NSL * cq, sweep, kPhaseMessenger, chain,
                                                a.key0, a.key1);
          box_muller(w.x0, w.x1, ga[0], ga[1]);
          box_muller(w.x2, w.x3, ga[2], ga[3]);
        }
        {
          const Words4 w = philox4x32_10<kXor3>(wa + N / 4 + NSL * cq, sweep, kPhaseMessenger,
                                                chain, a.key0, a.key1);
          box_muller(w.x0, w.x1, gb[0], gb[1]);
          box_muller(w.x2, w.x3, gb[2], gb[3]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = i * RL + cq + j * (RL / 4);
          R cf[4] = {R(1), R(1), R(0), R(0)};
          if ((obs >> e) & 1u) ld4(coef + (static_cast<size_t>(e) * NT + tid) * 4, cf);
          const cx<R> s = v[e];
          const R ta = cf[0] * s.x + cf[2] + noise_amp(tau * cf[0]) * ga[j];
          const R tb = cf[1] * s.y + cf[3] + noise_amp(tau * cf[1]) * gb[j];
          v[e] = cx<R>{ta, tb};
        }
      }
    }
  }
  __syncthreads();   // every lane is done with the inverse transform's LDS reads
  fft_regs<R, N, TL, NT, false, true>(v, lds, tw);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    int p = 0, k = 0;
    TL::template out_pos<true>(tid, e, p, k);
    lds[TL::lidx(p, k)] = v[e];
  }
  __syncthreads();
  for (int it = tid; it < (H + 1) * NPEN; it += NT) {
    const int k = it / NPEN, pen = it % NPEN;
    const cx<R> u = lds[TL::lidx(pen, k)];
    const cx<R> w = lds[TL::lidx(pen, (N - k) % N)];
    const cx<R> A{R(0.5) * (u.x + w.x), R(0.5) * (u.y - w.y)};
    const cx<R> B{R(0.5) * (u.y + w.y), R(0.5) * (w.x - u.x)};
    st2(spec + (static_cast<size_t>(k) * N + ix0 + pen / NPAIR) * N + iy0 + 2 * (pen % NPAIR), A, B);
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

// Sum of n per-workgroup partials in a fixed order by one workgroup of NTH
// threads: strided per thread, then a tree in `red` (NTH doubles) folded onto
// the largest power of two <= NTH.  The result is red[0] (all threads).
template <int NTH>
__device__ __forceinline__ double sum_partials(const double* part, int n, double* red) {
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int w = tid; w < n; w += NTH) s += part[w];
  red[tid] = s;
  __syncthreads();
  constexpr int P2 = 1 << ilog2(NTH);
  if (P2 < NTH) {
    if (tid < NTH - P2) red[tid] += red[tid + P2];
    __syncthreads();
  }
  for (int h = P2 / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  return red[0];
}

// P(k) step of bin b of chain c by one workgroup of NTH threads: sums the
// x-pass partials in a fixed order (sum_partials), forms
// sigma_b = M^2 sum w |s^/M|^2 and draws P_b = (sigma_b + 2 M b0) / (2 M g),
// g ~ Gamma(n_b / 2 + a0, 1) -- the inverse-gamma conditional of P_b under
// the InvGamma(a0, b0) prior, Jeffreys' prior at a0 = b0 = 0 -- then refreshes
// (A_b, B_b).  With pk_mode == kPkGrad the workgroup instead adds
// sum_wg partials / M to gacc[b] (the Wiener adjoint's d chi2 / d f_b);
// kPkNone does nothing.
template <typename R, int NTH>
__device__ __forceinline__ void pk_draw_block(const SweepArgs<R>& a, int b, int c, double* red) {
  if (a.pk_mode == kPkNone) return;
  const int tid = threadIdx.x;
  sum_partials<NTH>(a.partials + (static_cast<size_t>(c) * a.nb + b) * a.n_wg_x, a.n_wg_x, red);
  if (tid == 0 && a.pk_mode == kPkGrad) {
    a.gacc[static_cast<size_t>(c) * a.nb + b] += red[0] / static_cast<double>(a.m);
  } else if (tid == 0) {
    const double m = static_cast<double>(a.m);
    const double sigma = red[0] * m * m;
    const double tau = a.tau[c];
    double* pk = a.pk + static_cast<size_t>(c) * a.nb;
    double p = pk[b];
    if (a.trace != nullptr) {
      const int j = recorded(a, a.ctr[1]);
      if (j >= 0 && j < a.trace_cap)
        a.trace[(static_cast<size_t>(c) * a.trace_cap + j) * a.nb + b] = p * a.vcell;
    }
    if (a.sample_pk && a.counts[b] > 0.0) {
      const double g = gamma_mt(0.5 * a.counts[b] + a.prior_a, static_cast<uint32_t>(b), a.ctr[1],
                                a.chain0 + c, a.key0, a.key1);
      p = (sigma + 2.0 * m * a.prior_b) / (2.0 * m * g);
      if (!(g > 0.0) || !isfinite(p) || !isfinite(sigma)) {
        atomicOr(a.status + c, 1u);
        p = pk[b];
      }
      pk[b] = p;
    }
    write_table(a.table + static_cast<size_t>(c) * 2 * a.nb, b, p, tau, m);
  }
}

// The sweep counter has two slots so that no pass needs a grid-wide barrier:
// the z-pass reads slot 0 and copies it to slot 1, the forward y-pass (which
// reads neither) sets slot 0 to slot 1 + 1, and the x-pass and the P draw read
// slot 1.  Kernel boundaries on the stream order every write before the reads
// that follow it.
template <typename R>
__device__ __forceinline__ void advance_sweep(const SweepArgs<R>& a) {
  if (a.advance && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
    a.ctr[0] = a.ctr[1] + 1u;
}

// Truncated normal N(mean, sd^2) restricted to (0, inf), drawn exactly with
// the words of counter (b 2^16 + j, sweep, kPhaseMix, chain), attempt j.
// a = -mean/sd is the standardised bound; for a <= 0.5 the proposal is the
// cosine normal of (x0, x1), accepted when z > a; otherwise Robert's
// exponential proposal z = a - ln(U23(x0)) / r, r = (a + sqrt(a^2 + 4)) / 2,
// accepted when U23(x1) <= exp(-(z - r)^2 / 2).  u_mh = U23(x3) of attempt 0
// is the Metropolis-Hastings uniform.  Returns false after kMixAttempts
// attempts without a proposal.
constexpr int kMixAttempts = 64;

__device__ inline bool truncated_normal(double mean, double sd, uint32_t b, uint32_t sweep,
                                        uint32_t chain, uint32_t k0, uint32_t k1, double& u_new,
                                        double& u_mh) {
  const double a = -mean / sd;
  const double r = 0.5 * (a + sqrt(a * a + 4.0));
  for (int j = 0; j < kMixAttempts; ++j) {
    const Words4 w = philox4x32_10(b * 65536u + j, sweep, kPhaseMix, chain, k0, k1);
    if (j == 0) u_mh = u23<double>(w.x3);
    double z;
    bool ok;
    if (a <= 0.5) {
      double unused;
      box_muller(w.x0, w.x1, z, unused);
      ok = z > a;
    } else {
      z = a - log(u23<double>(w.x0)) / r;
      ok = u23<double>(w.x1) <= exp(-0.5 * (z - r) * (z - r));
    }
    if (ok) {
      u_new = mean + sd * z;
      return true;
    }
  }
  return false;
}

// Metropolis-Hastings move of S^_b = M P_b in the mixing sweep (Sec. 3.3,
// shell form), one workgroup per (bin, chain).  With y = s^/M drawn at the
// current P by the x-pass, H1 = sum w |y|^2 and H2 = sum w Re(conj(y) t^)
// (partials and partials2) give, for x^ = s^ / sqrt(S^),
//   X = sum |x^|^2 = M H1 / P,   R = sum Re(conj(x^) t^) = M H2 / sqrt(S^).
// U = sqrt(S^) has conditional density ~ U^-1 N(U; R/X, T^/X), T^ = M tau,
// under Jeffreys' prior, and ~ U^-(2 a0 + 1) exp(-M b0 / U^2) N(U; R/X, T^/X)
// under the InvGamma(a0, b0) prior; the proposal U' ~ N(R/X, T^/X) truncated
// to U' > 0 is accepted with probability min(1, U/U'), respectively
// min(1, (U/U')^(2 a0 + 1) exp(M b0 (1/U^2 - 1/U'^2))) (in logarithms).  Writes the new P, its table and the factor
// ratio = U'/U (1 if rejected) by which the x-pass output is rescaled.
template <typename R>
__global__ void __launch_bounds__(256)
mix_pk_kernel(SweepArgs<R> a) {
  __shared__ double red[256];
  const int b = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
  const size_t off = (static_cast<size_t>(c) * a.nb + b) * a.n_wg_x;
  const double h1 = sum_partials<256>(a.partials + off, a.n_wg_x, red);
  __syncthreads();
  const double h2 = sum_partials<256>(a.partials2 + off, a.n_wg_x, red);
  if (tid != 0) return;
  const double m = static_cast<double>(a.m), tau = a.tau[c];
  const uint32_t sweep = a.ctr[1];
  double* pk = a.pk + static_cast<size_t>(c) * a.nb;
  const double p = pk[b];
  if (a.trace != nullptr) {
    const int j = recorded(a, sweep);
    if (j >= 0 && j < a.trace_cap)
      a.trace[(static_cast<size_t>(c) * a.trace_cap + j) * a.nb + b] = p * a.vcell;
  }
  double ratio = 1.0, p_new = p;
  if (a.counts[b] > 0.0 && h1 > 0.0 && p > 0.0) {
    const double u = sqrt(m * p);
    const double xx = m * h1 / p, xt = m * h2 / u;
    double u_new = 0.0, u_mh = 1.0;
    bool ok = truncated_normal(xt / xx, sqrt(m * tau / xx), static_cast<uint32_t>(b), sweep,
                               a.chain0 + c, a.key0, a.key1, u_new, u_mh);
    if (ok) {
      if (a.prior_a == 0.0 && a.prior_b == 0.0) {
        ok = u_mh <= u / u_new;
      } else {
        const double lr = (2.0 * a.prior_a + 1.0) * log(u / u_new) +
                          m * a.prior_b * (1.0 / (u * u) - 1.0 / (u_new * u_new));
        ok = log(u_mh) <= lr;
      }
    }
    if (ok) {
      p_new = u_new * u_new / m;
      ratio = u_new / u;
    }
    if (!isfinite(p_new) || !(p_new > 0.0) || !isfinite(h1) || !isfinite(h2)) {
      atomicOr(a.status + c, 1u);
      p_new = p;
      ratio = 1.0;
    }
  }
  pk[b] = p_new;
  a.ratio[static_cast<size_t>(c) * a.nb + b] = ratio;
  write_table(a.table + static_cast<size_t>(c) * 2 * a.nb, b, p_new, tau, m);
}

// Table from the current P of every chain (set-up and state restore).
template <typename R>
__global__ void pk_table_kernel(SweepArgs<R> a) {
  const int c = blockIdx.y;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < a.nb; b += gridDim.x * blockDim.x)
    write_table(a.table + static_cast<size_t>(c) * 2 * a.nb, b,
                a.pk[static_cast<size_t>(c) * a.nb + b], a.tau[c], static_cast<double>(a.m));
}

// ---------------------------------------------------------------- y-pass
// Workgroup = NPEN consecutive contiguous y pencils (index kz * N + ix).  The
// inverse pass also carries the sweep's P(k) step: its first nb workgroups of
// every chain draw one bin each (the x-pass partials are complete when it
// starts, and the new P is first read by the next sweep's x-pass).
template <typename R, int N, bool INV>
__global__ void __launch_bounds__((YTile<R, N>::NT))
ypass_kernel(SweepArgs<R> a) {
  using T = YTile<R, N>;
  using TL = typename T::TL;
  constexpr int NT = T::NT, EPT = T::EPT;
  __shared__ cx<R> lds[T::NPEN * T::PSTR];
  __shared__ cx<R> tw[N];
  static_assert(T::NPEN * T::PSTR * sizeof(cx<R>) >= NT * sizeof(double), "reduction space");
  int blk = blockIdx.x;
  if (INV) {
    if (blk < a.nb) {
      pk_draw_block<R, NT>(a, blk, blockIdx.z, reinterpret_cast<double*>(lds));
      return;
    }
    blk -= a.nb;
  } else {
    advance_sweep(a);
  }
  const int tid = threadIdx.x;
  cx<R>* base = a.spec + static_cast<size_t>(blockIdx.z) * a.spec_stride +
                static_cast<size_t>(blk) * T::NPEN * N;
  load_twiddles(tw, a.tw, N, NT);
  cx<R> v[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    int pen = 0, n = 0;
    TL::template in_pos<false>(tid, e, pen, n);
    v[e] = base[pen * N + n];
  }
  fft_regs<R, N, TL, NT, INV, false>(v, lds, tw);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    int pen = 0, n = 0;
    TL::template out_pos<false>(tid, e, pen, n);
    base[pen * N + n] = v[e];
  }
}

// ---------------------------------------------------------------- x split
// For 32 <= N <= 256 the x transform is split in two (N = 16 NA, ix = q + 16 r
// with q < 16, r < NA; k = k1 + NA k2):
//   stage A, in the y-passes:  Y[q][k1] = W_N^{q k1} sum_r x[q + 16 r] W_NA^{r k1}
//   stage B, in the x-pass:    X[k1 + NA k2] = sum_q Y[q][k1] W_16^{q k2}
// Between them spec holds Y[q][k1] in row q + 16 k1 of each kz plane (the
// rows the forward y-pass workgroup of q read, so every pass stays in place).
// The x-pass then transforms 16 consecutive rows per thread entirely in
// registers, and the y-passes, which have arithmetic to spare, absorb the
// twiddles and the other half of the x transform.
template <int N>
__host__ __device__ constexpr bool split_x() { return N >= 32 && N <= 256; }

// Forward y-pass with x stage A (INV = false), or inverse x stage A with the
// inverse y-pass (INV = true, plus the P(k) step in the first nb workgroups).
// Workgroup = G units (kz, q), q = q0 .. q0 + G - 1: each the NA y pencils of
// rows ix = q + 16 r.  Variant V (searched by the autotuner) takes G0 / 2^V
// units, G0 the rule below.
template <typename R, int N, int V = 0>
struct YSTile {
  static constexpr int NA = N >= 32 ? N / 16 : 2;   // only meaningful when split_x<N>()
  static constexpr int EPT = ept<N>();
  static constexpr int TPU = NA * N / EPT;           // threads per (kz, q) unit
  static constexpr int COLS = EPT / NA;    // columns per thread in the x-stage layout
  static constexpr int PADS = pow2<Radices<N>::r[0]>() ? ilog2(Radices<N>::r[0]) : 2;
  static constexpr int PSTR = N + (N >> PADS);
  // units per workgroup: up to 256 threads and 48 KB of LDS
  static constexpr int GCAP_T = 256 / TPU;
  static constexpr int GCAP_L = 49152 / (NA * PSTR * 2 * static_cast<int>(sizeof(R)));
  static constexpr int G0 = pow2_divisor(16, GCAP_T < GCAP_L ? GCAP_T : GCAP_L);
  static constexpr int G = (G0 >> V) > 0 ? (G0 >> V) : 1;
  static constexpr int NT = G * TPU;
  using TL = Tile<N, G * NA, NT, false, PSTR, PADS>;
};

// RV runs the y transform's radix stages in reversed order (e.g. 4 x 4 x 6
// instead of 6 x 4 x 4 at 96): a choice of the radix schedule that changes
// no stored layout, since the transform's output and input pass through LDS
// in natural order.
template <typename R, int N, bool INV, int V = 0, bool RV = false>
__global__ void __launch_bounds__((YSTile<R, N, V>::NT))
ysplit_kernel(SweepArgs<R> a) {
  using T = YSTile<R, N, V>;
  using TL = typename T::TL;
  constexpr int NA = T::NA, NT = T::NT, EPT = T::EPT, COLS = T::COLS, G = T::G, TPU = T::TPU;
  __shared__ cx<R> lds[G * NA * T::PSTR];
  __shared__ cx<R> tw[N];
  static_assert(G * NA * T::PSTR * sizeof(cx<R>) >= NT * sizeof(double), "reduction space");
  int blk = blockIdx.x;
  if (INV) {
    if (blk < a.nb) {
      pk_draw_block<R, NT>(a, blk, blockIdx.z, reinterpret_cast<double*>(lds));
      return;
    }
    blk -= a.nb;
  } else {
    advance_sweep(a);
  }
  const int tid = threadIdx.x;
  const int kz = blk / (16 / G), q0 = (blk % (16 / G)) * G;
  const int ug = tid / TPU, ut = tid % TPU;   // this thread's unit and rank in it (stage A)
  const int q = q0 + ug;
  cx<R>* plane = a.spec + static_cast<size_t>(blockIdx.z) * a.spec_stride +
                 static_cast<size_t>(kz) * N * N;
  load_twiddles(tw, a.tw, N, NT);
  cx<R> v[EPT];
  // pencil pen of the y transform = unit pen / NA, row q0 + pen / NA + 16 (pen % NA)
  auto row_of = [&](int pen) { return q0 + pen / NA + 16 * (pen % NA); };
  if (!INV) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int pen = 0, n = 0;
      TL::template in_pos<RV>(tid, e, pen, n);
      v[e] = plane[static_cast<size_t>(row_of(pen)) * N + n];
    }
    fft_regs<R, N, TL, NT, false, RV>(v, lds, tw);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int pen = 0, n = 0;
      TL::template out_pos<RV>(tid, e, pen, n);
      lds[TL::lidx(pen, n)] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
      const int iy = ut + j * TPU;
      cx<R>* u = v + j * NA;
#pragma unroll
      for (int r = 0; r < NA; ++r) u[r] = lds[TL::lidx(ug * NA + r, iy)];
      dft<R, NA, false>(u);
#pragma unroll
      for (int k1 = 0; k1 < NA; ++k1) {
        const cx<R> w = k1 ? cmul(u[k1], tw[q * k1]) : u[k1];
        plane[static_cast<size_t>(q + 16 * k1) * N + iy] = w;
      }
    }
  } else {
    __syncthreads();   // twiddles in LDS
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
      const int iy = ut + j * TPU;
      cx<R>* u = v + j * NA;
#pragma unroll
      for (int k1 = 0; k1 < NA; ++k1) {
        const cx<R> w = plane[static_cast<size_t>(q + 16 * k1) * N + iy];
        u[k1] = k1 ? cmulc(w, tw[q * k1]) : w;
      }
      dft<R, NA, true>(u);
    }
#pragma unroll
    for (int j = 0; j < COLS; ++j) {
#pragma unroll
      for (int r = 0; r < NA; ++r) lds[TL::lidx(ug * NA + r, ut + j * TPU)] = v[j * NA + r];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int pen = 0, n = 0;
      TL::template in_pos<RV>(tid, e, pen, n);
      v[e] = lds[TL::lidx(pen, n)];
    }
    __syncthreads();   // the transform below rewrites the buffer
    fft_regs<R, N, TL, NT, true, RV>(v, lds, tw);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      int pen = 0, n = 0;
      TL::template out_pos<RV>(tid, e, pen, n);
      plane[static_cast<size_t>(row_of(pen)) * N + n] = v[e];
    }
  }
}

// ---------------------------------------------------------------- x-pass
__device__ __forceinline__ int wavenumber(int i, int n) { return i <= n / 2 ? i : i - n; }

// Bin of q >= 1: the largest b with Q_b <= q.  qthr (LDS) holds the nb
// thresholds Q_b and a sentinel INT32_MAX at index nb.  The float estimate
// floor(sqrt(q * qscale)), qscale = 4 nb^2 / (3 N^2), is the exact bin up to
// rounding, i.e. off by at most one either way; one comparison against each
// neighbouring threshold (read together) corrects it.
__device__ __forceinline__ int bin_of(int q, const int32_t* qthr, int nb, float qscale) {
  int b = static_cast<int>(__builtin_amdgcn_sqrtf(static_cast<float>(q) * qscale));
  b = b > nb - 1 ? nb - 1 : b;
  const int lo = qthr[b], hi = qthr[b + 1];
  return b + (q >= hi ? 1 : 0) - (q < lo ? 1 : 0);
}

// Re(conj(u) t) in FP64 (products of FP32 values are exact there).
template <typename R>
__device__ __forceinline__ double cross(cx<R> u, cx<R> t) {
  return static_cast<double>(u.x) * t.x + static_cast<double>(u.y) * t.y;
}

template <typename R>
struct DrawCtx {
  const int32_t* qthr;    // LDS
  const cx<R>* tab;       // LDS, (A_b, B_b)
  double* hist;           // this lane's LDS histogram
  double* hist2;          // its second histogram (mixing sweep) or nullptr
  float qscale;
  int nb;
  uint32_t chain;
  uint32_t sweep;
};

// k2 of register e in a slot of RL registers whose modes are ix = q + S k2:
// k2 = h0 + KS (e mod RL/2) + KS RL/2 (e div RL/2), with S KS RL = N.  A
// whole column or pencil (KS = 1, h0 = 0) holds k2 = e; one lane of a lane
// pair (KS = 2, RL = 8) holds the k2 of parity h0.  Registers e and e + RL/2
// are modes ix and ix + N/2.
template <int RL, int KS>
__device__ __forceinline__ int k2_of(int e, int h0) {
  return h0 + KS * (e % (RL / 2)) + KS * (RL / 2) * (e / (RL / 2));
}

// Signal draw of one register slot: v[e] holds t^ of mode (ix, iy, kz) with
// ix = q + S k2_of(e).  Each mode is drawn from the signal
// conditional
//   s^ = f t^ + sqrt(v/2) (G_re + i G_im),  f = P/(P + tau), v = M tau f,
// stored divided by M: s^/M = A_b t^ + B_b (G_re + i G_im), A_b = f/M,
// B_b = sqrt(tau f / (2M)).  (G_re, G_im) of (ix, iy, kz) come from Philox
// counter ((kz N + iy) N/2 + ix mod N/2, sweep, 1, chain): words (x0, x1)
// for ix < N/2, (x2, x3) for ix >= N/2 -- registers r and r + RL/2 share a
// call.
// |s^/M|^2 (squared in R) is added to the lane's LDS histogram; the weight
// w of the plane (1 on kz = 0, N/2, else 2) is applied per workgroup in
// draw_epilogue.  This is the form for planes 0 < kz < N/2, where every
// mode is drawn independently and q >= 1.
template <typename R, int N, int RL, int S, bool MIX, int KS = 1>
__device__ __forceinline__ void draw_slot_plain(cx<R>* v, int q, int iy, int kz,
                                                const SweepArgs<R>& a, const DrawCtx<R>& d,
                                                int h0 = 0) {
  constexpr int H = N / 2;
  const int my = wavenumber(iy, N);
  const int r2 = my * my + kz * kz;
#pragma unroll
  for (int r = 0; r < RL / 2; ++r) {
    const int ixl = q + S * k2_of<RL, KS>(r, h0);   // < N/2; its partner ixl + N/2 is element r + RL/2
    R g[4];
    {
      const uint32_t w0 = static_cast<uint32_t>((kz * N + iy) * H + ixl);
      const Words4 w = philox4x32_10(w0, d.sweep, kPhaseSignal, d.chain, a.key0, a.key1);
      box_muller(w.x0, w.x1, g[0], g[1]);
      box_muller(w.x2, w.x3, g[2], g[3]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = r + h * (RL / 2);
      const int mx = wavenumber(ixl + h * H, N);
      const int b = bin_of(mx * mx + r2, d.qthr, d.nb, d.qscale);
      const cx<R> ab = d.tab[b];
      const cx<R> t = v[e];
      const cx<R> out{ab.x * t.x + ab.y * g[2 * h], ab.x * t.y + ab.y * g[2 * h + 1]};
      atomicAdd(d.hist + b, static_cast<double>(out.x * out.x + out.y * out.y));
      if (MIX) atomicAdd(d.hist2 + b, cross(out, t));
      v[e] = out;
    }
  }
}

// The same on the kz = 0 and kz = N/2 planes, where s^ is Hermitian within
// the plane: self-conjugate modes are real with the full variance; the member
// of a conjugate pair with the larger ix*N + iy uses its partner's normals
// conjugated; q = 0 gives 0.
template <typename R, int N, int RL, int S, bool MIX, int KS = 1>
__device__ __forceinline__ void draw_slot_herm(cx<R>* v, int q, int iy, int kz,
                                               const SweepArgs<R>& a, const DrawCtx<R>& d,
                                               int h0 = 0) {
  constexpr int H = N / 2;
  const int my = wavenumber(iy, N);
  const int r2 = my * my + kz * kz;
  const int py = (N - iy) % N;
#pragma unroll
  for (int r = 0; r < RL / 2; ++r) {
    const int ixl = q + S * k2_of<RL, KS>(r, h0);
    R g[4];
    {
      const uint32_t w0 = static_cast<uint32_t>((kz * N + iy) * H + ixl);
      const Words4 w = philox4x32_10(w0, d.sweep, kPhaseSignal, d.chain, a.key0, a.key1);
      box_muller(w.x0, w.x1, g[0], g[1]);
      box_muller(w.x2, w.x3, g[2], g[3]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = r + h * (RL / 2);
      const int x = ixl + h * H;
      const int mx = wavenumber(x, N);
      const int qq = mx * mx + r2;
      const int plin = ((N - x) % N) * N + py, lin = x * N + iy;
      if (plin < lin) continue;   // drawn in the second loop
      cx<R> out{R(0), R(0)};
      if (qq > 0) {
        const int b = bin_of(qq, d.qthr, d.nb, d.qscale);
        const cx<R> ab = d.tab[b];
        const cx<R> t = v[e];
        if (plin == lin)   // self-conjugate: real, full variance
          out = cx<R>{ab.x * t.x + R(1.4142135623730950488) * ab.y * g[2 * h], R(0)};
        else
          out = cx<R>{ab.x * t.x + ab.y * g[2 * h], ab.x * t.y + ab.y * g[2 * h + 1]};
        atomicAdd(d.hist + b, static_cast<double>(out.x * out.x + out.y * out.y));
        if (MIX) atomicAdd(d.hist2 + b, cross(out, t));
      }
      v[e] = out;
    }
  }
#pragma unroll
  for (int e = 0; e < RL; ++e) {
    const int x = q + S * k2_of<RL, KS>(e, h0);
    const int px = (N - x) % N;
    if (px * N + py >= x * N + iy) continue;
    const int mx = wavenumber(x, N);
    const int b = bin_of(mx * mx + r2, d.qthr, d.nb, d.qscale);
    const cx<R> ab = d.tab[b];
    const uint32_t w0 = static_cast<uint32_t>((kz * N + py) * H + (px % H));
    const Words4 w = philox4x32_10(w0, d.sweep, kPhaseSignal, d.chain, a.key0, a.key1);
    R g0, g1;
    if (px >= H) box_muller(w.x2, w.x3, g0, g1);
    else box_muller(w.x0, w.x1, g0, g1);
    const cx<R> t = v[e];
    const cx<R> out{ab.x * t.x + ab.y * g0, ab.x * t.y - ab.y * g1};
    atomicAdd(d.hist + b, static_cast<double>(out.x * out.x + out.y * out.y));
    if (MIX) atomicAdd(d.hist2 + b, cross(out, t));
    v[e] = out;
  }
}

// MIX = true also adds Re(conj(s^/M) t^) to the second histogram (the
// mixing sweep's cross term).
template <typename R, int N, int RL, int S, bool MIX = false, int KS = 1>
__device__ __forceinline__ void draw_slot(cx<R>* v, int q, int iy, int kz,
                                          const SweepArgs<R>& a, const DrawCtx<R>& d,
                                          int h0 = 0) {
  if (kz == 0 || kz == N / 2) draw_slot_herm<R, N, RL, S, MIX, KS>(v, q, iy, kz, a, d, h0);
  else draw_slot_plain<R, N, RL, S, MIX, KS>(v, q, iy, kz, a, d, h0);
}

// Deterministic counterpart of draw_slot for the Wiener iteration: every mode
// becomes A_b t^ (the signal conditional's mean, f_b t^ / M).  XM = kXDet
// stores t^ to aux (when set); XM = kXAdj adds Re(conj(t^) u^) to the bin's
// histogram, u^ read from aux -- with the plane weight w applied in
// draw_epilogue, the per-bin sum of the adjoint's d chi2 / d f_b (before its
// 1/M).  aux element e sits at aux[e * astride].
template <typename R, int N, int RL, int S, int XM>
__device__ __forceinline__ void filter_slot(cx<R>* v, int q, int iy, int kz, const DrawCtx<R>& d,
                                            cx<R>* aux, size_t astride) {
  const int my = wavenumber(iy, N);
  const int r2 = my * my + kz * kz;
#pragma unroll
  for (int e = 0; e < RL; ++e) {
    const int mx = wavenumber(q + S * e, N);
    const int qq = mx * mx + r2;
    const cx<R> t = v[e];
    cx<R> out{R(0), R(0)};
    if (qq > 0) {
      const int b = bin_of(qq, d.qthr, d.nb, d.qscale);
      const R f = d.tab[b].x;
      out = cx<R>{f * t.x, f * t.y};
      if (XM == kXAdj) {
        const cx<R> u = aux[e * astride];
        atomicAdd(d.hist + b, static_cast<double>(t.x) * u.x + static_cast<double>(t.y) * u.y);
      }
    }
    if (XM == kXDet && aux != nullptr) aux[e * astride] = t;
    v[e] = out;
  }
}

// Doubles between consecutive LDS histogram copies: nb rounded up to an odd
// number, so that the copies of one bin fall on different LDS banks (lanes
// of one wave that add to the same bin of different copies then do not
// collide on a bank).
__host__ __device__ constexpr int hist_stride(int nb) { return nb | 1; }

// Doubles of LDS that the NH histogram sets of a workgroup take (NHIST
// copies each).
__host__ __device__ constexpr int hist_doubles(int nhist, int nb, int nh) {
  return nh * nhist * hist_stride(nb);
}

// Shared prologue / epilogue of the x-pass kernels: LDS tables and per-wave
// histograms (HG copies per wave by lane: lane l adds to copy l mod HG), then
// one partial per workgroup.  NH histogram sets (1, or 2 for the mixing
// sweep) of NHIST copies each, copies hist_stride(nb) doubles apart.
template <typename R, int NT, int NHIST, int HG, int NH = 1>
__device__ __forceinline__ DrawCtx<R> draw_prologue(const SweepArgs<R>& a, int c, double* dyn,
                                                    int n) {
  const int nb = a.nb, tid = threadIdx.x, hs = hist_stride(nb);
  constexpr int hg = HG, nhist = NHIST;
  double* hist = dyn;
  R* tab = reinterpret_cast<R*>(hist + NH * nhist * hs);
  int32_t* qthr = reinterpret_cast<int32_t*>(tab + 2 * nb);
  for (int i = tid; i < NH * nhist * hs; i += NT) hist[i] = 0.0;
  for (int i = tid; i < 2 * nb; i += NT) tab[i] = a.table[static_cast<size_t>(c) * 2 * nb + i];
  for (int i = tid; i <= nb; i += NT) qthr[i] = i < nb ? a.qthr[i] : INT32_MAX;
  DrawCtx<R> d;
  d.qthr = qthr;
  d.tab = reinterpret_cast<const cx<R>*>(tab);
  d.hist = hist + ((tid / 64) * hg + (tid % hg)) * hs;
  d.hist2 = NH == 2 ? d.hist + nhist * hs : nullptr;
  d.qscale = static_cast<float>(4.0 * nb * nb / (3.0 * n * n));
  d.nb = nb;
  d.chain = a.chain0 + c;
  d.sweep = a.ctr[1];
  return d;
}

// The workgroup's plane kz sets the weight w of its modes in the full-grid
// sums: 1 on kz = 0 and kz = N/2, 2 elsewhere (each mode stands for itself
// and its conjugate).
// `hist` is the set's first copy (NHIST copies).
template <typename R, int NT, int NHIST>
__device__ __forceinline__ void draw_epilogue(const SweepArgs<R>& a, int c, double* hist, int wg,
                                              double wgt, double* partials = nullptr) {
  __syncthreads();   // all histogram atomics are done
  const int nb = a.nb, tid = threadIdx.x, hs = hist_stride(nb);
  double* part = (partials ? partials : a.partials) + static_cast<size_t>(c) * a.n_wg_x * nb + wg;
  // Fixed-order reduction of the NHIST copies: G groups of PER consecutive
  // copies, each summed in ascending order into its first copy (every entry is
  // read and written by one thread only), then the G group sums in order.
  // G = gcd(NHIST, 8) from 16 copies up, else 1.
  constexpr int G = NHIST < 16 ? 1 : (NHIST % 8 == 0 ? 8 : (NHIST % 4 == 0 ? 4 : (NHIST % 2 == 0 ? 2 : 1)));
  constexpr int PER = NHIST / G;
  if (G > 1) {
    for (int it = tid; it < nb * G; it += NT) {
      const int b = it % nb, g = it / nb;
      double s = 0.0;
      for (int w = 0; w < PER; ++w) s += hist[(g * PER + w) * hs + b];
      hist[g * PER * hs + b] = s;
    }
    __syncthreads();
  }
  // group sums sit at copies 0, PER, 2 PER, ...; with one group, every copy
  constexpr int STEP = G > 1 ? PER : 1;
  constexpr int COUNT = G > 1 ? G : NHIST;
  for (int b = tid; b < nb; b += NT) {
    double s = 0.0;
    for (int g = 0; g < COUNT; ++g) s += hist[g * STEP * hs + b];
    part[static_cast<size_t>(b) * a.n_wg_x] = wgt * s;
  }
}

// Split x-pass (32 <= N <= 256): workgroup = one kz plane, P consecutive iy
// columns and K1 of the NA values of k1; thread (col, k1) holds rows
// 16 k1 .. 16 k1 + 15 of its column, i.e. Y[0..15][k1], and runs x stage B,
// the draw and the inverse stage B in registers.  The workgroup reads and
// writes runs of P consecutive complex values per row, and long runs are what
// HBM rewards: sides divisible by 64 with NA >= 4 take P = min(N, 128) (1 KiB
// runs in FP32) and K1 = 256 / P, so NA / K1 workgroups share a column block.
// At 256^3 that took the pass from 41.7 us (P = 16) to 36.7 us.  The other
// sides take every k1 of a column.
// Variants: 0 is this tile with 8 LDS histogram copies per wave, for up to
// 255 bins (neighbouring lanes hold neighbouring iy, whose bins are mostly
// equal, so more copies mean fewer lanes adding to one address per
// instruction: the 256^3 x-pass takes 32.0 us against 33.6 us with 2
// copies); 1 is the same tile with 2 copies, for any bin count and for the
// mixing sweep and the Wiener iteration; 2 splits every column over a pair
// of neighbouring lanes (LANES = 2), each holding 8 of its 16 rows, with 8
// copies: twice the waves, each with half the work, for a grid that
// otherwise gives each SIMD few rounds of waves (below).  The autotuner
// chooses among them.
template <typename R, int N, int V = 0>
struct XSTile {
  static constexpr int NA = N >= 32 ? N / 16 : 2;   // only meaningful when split_x<N>()
  static constexpr bool WIDE = N % 64 == 0 && NA >= 4 && NA % 4 == 0;
  static constexpr int LANES = V == 2 ? 2 : 1;       // lanes per column
  static constexpr int P0 = WIDE ? (N < 128 ? N : 128) : divisor_below(N, 256 / NA);
  static constexpr int P = V < 2 ? P0 : (N < 128 ? N : 128);       // columns per workgroup
  static constexpr int K1 = V < 2 ? (WIDE ? 256 / P0 : NA) : divisor_below(NA, 128 / P);   // k1 values
  static constexpr int KB = NA / K1;                 // workgroups per column block
  static constexpr int NT = LANES * P * K1;
  static constexpr int WPP = (N / P) * KB;           // workgroups per kz plane
  static constexpr int NWAVES = (NT + 63) / 64;
  static constexpr int HG = V == 1 ? 2 : 8;          // LDS histogram copies per wave
  static constexpr int NHIST = NWAVES * HG;
  static constexpr int MAX_BINS = HG == 8 ? 255 : 1024;   // 8 copies: 64 KiB of LDS at most
  static_assert(N % P == 0 && NA % K1 == 0 && NT <= 256, "x-pass tile must cover the plane");
  // FP32 at N = 256 would take 98 VGPRs (4 waves per SIMD); held to 96 (5
  // waves, no spill) the pass runs 33.2 us instead of 35.5 us.
  static constexpr int MIN_WAVES = (V < 2 && sizeof(R) == 4 && N == 256) ? 5 : 1;
};

// The value of the other lane of this lane's pair (lanes 2p and 2p + 1), by
// a quad permutation [1, 0, 3, 2] of the wave's lanes (DPP, no LDS).
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              static_cast<long long>(static_cast<unsigned int>(lo)));
}
template <typename R>
__device__ __forceinline__ cx<R> pair_swap(cx<R> z) {
  return cx<R>{pair_swap(z.x), pair_swap(z.y)};
}

// x stage B of a column split over a lane pair: lane h (0 or 1) holds rows
// 8 h + i (i < 8) of the column, x_n = Y[n][k1].  The 16-point transform's
// first radix-2 stage (decimation in frequency) pairs rows i and i + 8: lane
// 0 keeps x_i + x_{i+8}, lane 1 keeps (x_i - x_{i+8}) W_16^i.  The rest is an
// 8-point transform of each lane's own values, after which register j of lane
// h holds X[2 j + h], i.e. k2 = 2 j + h.  The same operations as the
// 16-point transform of one lane, in the same order.
template <typename R>
__device__ __forceinline__ void pair_dft16_fwd(cx<R>* v, int h) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const cx<R> o = pair_swap(v[i]);
    const cx<R> sum{v[i].x + o.x, v[i].y + o.y};
    const cx<R> dif = rot16<R, false>(cx<R>{o.x - v[i].x, o.y - v[i].y}, i);
    v[i] = h ? dif : sum;
  }
  dft<R, 8, false>(v);
}

// Its inverse, unnormalised (16 x_n, as the 16-point inverse gives): each
// lane's 8-point inverse gives 8 (x_i + x_{i+8}) on lane 0 and
// 8 (x_i - x_{i+8}) W_16^i on lane 1; lane 1 removes the twiddle, and the
// pair's sum and difference give lane 0 its rows 16 x_i and lane 1 its rows
// 16 x_{i+8}.
template <typename R>
__device__ __forceinline__ void pair_dft16_inv(cx<R>* v, int h) {
  dft<R, 8, true>(v);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const cx<R> own = h ? rot16<R, true>(v[i], i) : v[i];
    const cx<R> o = pair_swap(own);
    v[i] = h ? cx<R>{o.x - own.x, o.y - own.y} : cx<R>{own.x + o.x, own.y + o.y};
  }
}

template <typename R, int N, int XM, int V = 0>
__global__ void __launch_bounds__((XSTile<R, N, V>::NT), (XSTile<R, N, V>::MIN_WAVES))
xsplit_kernel(SweepArgs<R> a) {
  using T = XSTile<R, N, V>;
  constexpr int P = T::P, NT = T::NT, NA = T::NA;
  extern __shared__ double dyn[];      // histograms (hist_doubles), table (2 nb R), qthr (nb + 1)
  const int tid = threadIdx.x;
  const int iy0 = (blockIdx.x / T::KB) * P;
  const int kz = blockIdx.y;
  const int c = blockIdx.z;
  constexpr int NH = XM == kXMix ? 2 : 1;
  const DrawCtx<R> d = draw_prologue<R, NT, T::NHIST, T::HG, NH>(a, c, dyn, N);
  if constexpr (T::LANES == 2) {
    static_assert(XM == kXSample, "the lane-pair tile serves Gibbs sweeps only");
    // lanes 2 p and 2 p + 1 share column p: lane h holds rows 8 h .. 8 h + 7
    const int pr = tid >> 1, h = tid & 1;
    const int col = pr % P, k1 = (blockIdx.x % T::KB) * T::K1 + pr / P;
    cx<R>* base = a.spec + static_cast<size_t>(c) * a.spec_stride +
                  (static_cast<size_t>(kz) * N + 16 * k1 + 8 * h) * N + iy0 + col;
    cx<R> v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = base[static_cast<size_t>(j) * N];
    pair_dft16_fwd(v, h);                // v[j] = X[k1 + NA (2 j + h)]
    __syncthreads();                     // tables and histograms ready
    draw_slot<R, N, 8, NA, false, 2>(v, k1, iy0 + col, kz, a, d, h);
    pair_dft16_inv(v, h);
#pragma unroll
    for (int j = 0; j < 8; ++j) base[static_cast<size_t>(j) * N] = v[j];
    const int wg = blockIdx.y * gridDim.x + blockIdx.x;
    draw_epilogue<R, NT, T::NHIST>(a, c, dyn, wg, (kz == 0 || kz == N / 2) ? 1.0 : 2.0);
    return;
  }
  const int col = tid % P, k1 = (blockIdx.x % T::KB) * T::K1 + tid / P;
  cx<R>* base = a.spec + static_cast<size_t>(c) * a.spec_stride +
                (static_cast<size_t>(kz) * N + 16 * k1) * N + iy0 + col;
  cx<R> v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = base[static_cast<size_t>(j) * N];
  dft<R, 16, false>(v);                 // v[k2] = X[k1 + NA k2]
  __syncthreads();                      // tables and histograms ready
  if (XM == kXSample || XM == kXMix) {
    draw_slot<R, N, 16, NA, XM == kXMix>(v, k1, iy0 + col, kz, a, d);
  } else {
    cx<R>* aux = a.aux == nullptr ? nullptr : a.aux + (base - a.spec);
    filter_slot<R, N, 16, NA, XM>(v, k1, iy0 + col, kz, d, aux, N);
  }
  // the mixing sweep stores the drawn modes untransformed (row 16 k1 + j
  // holds mode k1 + NA j) for the rescaling pass, which runs the inverse
  if (XM != kXMix) dft<R, 16, true>(v);
#pragma unroll
  for (int j = 0; j < 16; ++j) base[static_cast<size_t>(j) * N] = v[j];
  const int wg = blockIdx.y * gridDim.x + blockIdx.x;
  const double wgt = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
  if (XM != kXDet) draw_epilogue<R, NT, T::NHIST>(a, c, dyn, wg, wgt);
  if (XM == kXMix)
    draw_epilogue<R, NT, T::NHIST>(a, c, dyn + T::NHIST * hist_stride(a.nb), wg, wgt, a.partials2);
}

// Second half of the mixing sweep's x-pass: every mode of bin b, stored by
// xsplit_kernel<.., kXMix> in its post-DFT layout, is multiplied by ratio_b =
// sqrt(S^'_b / S^_b) from the Metropolis-Hastings move, then the inverse
// 16-point DFT restores the split layout for the inverse y-pass.
template <typename R, int N>
__global__ void __launch_bounds__((XSTile<R, N, 1>::NT))
xmixinv_kernel(SweepArgs<R> a) {
  using T = XSTile<R, N, 1>;
  constexpr int P = T::P, NT = T::NT, NA = T::NA;
  extern __shared__ double dyn[];      // ratio (nb R), qthr (nb + 1)
  const int tid = threadIdx.x, nb = a.nb;
  const int iy0 = (blockIdx.x / T::KB) * P, kz = blockIdx.y, c = blockIdx.z;
  R* rat = reinterpret_cast<R*>(dyn);
  int32_t* qthr = reinterpret_cast<int32_t*>(rat + nb);
  for (int i = tid; i < nb; i += NT) rat[i] = static_cast<R>(a.ratio[static_cast<size_t>(c) * nb + i]);
  for (int i = tid; i <= nb; i += NT) qthr[i] = i < nb ? a.qthr[i] : INT32_MAX;
  const float qscale = static_cast<float>(4.0 * nb * nb / (3.0 * N * N));
  const int col = tid % P, k1 = (blockIdx.x % T::KB) * T::K1 + tid / P;
  cx<R>* base = a.spec + static_cast<size_t>(c) * a.spec_stride +
                (static_cast<size_t>(kz) * N + 16 * k1) * N + iy0 + col;
  cx<R> v[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = base[static_cast<size_t>(j) * N];
  __syncthreads();
  const int my = wavenumber(iy0 + col, N);
  const int r2 = my * my + kz * kz;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int mx = wavenumber(k1 + NA * j, N);
    const int q = mx * mx + r2;
    if (q > 0) {
      const R f = rat[bin_of(q, qthr, nb, qscale)];
      v[j] = cx<R>{v[j].x * f, v[j].y * f};
    }
  }
  dft<R, 16, true>(v);
#pragma unroll
  for (int j = 0; j < 16; ++j) base[static_cast<size_t>(j) * N] = v[j];
}

// Whole-transform x-pass (the only path for N = 8, 16, 512; the alternative
// to the split path elsewhere): workgroup = one kz plane and P
// consecutive iy columns; forward x-DFT, draw, inverse x-DFT (in the reversed
// radix order, so it starts from the same registers).
template <typename R, int N>
__global__ void __launch_bounds__((XTile<R, N>::NT))
xpass_kernel(SweepArgs<R> a) {
  using T = XTile<R, N>;
  using TL = typename T::TL;
  constexpr int P = T::P, NT = T::NT, EPT = T::EPT;
  constexpr int RL = radix_at<N, false>(Radices<N>::n - 1);
  constexpr int NSL = N / RL;
  __shared__ cx<R> lds[P * T::PSTR];
  __shared__ cx<R> tw[N];
  extern __shared__ double dyn[];
  const int tid = threadIdx.x;
  const int iy0 = blockIdx.x * P;
  const int kz = blockIdx.y;
  const int c = blockIdx.z;
  cx<R>* spec = a.spec + static_cast<size_t>(c) * a.spec_stride +
                static_cast<size_t>(kz) * N * N;
  load_twiddles(tw, a.tw, N, NT);
  const DrawCtx<R> d = draw_prologue<R, NT, T::NHIST, T::HG>(a, c, dyn, N);
  cx<R> v[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    int col = 0, ix = 0;
    TL::template in_pos<false>(tid, e, col, ix);
    v[e] = spec[static_cast<size_t>(ix) * N + iy0 + col];
  }
  __syncthreads();   // tables and histograms ready (single-stage sizes have no barrier)
  fft_regs<R, N, TL, NT, false, false>(v, lds, tw);
#pragma unroll
  for (int i = 0; i < EPT / RL; ++i) {
    int col = 0, q = 0;
    TL::split(tid + i * NT, NSL, col, q);
    draw_slot<R, N, RL, NSL>(v + i * RL, q, iy0 + col, kz, a, d);
  }
  __syncthreads();   // every lane is done with the forward transform's LDS reads
  fft_regs<R, N, TL, NT, true, true>(v, lds, tw);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    int col = 0, ix = 0;
    TL::template out_pos<true>(tid, e, col, ix);
    spec[static_cast<size_t>(ix) * N + iy0 + col] = v[e];
  }
  draw_epilogue<R, NT, T::NHIST>(a, c, dyn, blockIdx.y * gridDim.x + blockIdx.x,
                                 (kz == 0 || kz == N / 2) ? 1.0 : 2.0);
}

}  // namespace mf
