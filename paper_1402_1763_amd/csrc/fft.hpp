// LDS-resident batched pencil FFTs for gfx950.
//
// A workgroup holds a tile of NPEN pencils of length N in LDS (pencil p at
// buf + p * PSTR) and transforms all of them with a Stockham autosort
// schedule: each stage reads every butterfly's inputs into registers,
// applies the inter-stage twiddles, runs an unrolled radix-R DFT in
// registers, and writes the outputs back in place after a barrier.  With
// E = NPEN * N elements and NT threads, every thread owns E / NT elements in
// every stage whatever the radix.
//
// The transform is unnormalised: forward X_k = sum_n x_n exp(-2 pi i n k / N),
// inverse x_n = sum_k X_k exp(+2 pi i n k / N).  Inter-stage twiddles come
// from a table tw[j] = exp(-2 pi i j / N) computed in FP64 on the host and
// rounded once to the working precision.
#pragma once

#include <hip/hip_runtime.h>

namespace mf {

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return cx<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return cx<R>{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// cos and sin of 2 pi m / 16, m = 0..7, to double precision.
__device__ constexpr double kCos16[8] = {1.0,
                                         0.92387953251128675613,
                                         0.70710678118654752440,
                                         0.38268343236508977173,
                                         0.0,
                                         -0.38268343236508977173,
                                         -0.70710678118654752440,
                                         -0.92387953251128675613};
__device__ constexpr double kSin16[8] = {0.0,
                                         0.38268343236508977173,
                                         0.70710678118654752440,
                                         0.92387953251128675613,
                                         1.0,
                                         0.92387953251128675613,
                                         0.70710678118654752440,
                                         0.38268343236508977173};

// d * exp(-+ 2 pi i m / 16) (minus sign for the forward transform).
template <typename R, bool INV>
__device__ __forceinline__ cx<R> rot16(cx<R> d, int m) {
  if (m == 0) return d;
  if (m == 4) return INV ? cx<R>{-d.y, d.x} : cx<R>{d.y, -d.x};
  const R c = static_cast<R>(kCos16[m]);
  const R s = static_cast<R>(kSin16[m]);
  if (INV) return cx<R>{d.x * c - d.y * s, d.y * c + d.x * s};
  return cx<R>{d.x * c + d.y * s, d.y * c - d.x * s};
}

__host__ __device__ constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// In-register DFT of size RAD (2..16), natural order in and out.
// Decimation in frequency with radix-2 butterflies, then a bit-reversal
// permutation; every index is a compile-time constant after unrolling.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cx<R> (&v)[RAD]) {
#pragma unroll
  for (int len = RAD; len >= 2; len >>= 1) {
    const int half = len / 2;
#pragma unroll
    for (int start = 0; start < RAD; start += len) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const cx<R> a = v[start + j];
        const cx<R> b = v[start + j + half];
        v[start + j] = cx<R>{a.x + b.x, a.y + b.y};
        v[start + j + half] = rot16<R, INV>(cx<R>{a.x - b.x, a.y - b.y}, j * (16 / len));
      }
    }
  }
  cx<R> t[RAD];
#pragma unroll
  for (int i = 0; i < RAD; ++i) t[i] = v[bitrev(i, ilog2(RAD))];
#pragma unroll
  for (int i = 0; i < RAD; ++i) v[i] = t[i];
}

// One Stockham stage of radix RAD after NS points have been combined.
template <typename R, int N, int RAD, int NS, int NPEN, int PSTR, int NT, bool INV>
__device__ __forceinline__ void stockham_stage(cx<R>* buf, const cx<R>* tw) {
  constexpr int BPP = N / RAD;             // butterflies per pencil
  constexpr int TOTAL = NPEN * BPP;
  constexpr int BPT = (TOTAL + NT - 1) / NT;
  cx<R> v[BPT][RAD];
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int bf = tid + i * NT;
    if (TOTAL % NT == 0 || bf < TOTAL) {
      const int pen = bf / BPP, q = bf % BPP;
      const cx<R>* base = buf + pen * PSTR;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[i][r] = base[q + r * BPP];
      if (NS > 1) {
        const int k = q % NS;
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          const cx<R> w = tw[r * k * (N / (NS * RAD))];
          v[i][r] = INV ? cmulc(v[i][r], w) : cmul(v[i][r], w);
        }
      }
      dft<R, RAD, INV>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BPT; ++i) {
    const int bf = tid + i * NT;
    if (TOTAL % NT == 0 || bf < TOTAL) {
      const int pen = bf / BPP, q = bf % BPP;
      const int k = q % NS;
      cx<R>* base = buf + pen * PSTR + (q / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) base[r * NS] = v[i][r];
    }
  }
  __syncthreads();
}

// Radix schedule per size.
template <int N>
struct Radices;
template <> struct Radices<8> { static constexpr int n = 1, r0 = 8, r1 = 1, r2 = 1; };
template <> struct Radices<16> { static constexpr int n = 1, r0 = 16, r1 = 1, r2 = 1; };
template <> struct Radices<32> { static constexpr int n = 2, r0 = 8, r1 = 4, r2 = 1; };
template <> struct Radices<64> { static constexpr int n = 2, r0 = 8, r1 = 8, r2 = 1; };
template <> struct Radices<128> { static constexpr int n = 2, r0 = 16, r1 = 8, r2 = 1; };
template <> struct Radices<256> { static constexpr int n = 2, r0 = 16, r1 = 16, r2 = 1; };
template <> struct Radices<512> { static constexpr int n = 3, r0 = 8, r1 = 8, r2 = 8; };

// Transform NPEN pencils of length N held in LDS.  The caller must have
// synchronised after writing the tile; the tile is complete and visible to
// the whole workgroup on return.
template <typename R, int N, int NPEN, int PSTR, int NT, bool INV>
__device__ __forceinline__ void lds_fft(cx<R>* buf, const cx<R>* tw) {
  using P = Radices<N>;
  stockham_stage<R, N, P::r0, 1, NPEN, PSTR, NT, INV>(buf, tw);
  if constexpr (P::n >= 2) stockham_stage<R, N, P::r1, P::r0, NPEN, PSTR, NT, INV>(buf, tw);
  if constexpr (P::n >= 3)
    stockham_stage<R, N, P::r2, P::r0 * P::r1, NPEN, PSTR, NT, INV>(buf, tw);
}

}  // namespace mf
