// Register-resident batched pencil FFTs for gfx950.
//
// A workgroup transforms NPEN pencils of length N.  Every thread owns EPT =
// NPEN * N / NT elements, held in registers, and the transform is a Stockham
// autosort sequence of radix-R stages: a stage runs unrolled radix-R DFTs on
// the thread's registers, and the data cross between threads only between
// stages, through one LDS buffer.  So a two-stage size (N = 64 .. 256) costs a
// single LDS round trip, and the caller loads the first stage's inputs
// straight from HBM and stores the last stage's outputs straight back.
//
// Thread layout.  In a stage of radix R with BPP = N / R butterflies per
// pencil, the thread's slot i (i < EPT / R) is butterfly bf = tid + i * NT,
// mapped to (pencil, q) either pencil-fastest (pen = bf % NPEN, q = bf / NPEN:
// neighbouring lanes work on neighbouring pencils, for pencils strided in
// memory) or q-fastest (pen = bf / BPP, q = bf % BPP: for contiguous pencils).
// Slot i holds elements v[i*R + r], r < R, at pencil positions q + r * BPP on
// input of the first stage, and at q + r * (N / R) on output of the last
// stage.  The first stage of the reversed radix order has the same layout as
// the last stage of the normal order, so a forward transform in one order and
// an inverse in the other meet in registers.
//
// The transform is unnormalised: forward X_k = sum_n x_n exp(-2 pi i n k / N),
// inverse with exp(+2 pi i n k / N).  Inter-stage twiddles come from a table
// tw[j] = exp(-2 pi i j / N) computed in FP64 on the host, rounded once.
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

// cos and sin of 2 pi m / 16, m = 0..7.
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

// In-register DFT of a power-of-two size RAD (2..16) on v[0 .. RAD), natural
// order in and out: radix-2 decimation in frequency, then a bit-reversal
// permutation.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft_pow2(cx<R>* v) {
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

// -i z (forward) or +i z (inverse)
template <typename R, bool INV>
__device__ __forceinline__ cx<R> mul_mi(cx<R> z) {
  return INV ? cx<R>{-z.y, z.x} : cx<R>{z.y, -z.x};
}

// 3-point DFT: X0 = a + (b + c), X1,2 = a - (b + c)/2 -+ i sin(2pi/3) (b - c).
template <typename R, bool INV>
__device__ __forceinline__ void dft3(cx<R>* v) {
  const R s3 = R(0.86602540378443864676);
  const cx<R> a = v[0], b = v[1], c = v[2];
  const cx<R> t1{b.x + c.x, b.y + c.y};
  const cx<R> t2{a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y};
  const cx<R> d = mul_mi<R, INV>(cx<R>{s3 * (b.x - c.x), s3 * (b.y - c.y)});
  v[0] = cx<R>{a.x + t1.x, a.y + t1.y};
  v[1] = cx<R>{t2.x + d.x, t2.y + d.y};
  v[2] = cx<R>{t2.x - d.x, t2.y - d.y};
}

// 5-point DFT from the symmetric / antisymmetric pairs (a1 +- a4, a2 +- a3)
// with c_k = cos(2 pi k / 5), s_k = sin(2 pi k / 5).
template <typename R, bool INV>
__device__ __forceinline__ void dft5(cx<R>* v) {
  const R c1 = R(0.30901699437494742410), c2 = R(-0.80901699437494742410);
  const R s1 = R(0.95105651629515357212), s2 = R(0.58778525229247312917);
  const cx<R> a0 = v[0];
  const cx<R> p1{v[1].x + v[4].x, v[1].y + v[4].y}, m1{v[1].x - v[4].x, v[1].y - v[4].y};
  const cx<R> p2{v[2].x + v[3].x, v[2].y + v[3].y}, m2{v[2].x - v[3].x, v[2].y - v[3].y};
  const cx<R> e1{a0.x + c1 * p1.x + c2 * p2.x, a0.y + c1 * p1.y + c2 * p2.y};
  const cx<R> e2{a0.x + c2 * p1.x + c1 * p2.x, a0.y + c2 * p1.y + c1 * p2.y};
  const cx<R> o1 = mul_mi<R, INV>(cx<R>{s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y});
  const cx<R> o2 = mul_mi<R, INV>(cx<R>{s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y});
  v[0] = cx<R>{a0.x + p1.x + p2.x, a0.y + p1.y + p2.y};
  v[1] = cx<R>{e1.x + o1.x, e1.y + o1.y};
  v[4] = cx<R>{e1.x - o1.x, e1.y - o1.y};
  v[2] = cx<R>{e2.x + o2.x, e2.y + o2.y};
  v[3] = cx<R>{e2.x - o2.x, e2.y - o2.y};
}

// 6-point DFT: two 3-point DFTs of the even and odd samples, combined with
// w6^k = exp(-+ i pi k / 3): X_k = E_k + w6^k O_k, X_{k+3} = E_k - w6^k O_k.
template <typename R, bool INV>
__device__ __forceinline__ void dft6(cx<R>* v) {
  cx<R> e[3] = {v[0], v[2], v[4]}, o[3] = {v[1], v[3], v[5]};
  dft3<R, INV>(e);
  dft3<R, INV>(o);
  const R h = R(0.5), s3 = R(0.86602540378443864676);
  const cx<R> w1 = INV ? cx<R>{h, s3} : cx<R>{h, -s3};
  const cx<R> w2 = INV ? cx<R>{-h, s3} : cx<R>{-h, -s3};
  const cx<R> t0 = o[0], t1 = cmul(o[1], w1), t2 = cmul(o[2], w2);
  v[0] = cx<R>{e[0].x + t0.x, e[0].y + t0.y};
  v[3] = cx<R>{e[0].x - t0.x, e[0].y - t0.y};
  v[1] = cx<R>{e[1].x + t1.x, e[1].y + t1.y};
  v[4] = cx<R>{e[1].x - t1.x, e[1].y - t1.y};
  v[2] = cx<R>{e[2].x + t2.x, e[2].y + t2.y};
  v[5] = cx<R>{e[2].x - t2.x, e[2].y - t2.y};
}

// In-register DFT of size RAD (1, 2, 3, 4, 5, 6, 8, 16), natural order.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (RAD == 1) return;
  else if constexpr (RAD == 3) dft3<R, INV>(v);
  else if constexpr (RAD == 5) dft5<R, INV>(v);
  else if constexpr (RAD == 6) dft6<R, INV>(v);
  else dft_pow2<R, RAD, INV>(v);
}

// Radix schedule per size (normal order); the reversed order runs it backwards.
template <int N>
struct Radices;
template <> struct Radices<8> { static constexpr int n = 1; static constexpr int r[3] = {8, 1, 1}; };
template <> struct Radices<16> { static constexpr int n = 1; static constexpr int r[3] = {16, 1, 1}; };
template <> struct Radices<32> { static constexpr int n = 2; static constexpr int r[3] = {8, 4, 1}; };
template <> struct Radices<64> { static constexpr int n = 2; static constexpr int r[3] = {8, 8, 1}; };
template <> struct Radices<128> { static constexpr int n = 2; static constexpr int r[3] = {16, 8, 1}; };
template <> struct Radices<256> { static constexpr int n = 2; static constexpr int r[3] = {16, 16, 1}; };
template <> struct Radices<512> { static constexpr int n = 3; static constexpr int r[3] = {8, 8, 8}; };
template <> struct Radices<48> { static constexpr int n = 3; static constexpr int r[3] = {3, 4, 4}; };
template <> struct Radices<80> { static constexpr int n = 3; static constexpr int r[3] = {5, 4, 4}; };
// 96 = 6 x 4 x 4 rather than 3 x 4 x 8: 12 elements per thread instead of 24
// (the z-pass needs 98 VGPRs instead of 198, 4 waves per SIMD instead of 2).
template <> struct Radices<96> { static constexpr int n = 3; static constexpr int r[3] = {6, 4, 4}; };

__host__ __device__ constexpr int gcd_(int a, int b) { return b == 0 ? a : gcd_(b, a % b); }

// Elements per thread of a size-N pencil tile: 16, or the least common
// multiple of the radices for mixed-radix sizes.
template <int N>
__host__ __device__ constexpr int ept() {
  int l = 1;
  for (int i = 0; i < Radices<N>::n; ++i) l = l / gcd_(l, Radices<N>::r[i]) * Radices<N>::r[i];
  return (16 % l == 0) ? 16 : l;
}

template <int N>
__host__ __device__ constexpr bool pow2() { return (N & (N - 1)) == 0; }

template <int N, bool REV>
__host__ __device__ constexpr int radix_at(int s) {
  return REV ? Radices<N>::r[Radices<N>::n - 1 - s] : Radices<N>::r[s];
}

template <int N, bool REV>
__host__ __device__ constexpr int span_before(int s) {   // NS of stage s
  int ns = 1;
  for (int t = 0; t < s; ++t) ns *= radix_at<N, REV>(t);
  return ns;
}

// Geometry of a tile: NPEN pencils, NT threads, pencil-fastest or q-fastest
// thread mapping, LDS pencil stride PSTR and intra-pencil padding of one
// element every 2^PADS elements (PADS = 0: none).
template <int N, int NPEN, int NT, bool PENFAST, int PSTR, int PADS>
struct Tile {
  static constexpr int EPT = NPEN * N / NT;
  __host__ __device__ static constexpr void split(int bf, int bpp, int& pen, int& q) {
    if (PENFAST) {
      pen = bf % NPEN;
      q = bf / NPEN;
    } else {
      pen = bf / bpp;
      q = bf % bpp;
    }
  }
  __host__ __device__ static constexpr int lidx(int pen, int i) {
    return pen * PSTR + (PADS ? i + (i >> PADS) : i);
  }
  // Pencil and position of the thread's element e on input of the first stage.
  template <bool REV>
  __host__ __device__ static constexpr void in_pos(int tid, int e, int& pen, int& pos) {
    constexpr int R0 = radix_at<N, REV>(0);
    int q = 0;
    split(tid + (e / R0) * NT, N / R0, pen, q);
    pos = q + (e % R0) * (N / R0);
  }
  // Pencil and position of the thread's element e on output of the last stage.
  template <bool REV>
  __host__ __device__ static constexpr void out_pos(int tid, int e, int& pen, int& pos) {
    constexpr int RL = radix_at<N, REV>(Radices<N>::n - 1);
    int q = 0;
    split(tid + (e / RL) * NT, N / RL, pen, q);
    pos = q + (e % RL) * (N / RL);
  }
};

// Stage s of the (REV-ordered) schedule on registers: optional LDS read with
// twiddles, DFTs, optional LDS write of the outputs.
template <typename R, int N, class TL, int NT, bool INV, bool REV, int S>
__device__ __forceinline__ void fft_stage(cx<R>* v, cx<R>* lds, const cx<R>* tw, bool read,
                                          bool write) {
  constexpr int RAD = radix_at<N, REV>(S);
  constexpr int NS = span_before<N, REV>(S);
  constexpr int BPP = N / RAD;
  constexpr int SLOTS = TL::EPT / RAD;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < SLOTS; ++i) {
    int pen = 0, q = 0;
    TL::split(tid + i * NT, BPP, pen, q);
    cx<R>* x = v + i * RAD;
    if (read) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) x[r] = lds[TL::lidx(pen, q + r * BPP)];
      if (NS > 1) {
        const int k = q % NS;
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          const cx<R> w = tw[r * k * (N / (NS * RAD))];
          x[r] = INV ? cmulc(x[r], w) : cmul(x[r], w);
        }
      }
    }
    dft<R, RAD, INV>(x);
  }
  if (write) {
#pragma unroll
    for (int i = 0; i < SLOTS; ++i) {
      int pen = 0, q = 0;
      TL::split(tid + i * NT, BPP, pen, q);
      const int base = (q / NS) * NS * RAD + q % NS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds[TL::lidx(pen, base + r * NS)] = v[i * RAD + r];
    }
  }
}

// Full transform of the thread's EPT registers (first-stage input layout in,
// last-stage output layout out).  The LDS buffer must be free on entry (the
// caller synchronises after its own last use); on return the LDS buffer may
// still be read by other threads, so a caller reusing it synchronises first.
template <typename R, int N, class TL, int NT, bool INV, bool REV>
__device__ __forceinline__ void fft_regs(cx<R>* v, cx<R>* lds, const cx<R>* tw) {
  constexpr int S = Radices<N>::n;
  fft_stage<R, N, TL, NT, INV, REV, 0>(v, lds, tw, false, S > 1);
  if constexpr (S > 1) {
    __syncthreads();
    fft_stage<R, N, TL, NT, INV, REV, 1>(v, lds, tw, true, false);
  }
  if constexpr (S > 2) {
    __syncthreads();   // every stage-1 read is done before the buffer is rewritten
    constexpr int RAD = radix_at<N, REV>(1);
    constexpr int NS = span_before<N, REV>(1);
    constexpr int BPP = N / RAD;
#pragma unroll
    for (int i = 0; i < TL::EPT / RAD; ++i) {
      int pen = 0, q = 0;
      TL::split(threadIdx.x + i * NT, BPP, pen, q);
      const int base = (q / NS) * NS * RAD + q % NS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds[TL::lidx(pen, base + r * NS)] = v[i * RAD + r];
    }
    __syncthreads();
    fft_stage<R, N, TL, NT, INV, REV, 2>(v, lds, tw, true, false);
  }
}

}  // namespace mf
