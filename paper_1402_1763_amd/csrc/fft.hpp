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

// In-register DFT of size RAD (2..16) on v[0 .. RAD), natural order in and
// out: radix-2 decimation in frequency, then a bit-reversal permutation.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cx<R>* v) {
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
