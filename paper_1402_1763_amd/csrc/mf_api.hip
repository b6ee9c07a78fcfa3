// C ABI of the messenger-field Gibbs sampler (declarations and contract in
// include/mf.h).  Host side:
//  - descriptor validation and the workspace layout;
//  - FP64 set-up of the per-voxel messenger coefficients, tau, bin
//    thresholds, mode counts and twiddles;
//  - the launch sequences of the Gibbs and mixing sweeps and of the Wiener
//    iteration and its adjoint;
//  - state, checkpoints, graphs, diagnostics and the x-transform autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "mf.h"
#include "stream_kernels.hpp"
#include "sweep_kernels.hpp"
#include "wiener_kernels.hpp"

namespace {

thread_local std::string g_last_error = "no error";

mf_status fail(mf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define MF_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(MF_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool supported(int n) {
  return n == 8 || n == 16 || n == 32 || n == 48 || n == 64 || n == 80 || n == 96 || n == 128 ||
         n == 256 || n == 512;
}

// The two ways of running the x transform.  kPathSplit (32 <= N <= 256):
// the y-passes carry its radix-N/16 half, and the x-pass runs 16-point DFTs
// in registers.  kPathWhole: the x-pass runs whole x pencils through LDS.
// Both leave the same state between sweeps, so a problem may switch.
enum XPath : int { kPathSplit = 0, kPathWhole = 1 };

// Tile variants of the split path searched by the autotuner: x-pass tiles
// (XSTile<R, N, V>) and y-pass workgroup sizes (YSTile<R, N, V>).
constexpr int kTileVariants = 3;

template <typename R, int N>
struct Geometry {
  template <int V>
  static constexpr int split_wpp() {
    if constexpr (mf::split_x<N>()) return mf::XSTile<R, N, V>::WPP;
    else return N / mf::XTile<R, N>::P;
  }
  template <int V>
  static constexpr int y_units() {
    if constexpr (mf::split_x<N>()) return mf::YSTile<R, N, V>::G;
    else return 0;
  }
  // the y transform's radix schedule differs from its reverse (it is not a
  // palindrome, e.g. 6 x 4 x 4 at 96 but 16 x 16 at 256)
  static constexpr bool y_rev_distinct() {
    for (int i = 0; i < mf::Radices<N>::n; ++i)
      if (mf::Radices<N>::r[i] != mf::Radices<N>::r[mf::Radices<N>::n - 1 - i]) return true;
    return false;
  }
  template <int V>
  static constexpr int x_cols() {
    if constexpr (mf::split_x<N>()) return mf::XSTile<R, N, V>::P;
    else return 0;
  }
  template <int V>
  static constexpr int x_k1() {
    if constexpr (mf::split_x<N>()) return mf::XSTile<R, N, V>::K1;
    else return 0;
  }
  template <int V>
  static constexpr int x_hist() {
    if constexpr (mf::split_x<N>()) return mf::XSTile<R, N, V>::HG;
    else return 0;
  }
  template <int V>
  static constexpr int x_max_bins() {
    if constexpr (mf::split_x<N>()) return mf::XSTile<R, N, V>::MAX_BINS;
    else return 0;
  }
  static constexpr int xp_whole = N / mf::XTile<R, N>::P;
  static constexpr int ztiles = (N / mf::ZTile<R, N>::IXB) * (N / mf::ZTile<R, N>::P);
  static constexpr int zept = mf::ZTile<R, N>::EPT;
};

struct Shape {
  int xp_split[kTileVariants];   // split x-pass workgroups per kz plane, per tile variant
  int x_cols[kTileVariants];     // their iy columns and k1 values per workgroup
  int x_k1[kTileVariants];
  int x_hist[kTileVariants];     // LDS histogram copies per wave
  int x_max_bins[kTileVariants]; // most bins whose histograms fit the variant's LDS
  int y_units[kTileVariants];    // (kz, q) units per split y-pass workgroup, per variant
  int y_rev_distinct;            // the y radix schedule differs from its reverse
  int xp_whole;                  // whole-pencil x-pass workgroups per kz plane
  int ztiles;                    // z-pass tiles per chain
  int zept;                      // elements per z-pass lane (observation bits per tile)
};

template <typename R>
Shape shape_of(int n) {
  switch (n) {
#define MF_SHAPE(NN)                                                                       \
  case NN: {                                                                               \
    using G = Geometry<R, NN>;                                                             \
    return Shape{{G::template split_wpp<0>(), G::template split_wpp<1>(), G::template split_wpp<2>()}, \
                 {G::template x_cols<0>(), G::template x_cols<1>(), G::template x_cols<2>()},   \
                 {G::template x_k1<0>(), G::template x_k1<1>(), G::template x_k1<2>()},         \
                 {G::template x_hist<0>(), G::template x_hist<1>(), G::template x_hist<2>()},   \
                 {G::template x_max_bins<0>(), G::template x_max_bins<1>(),                   \
                  G::template x_max_bins<2>()},                                            \
                 {G::template y_units<0>(), G::template y_units<1>(), G::template y_units<2>()}, \
                 G::y_rev_distinct() ? 1 : 0, G::xp_whole, G::ztiles, G::zept};           \
  }
    MF_SHAPE(8) MF_SHAPE(16) MF_SHAPE(32) MF_SHAPE(48) MF_SHAPE(64) MF_SHAPE(80) MF_SHAPE(96)
    MF_SHAPE(128) MF_SHAPE(256) MF_SHAPE(512)
#undef MF_SHAPE
  }
  return Shape{};
}

struct Layout {
  size_t ctr, tw, qthr, counts, tau, pk, table, status, partials, ratio, tobs, coef, omw, spec,
      staging, rinv, total;
  size_t spec_elems, spec_stride;
  int n_wg_split[kTileVariants];   // split x-pass workgroups (one shell partial each) per variant
  int n_wg_whole;                  // whole-pencil x-pass workgroups
  int n_wg_max;
};

Layout make_layout(const mf_chain_desc& d) {
  const bool fp64 = d.precision == MF_PREC_FP64;
  const size_t rs = fp64 ? 8 : 4;
  const size_t n = static_cast<size_t>(d.n), m = n * n * n, nb = d.n_bins, nc = d.n_chains;
  const Shape sh = fp64 ? shape_of<double>(d.n) : shape_of<float>(d.n);
  Layout L{};
  L.spec_elems = (n / 2 + 1) * n * n;
  L.spec_stride = align_up(L.spec_elems * 2 * rs) / (2 * rs);
  L.n_wg_whole = static_cast<int>((n / 2 + 1) * sh.xp_whole);
  L.n_wg_max = L.n_wg_whole;
  for (int v = 0; v < kTileVariants; ++v) {
    L.n_wg_split[v] = static_cast<int>((n / 2 + 1) * sh.xp_split[v]);
    L.n_wg_max = std::max(L.n_wg_max, L.n_wg_split[v]);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.ctr = take(2 * 4);
  L.tw = take(n * 2 * rs);
  L.qthr = take(nb * 4);
  L.counts = take(nb * 8);
  L.tau = take(nc * 8);
  L.pk = take(nc * nb * 8);
  L.table = take(nc * nb * 2 * rs);
  L.status = take(nc * 4);
  L.partials = take(2 * nc * static_cast<size_t>(L.n_wg_max) * nb * 8);   // two sets (mixing)
  L.ratio = take(nc * nb * 8);
  L.tobs = take(nc * static_cast<size_t>(sh.ztiles) * 4);
  L.coef = take(nc * 2 * m * rs);
  L.omw = take(nc * m * rs);      // tau R^2 / N = 1 - alpha per voxel (Wiener filter only)
  L.spec = take(nc * L.spec_stride * 2 * rs);
  L.staging = take(m * rs);
  L.rinv = take(d.has_response ? nc * m * 8 : 0);   // 1 / R per voxel (0 unobserved), FP64
  L.total = off;
  return L;
}

mf_status check_desc(const mf_chain_desc* d) {
  if (!d) return fail(MF_E_INVALID_ARG, "descriptor is NULL");
  if (!supported(d->n))
    return fail(MF_E_UNSUPPORTED_SIZE, "grid side %d unsupported (8, 16, 32, 48, 64, 80, 96, 128, 256 or 512)", d->n);
  if (d->n_bins < 1 || d->n_bins > 1024)
    return fail(MF_E_INVALID_ARG, "n_bins %d outside [1, 1024]", d->n_bins);
  if (!(d->box > 0.0) || !std::isfinite(d->box))
    return fail(MF_E_INVALID_ARG, "box side must be positive and finite");
  if (d->precision != MF_PREC_FP64 && d->precision != MF_PREC_FP32)
    return fail(MF_E_INVALID_ARG, "unknown precision %d", d->precision);
  if (d->n_chains < 1 || d->n_chains > 4096)
    return fail(MF_E_INVALID_ARG, "n_chains %d outside [1, 4096]", d->n_chains);
  if (d->sample_pk != 0 && d->sample_pk != 1)
    return fail(MF_E_INVALID_ARG, "sample_pk must be 0 or 1");
  if (std::isnan(d->tau)) return fail(MF_E_INVALID_ARG, "tau is NaN");
  if (d->has_response != 0 && d->has_response != 1)
    return fail(MF_E_INVALID_ARG, "has_response must be 0 or 1");
  if (!std::isfinite(d->pk_prior_shape) || !std::isfinite(d->pk_prior_scale) ||
      d->pk_prior_shape < 0.0 || d->pk_prior_scale < 0.0)
    return fail(MF_E_INVALID_ARG, "the InvGamma prior (a0, b0) on P needs finite a0, b0 >= 0");
  return MF_OK;
}

// Smallest q of every bin: Q_0 = 1, Q_b = ceil(3 b^2 N^2 / (4 nb^2)) (exact).
std::vector<int32_t> bin_thresholds(int n, int nb) {
  std::vector<int32_t> q(nb);
  q[0] = 1;
  const unsigned long long den = 4ull * nb * nb;
  for (int b = 1; b < nb; ++b) {
    const unsigned long long num = 3ull * b * b * static_cast<unsigned long long>(n) * n;
    q[b] = static_cast<int32_t>((num + den - 1) / den);
  }
  return q;
}

// Full-grid modes per bin, counted over the half grid with weights 1 on the
// kz = 0 and kz = N/2 planes and 2 elsewhere.
std::vector<double> bin_counts(int n, int nb, const std::vector<int32_t>& qthr) {
  std::vector<long long> cnt(nb, 0);
  const int h = n / 2;
  std::vector<int> m2(n);
  for (int i = 0; i < n; ++i) {
    const int m = i <= h ? i : i - n;
    m2[i] = m * m;
  }
  for (int ix = 0; ix < n; ++ix)
    for (int iy = 0; iy < n; ++iy)
      for (int kz = 0; kz <= h; ++kz) {
        const int q = m2[ix] + m2[iy] + kz * kz;
        if (q == 0) continue;
        const int b = static_cast<int>(std::upper_bound(qthr.begin(), qthr.end(), q) - qthr.begin()) - 1;
        cnt[b] += (kz == 0 || kz == h) ? 1 : 2;
      }
  return std::vector<double>(cnt.begin(), cnt.end());
}

// exp(-2 pi i j / N) in FP64 from long-double angles.
std::vector<double> twiddles(int n) {
  std::vector<double> tw(2 * n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n; ++j) {
    const long double ang = 2.0L * pi * j / n;
    double c = static_cast<double>(cosl(ang)), s = -static_cast<double>(sinl(ang));
    if (std::fabs(c) < 1e-18) c = 0.0;
    if (std::fabs(s) < 1e-18) s = 0.0;
    tw[2 * j] = c;
    tw[2 * j + 1] = s;
  }
  return tw;
}

}  // namespace

// The last Wiener forward run, whose checkpoints a backward run reads.
struct WienerRun {
  const void* gws = nullptr;
  int chain = -1, n_iter = 0, every = 0;
};

// Recording of samples for the chain diagnostics (caller-owned buffers).
struct DiagRec {
  double* trace = nullptr;    // [chain][cap][nb]
  double* mom = nullptr;      // [chain][2][m]
  uint64_t start = 0;
  int thin = 0, cap = 0;
};

struct mf_problem {
  mf_chain_desc desc;
  Layout L;
  Shape sh;
  char* ws;
  std::vector<double> tau;
  uint64_t sweep;
  WienerRun wiener;
  DiagRec diag;
  std::vector<int> obs_chunks;  // per chain: z-pass (tile, element) chunks holding an observed voxel
  int xpath;                    // XPath of Gibbs sweeps
  int xvar = 0, yvar = 0;       // split-path tile variants of Gibbs sweeps (autotuner)
  int yrad = 0;                 // 1: the split y-passes run their radix stages reversed
  int graphs = 0;               // live graphs that captured this problem's sweep
  // x-pass workgroups of a path; the split path's with x-tile variant xv
  int n_wg(int path, int xv) const { return path == kPathSplit ? L.n_wg_split[xv] : L.n_wg_whole; }
  // the default split x tile: 8 histogram copies per wave where they fit
  int default_xvar() const { return desc.n_bins <= sh.x_max_bins[0] ? 0 : 1; }
  bool fp64() const { return desc.precision == MF_PREC_FP64; }
};

namespace {

// Sweep arguments with the x-pass on `path` (< 0: the problem's Gibbs path)
// and split x-tile variant xv (< 0: the problem's Gibbs variant).
template <typename R>
mf::SweepArgs<R> args_of(const mf_problem* p, int path = -1, int xv = -1) {
  if (path < 0) path = p->xpath;
  if (xv < 0) xv = p->xvar;
  mf::SweepArgs<R> a{};
  char* ws = p->ws;
  a.spec = reinterpret_cast<mf::cx<R>*>(ws + p->L.spec);
  a.coef = reinterpret_cast<const R*>(ws + p->L.coef);
  a.tile_obs = reinterpret_cast<const uint32_t*>(ws + p->L.tobs);
  a.ztiles = p->sh.ztiles;
  a.staging = reinterpret_cast<R*>(ws + p->L.staging);
  a.tau = reinterpret_cast<const double*>(ws + p->L.tau);
  a.pk = reinterpret_cast<double*>(ws + p->L.pk);
  a.table = reinterpret_cast<R*>(ws + p->L.table);
  a.partials = reinterpret_cast<double*>(ws + p->L.partials);
  a.partials2 = a.partials + static_cast<size_t>(p->desc.n_chains) * p->L.n_wg_max * p->desc.n_bins;
  a.ratio = reinterpret_cast<double*>(ws + p->L.ratio);
  a.qthr = reinterpret_cast<const int32_t*>(ws + p->L.qthr);
  a.counts = reinterpret_cast<const double*>(ws + p->L.counts);
  a.tw = reinterpret_cast<const mf::cx<R>*>(ws + p->L.tw);
  a.status = reinterpret_cast<uint32_t*>(ws + p->L.status);
  a.ctr = reinterpret_cast<uint32_t*>(ws + p->L.ctr);
  a.spec_stride = p->L.spec_stride;
  a.m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  a.nb = p->desc.n_bins;
  a.n_wg_x = p->n_wg(path, xv);
  a.staging_chain = 0;
  a.sample_pk = p->desc.sample_pk;
  a.chain0 = p->desc.chain_id;
  a.key0 = static_cast<uint32_t>(p->desc.seed);
  a.key1 = static_cast<uint32_t>(p->desc.seed >> 32);
  a.cs = R(1);
  a.cb = R(1);
  a.advance = 1;
  a.pk_mode = mf::kPkDraw;
  a.trace = p->diag.trace;
  a.mom = p->diag.mom;
  a.diag_start = static_cast<uint32_t>(p->diag.start);
  a.diag_thin = p->diag.thin;
  a.trace_cap = p->diag.cap;
  a.vcell = std::pow(p->desc.box / p->desc.n, 3);
  a.prior_a = p->desc.pk_prior_shape;
  a.prior_b = p->desc.pk_prior_scale / a.vcell;
  return a;
}

enum KernelId {
  kZ = 0, kYF = 1, kX = 2, kYI = 3, kZSet = 10, kZGet = 11, kTable = 12,
  kZDetK = 13, kZAccK = 14, kXDetK = 15, kXAdjK = 16, kXMixK = 17, kMixPkK = 18, kXMixInvK = 19
};

// Split-path y-pass with units variant V and radix order RV.
template <typename R, int N, bool INV, int V, bool RV>
void launch_ysplit(const mf::SweepArgs<R>& a, int nch, hipStream_t st) {
  using YS = mf::YSTile<R, N, V>;
  const int extra = INV ? a.nb : 0;   // the P(k) workgroups
  hipLaunchKernelGGL((mf::ysplit_kernel<R, N, INV, V, RV>),
                     dim3(16 / YS::G * (N / 2 + 1) + extra, 1, nch), dim3(YS::NT), 0, st, a);
}

// The split y-pass of y variant yv: units variant yv % 3 (G, G/2, G/4), radix
// stages in reversed order when yv >= 3.
template <typename R, int N, bool INV>
void launch_ysplit_v(const mf::SweepArgs<R>& a, int nch, hipStream_t st, int yv) {
  switch (yv) {
    case 1: launch_ysplit<R, N, INV, 1, false>(a, nch, st); break;
    case 2: launch_ysplit<R, N, INV, 2, false>(a, nch, st); break;
    case 3: launch_ysplit<R, N, INV, 0, true>(a, nch, st); break;
    case 4: launch_ysplit<R, N, INV, 1, true>(a, nch, st); break;
    case 5: launch_ysplit<R, N, INV, 2, true>(a, nch, st); break;
    default: launch_ysplit<R, N, INV, 0, false>(a, nch, st); break;
  }
}

// Split-path Gibbs x-pass with tile variant V.
template <typename R, int N, int V>
void launch_xsplit(const mf::SweepArgs<R>& a, int nch, hipStream_t st) {
  using XS = mf::XSTile<R, N, V>;
  const size_t tables = 2 * a.nb * sizeof(R) + (a.nb + 1) * 4;
  hipLaunchKernelGGL((mf::xsplit_kernel<R, N, mf::kXSample, V>), dim3(XS::WPP, N / 2 + 1, nch),
                     dim3(XS::NT), mf::hist_doubles(XS::NHIST, a.nb, 1) * sizeof(double) + tables, st, a);
}

// xv, yv: split-path tile variants of the Gibbs x-pass and of the y-passes
// (yv: units variant + 3 x radix order, launch_ysplit_v); the other x-pass
// modes (mixing, Wiener) run x-tile variant 1.
template <typename R, int N>
void launch_n(int id, const mf::SweepArgs<R>& a, int nch, hipStream_t st, bool whole, int xv,
              int yv) {
  using ZT = mf::ZTile<R, N>;
  using YT = mf::YTile<R, N>;
  using XT = mf::XTile<R, N>;
  using XS = mf::XSTile<R, N, 1>;   // the modes other than Gibbs sampling
  constexpr bool can_split = mf::split_x<N>();
  const bool split = can_split && !whole;
  const dim3 zgrid(N / ZT::P, N / ZT::IXB, nch), zgrid1(N / ZT::P, N / ZT::IXB, 1);
  const size_t tables = 2 * a.nb * sizeof(R) + (a.nb + 1) * 4;
  switch (id) {
    case kZ:
      hipLaunchKernelGGL((mf::zpass_kernel<R, N, mf::kZSweep>), zgrid, dim3(ZT::NT), 0, st, a);
      break;
    case kZSet:
      hipLaunchKernelGGL((mf::zpass_kernel<R, N, mf::kZSetState>), zgrid1, dim3(ZT::NT), 0, st, a);
      break;
    case kZGet:
      hipLaunchKernelGGL((mf::zpass_kernel<R, N, mf::kZGetState>), zgrid1, dim3(ZT::NT), 0, st, a);
      break;
    case kZDetK:
      hipLaunchKernelGGL((mf::zpass_kernel<R, N, mf::kZDet>), zgrid, dim3(ZT::NT), 0, st, a);
      break;
    case kZAccK:
      hipLaunchKernelGGL((mf::zpass_kernel<R, N, mf::kZAccum>), zgrid, dim3(ZT::NT), 0, st, a);
      break;
    case kYF:
      if constexpr (can_split) {
        if (split) {
          launch_ysplit_v<R, N, false>(a, nch, st, yv);
          break;
        }
      }
      hipLaunchKernelGGL((mf::ypass_kernel<R, N, false>), dim3((N / 2 + 1) * N / YT::NPEN, 1, nch),
                         dim3(YT::NT), 0, st, a);
      break;
    case kYI:
      if constexpr (can_split) {
        if (split) {
          launch_ysplit_v<R, N, true>(a, nch, st, yv);
          break;
        }
      }
      hipLaunchKernelGGL((mf::ypass_kernel<R, N, true>),
                         dim3((N / 2 + 1) * N / YT::NPEN + a.nb, 1, nch), dim3(YT::NT), 0, st, a);
      break;
    case kXDetK:
      if constexpr (can_split)
        hipLaunchKernelGGL((mf::xsplit_kernel<R, N, mf::kXDet, 1>), dim3(XS::WPP, N / 2 + 1, nch),
                           dim3(XS::NT), mf::hist_doubles(XS::NHIST, a.nb, 1) * sizeof(double) + tables, st, a);
      break;
    case kXMixK:
      if constexpr (can_split)
        hipLaunchKernelGGL((mf::xsplit_kernel<R, N, mf::kXMix, 1>), dim3(XS::WPP, N / 2 + 1, nch),
                           dim3(XS::NT), mf::hist_doubles(XS::NHIST, a.nb, 2) * sizeof(double) + tables, st, a);
      break;
    case kXMixInvK:
      if constexpr (can_split)
        hipLaunchKernelGGL((mf::xmixinv_kernel<R, N>), dim3(XS::WPP, N / 2 + 1, nch), dim3(XS::NT),
                           a.nb * sizeof(R) + (a.nb + 1) * 4, st, a);
      break;
    case kMixPkK:
      hipLaunchKernelGGL((mf::mix_pk_kernel<R>), dim3(a.nb, nch), dim3(256), 0, st, a);
      break;
    case kXAdjK:
      if constexpr (can_split)
        hipLaunchKernelGGL((mf::xsplit_kernel<R, N, mf::kXAdj, 1>), dim3(XS::WPP, N / 2 + 1, nch),
                           dim3(XS::NT), mf::hist_doubles(XS::NHIST, a.nb, 1) * sizeof(double) + tables, st, a);
      break;
    case kX:
      if constexpr (can_split) {
        if (split) {
          if (xv == 1) launch_xsplit<R, N, 1>(a, nch, st);
          else if (xv == 2) launch_xsplit<R, N, 2>(a, nch, st);
          else launch_xsplit<R, N, 0>(a, nch, st);
          break;
        }
      }
      hipLaunchKernelGGL((mf::xpass_kernel<R, N>), dim3(N / XT::P, N / 2 + 1, nch), dim3(XT::NT),
                         mf::hist_doubles(XT::NHIST, a.nb, 1) * sizeof(double) + tables, st, a);
      break;
    case kTable:
      hipLaunchKernelGGL((mf::pk_table_kernel<R>), dim3((a.nb + 63) / 64, nch), dim3(64), 0, st, a);
      break;
  }
}

template <typename R>
void launch(int id, const mf::SweepArgs<R>& a, int n, int nch, hipStream_t st, bool whole = false,
            int xv = 0, int yv = 0) {
  switch (n) {
    case 8: launch_n<R, 8>(id, a, nch, st, whole, xv, yv); break;
    case 16: launch_n<R, 16>(id, a, nch, st, whole, xv, yv); break;
    case 32: launch_n<R, 32>(id, a, nch, st, whole, xv, yv); break;
    case 48: launch_n<R, 48>(id, a, nch, st, whole, xv, yv); break;
    case 64: launch_n<R, 64>(id, a, nch, st, whole, xv, yv); break;
    case 80: launch_n<R, 80>(id, a, nch, st, whole, xv, yv); break;
    case 96: launch_n<R, 96>(id, a, nch, st, whole, xv, yv); break;
    case 128: launch_n<R, 128>(id, a, nch, st, whole, xv, yv); break;
    case 256: launch_n<R, 256>(id, a, nch, st, whole, xv, yv); break;
    case 512: launch_n<R, 512>(id, a, nch, st, whole, xv, yv); break;
  }
}

// path < 0: the problem's Gibbs-sweep path and tile variants; a given path
// (the mixing sweep's split path) runs x-tile variant 1.
mf_status launch_checked(mf_problem* p, int id, int staging_chain, hipStream_t st, int path = -1,
                         int pk_mode = mf::kPkDraw) {
  const int nch = p->desc.n_chains;
  const int xv = path < 0 ? p->xvar : 1, yv = p->yvar + 3 * p->yrad;
  if (path < 0) path = p->xpath;
  if (p->fp64()) {
    auto a = args_of<double>(p, path, xv);
    a.staging_chain = staging_chain;
    a.pk_mode = pk_mode;
    launch<double>(id, a, p->desc.n, nch, st, path == kPathWhole, xv, yv);
  } else {
    auto a = args_of<float>(p, path, xv);
    a.staging_chain = staging_chain;
    a.pk_mode = pk_mode;
    launch<float>(id, a, p->desc.n, nch, st, path == kPathWhole, xv, yv);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MF_E_DEVICE, "kernel %d launch failed: %s", id, hipGetErrorString(e));
  return MF_OK;
}

// The sweep index is Philox counter word 1, a 32-bit word: indices at or
// beyond 2^32 would repeat earlier sweeps' random numbers.
constexpr uint64_t kMaxSweep = 0xffffffffull;

mf_status check_sweep_index(uint64_t sweep) {
  if (sweep > kMaxSweep)
    return fail(MF_E_INVALID_ARG, "sweep index %llu beyond 2^32 - 1 (Philox counter word 1)",
                static_cast<unsigned long long>(sweep));
  return MF_OK;
}

// n more sweeps from the problem's current index must leave it at most
// 2^32 - 1, so that every state a chain reaches can be set and reloaded.
mf_status check_sweep_room(const mf_problem* p, int64_t n) {
  if (p->sweep + static_cast<uint64_t>(n) > kMaxSweep)
    return fail(MF_E_INVALID_ARG, "%lld sweeps from index %llu would pass 2^32 - 1 "
                "(Philox counter word 1)", static_cast<long long>(n),
                static_cast<unsigned long long>(p->sweep));
  return MF_OK;
}

// Device sweep counter := sweep in both slots (the z-pass reads slot 0, the
// x-pass and the P draw slot 1; the forward y-pass advances slot 0).
mf_status write_counter(mf_problem* p, uint64_t sweep, hipStream_t st) {
  const mf_status chk = check_sweep_index(sweep);
  if (chk != MF_OK) return chk;
  const uint32_t c[2] = {static_cast<uint32_t>(sweep), static_cast<uint32_t>(sweep)};
  MF_HIP(hipMemcpyAsync(p->ws + p->L.ctr, c, sizeof(c), hipMemcpyHostToDevice, st));
  MF_HIP(hipStreamSynchronize(st));
  return MF_OK;
}

const int kSweepOrder[MF_NUM_KERNELS] = {kZ, kYF, kX, kYI};

// Host FP64 -> device R copy through a temporary host buffer.
mf_status upload_real(mf_problem* p, void* dst, const double* src, size_t count, hipStream_t st) {
  if (p->fp64()) {
    MF_HIP(hipMemcpyAsync(dst, src, count * 8, hipMemcpyHostToDevice, st));
    MF_HIP(hipStreamSynchronize(st));
  } else {
    std::vector<float> tmp(count);
    for (size_t i = 0; i < count; ++i) tmp[i] = static_cast<float>(src[i]);
    MF_HIP(hipMemcpyAsync(dst, tmp.data(), count * 4, hipMemcpyHostToDevice, st));
    MF_HIP(hipStreamSynchronize(st));
  }
  return MF_OK;
}

mf_status download_real(mf_problem* p, double* dst, const void* src, size_t count, hipStream_t st) {
  if (p->fp64()) {
    MF_HIP(hipMemcpyAsync(dst, src, count * 8, hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
  } else {
    std::vector<float> tmp(count);
    MF_HIP(hipMemcpyAsync(tmp.data(), src, count * 4, hipMemcpyDeviceToHost, st));
    MF_HIP(hipStreamSynchronize(st));
    for (size_t i = 0; i < count; ++i) dst[i] = tmp[i];
  }
  return MF_OK;
}

// Voxel i is observed when its noise variance is finite and its response
// (1 without one) is not zero.
bool observed(const double* noise_var, const double* response, size_t i) {
  return !std::isinf(noise_var[i]) && (!response || response[i] != 0.0);
}

// Messenger coefficients of Sec. 3.1 with T = tau and N~ = N - tau R^2:
// mean = alpha s + beta with alpha = N~ / N = 1 - tau R^2 / N and
// beta = tau R d / N; (1, 0) where unobserved.  alpha is 0 in exact
// arithmetic where N / R^2 is smallest (tau is that minimum); rounding of
// tau R^2 / N there can leave -1 ulp, which is set back to 0.
// Also o = tau R^2 / N (0 where unobserved) per voxel, entry order
// [entry][2], for the Wiener filter's data-dependent coefficients.
template <typename R, int N>
void permute_coef(std::vector<R>& out, std::vector<R>& omw, std::vector<uint32_t>& obs,
                  const double* data, const double* noise_var, const double* response,
                  double tau) {
  using T = mf::ZTile<R, N>;
  const int tiles = (N / T::IXB) * (N / T::P);
  out.assign(static_cast<size_t>(2) * N * N * N, R(0));
  omw.assign(static_cast<size_t>(N) * N * N, R(0));
  obs.assign(tiles, 0);
  auto resp = [&](size_t i) { return response ? response[i] : 1.0; };
  auto alpha = [&](size_t i) {
    return observed(noise_var, response, i)
               ? std::max(0.0, 1.0 - tau * resp(i) * resp(i) / noise_var[i]) : 1.0;
  };
  auto beta = [&](size_t i) {
    return observed(noise_var, response, i) ? tau * resp(i) * data[i] / noise_var[i] : 0.0;
  };
  auto one_minus_alpha = [&](size_t i) {
    return observed(noise_var, response, i)
               ? std::min(1.0, tau * resp(i) * resp(i) / noise_var[i]) : 0.0;
  };
  for (int tile = 0; tile < tiles; ++tile)
    for (int e = 0; e < T::EPT; ++e)
      for (int tid = 0; tid < T::NT; ++tid) {
        int ix = 0, iya = 0, n = 0;
        mf::zpass_coef_voxel<R, N>(tile, e, tid, ix, iya, n);
        const size_t va = (static_cast<size_t>(ix) * N + iya) * N + n, vb = va + N;
        const size_t entry = (static_cast<size_t>(tile) * T::EPT + e) * T::NT + tid;
        R* o = &out[entry * 4];
        o[0] = static_cast<R>(alpha(va));
        o[1] = static_cast<R>(alpha(vb));
        o[2] = static_cast<R>(beta(va));
        o[3] = static_cast<R>(beta(vb));
        omw[entry * 2] = static_cast<R>(one_minus_alpha(va));
        omw[entry * 2 + 1] = static_cast<R>(one_minus_alpha(vb));
        if (observed(noise_var, response, va) || observed(noise_var, response, vb))
          obs[tile] |= 1u << e;
      }
}

template <typename R>
mf_status upload_coef(mf_problem* p, int c, const double* data, const double* noise_var,
                      const double* response, double tau, hipStream_t st) {
  std::vector<R> buf, omw;
  std::vector<uint32_t> obs;
  switch (p->desc.n) {
#define MF_PERMUTE(NN) \
  case NN: permute_coef<R, NN>(buf, omw, obs, data, noise_var, response, tau); break;
    MF_PERMUTE(8) MF_PERMUTE(16) MF_PERMUTE(32) MF_PERMUTE(48) MF_PERMUTE(64) MF_PERMUTE(80)
    MF_PERMUTE(96) MF_PERMUTE(128) MF_PERMUTE(256) MF_PERMUTE(512)
#undef MF_PERMUTE
  }
  MF_HIP(hipMemcpyAsync(p->ws + p->L.coef + static_cast<size_t>(c) * buf.size() * sizeof(R),
                        buf.data(), buf.size() * sizeof(R), hipMemcpyHostToDevice, st));
  MF_HIP(hipMemcpyAsync(p->ws + p->L.omw + static_cast<size_t>(c) * omw.size() * sizeof(R),
                        omw.data(), omw.size() * sizeof(R), hipMemcpyHostToDevice, st));
  MF_HIP(hipMemcpyAsync(p->ws + p->L.tobs + static_cast<size_t>(c) * obs.size() * 4, obs.data(),
                        obs.size() * 4, hipMemcpyHostToDevice, st));
  if (p->obs_chunks.size() < static_cast<size_t>(p->desc.n_chains)) p->obs_chunks.resize(p->desc.n_chains);
  int chunks = 0;
  for (uint32_t m : obs) chunks += __builtin_popcount(m);
  p->obs_chunks[c] = chunks;
  MF_HIP(hipStreamSynchronize(st));
  return MF_OK;
}

mf_status set_state(mf_problem* p, int chain, const double* s, const double* pk, hipStream_t st) {
  const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  const size_t rs = p->fp64() ? 8 : 4;
  if (s) {
    mf_status r = upload_real(p, p->ws + p->L.staging, s, m, st);
    if (r != MF_OK) return r;
    r = launch_checked(p, kZSet, chain, st);
    if (r != MF_OK) return r;
  }
  if (pk) {
    const double vc = std::pow(p->desc.box / p->desc.n, 3);
    std::vector<double> pg(p->desc.n_bins);
    for (int b = 0; b < p->desc.n_bins; ++b) {
      if (!std::isfinite(pk[b]) || pk[b] < 0.0)
        return fail(MF_E_NONFINITE, "P of bin %d is negative or not finite", b);
      pg[b] = pk[b] / vc;
    }
    MF_HIP(hipMemcpyAsync(p->ws + p->L.pk + static_cast<size_t>(chain) * p->desc.n_bins * 8,
                          pg.data(), pg.size() * 8, hipMemcpyHostToDevice, st));
    MF_HIP(hipStreamSynchronize(st));
    mf_status r = launch_checked(p, kTable, chain, st);
    if (r != MF_OK) return r;
  }
  (void)rs;
  MF_HIP(hipStreamSynchronize(st));
  return MF_OK;
}

}  // namespace

extern "C" {

int32_t mf_supported_n(int32_t n) { return supported(n) ? 1 : 0; }

mf_status mf_workspace_bytes(const mf_chain_desc* desc, size_t* bytes) {
  if (!bytes) return fail(MF_E_INVALID_ARG, "bytes is NULL");
  const mf_status st = check_desc(desc);
  if (st != MF_OK) return st;
  *bytes = make_layout(*desc).total;
  return MF_OK;
}

mf_status mf_init_problem(const mf_chain_desc* desc, const double* const* data,
                          const double* const* noise_var, const double* const* response,
                          const double* const* pk_init, const double* const* s_init,
                          void* workspace, size_t workspace_bytes, void* stream,
                          mf_problem** out) {
  if (!out) return fail(MF_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  mf_status st = check_desc(desc);
  if (st != MF_OK) return st;
  if (!data || !noise_var || !pk_init) return fail(MF_E_INVALID_ARG, "input arrays are NULL");
  const int n = desc->n, nb = desc->n_bins, nch = desc->n_chains;
  for (int c = 0; c < nch; ++c)
    if (!data[c] || !noise_var[c] || !pk_init[c])
      return fail(MF_E_INVALID_ARG, "input array of chain %d is NULL", c);
  if (desc->has_response) {
    if (!response) return fail(MF_E_INVALID_ARG, "has_response = 1 but response is NULL");
    for (int c = 0; c < nch; ++c)
      if (!response[c]) return fail(MF_E_INVALID_ARG, "response of chain %d is NULL", c);
  } else if (response) {
    return fail(MF_E_INVALID_ARG, "a response is given but has_response = 0");
  }
  const Layout L = make_layout(*desc);
  if (!workspace) return fail(MF_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(MF_E_WORKSPACE, "workspace is not %zu-byte aligned", kAlign);
  if (workspace_bytes < L.total)
    return fail(MF_E_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);

  const size_t m = static_cast<size_t>(n) * n * n;
  const double vc = std::pow(desc->box / n, 3);
  // tau per chain and input checks (Sec. 2: 0 < tau <= N_i / R_i^2 on
  // observed voxels)
  std::vector<double> tau(nch);
  for (int c = 0; c < nch; ++c) {
    const double* resp = response ? response[c] : nullptr;
    double tmin = std::numeric_limits<double>::infinity();
    size_t n_obs = 0;
    for (size_t i = 0; i < m; ++i) {
      const double nv = noise_var[c][i];
      const double rr = resp ? resp[i] : 1.0;
      if (!std::isfinite(rr))
        return fail(MF_E_NONFINITE, "chain %d voxel %zu: response not finite", c, i);
      if (rr == 0.0 || (std::isinf(nv) && nv > 0)) continue;
      if (!(nv > 0.0) || !std::isfinite(nv))
        return fail(MF_E_NONFINITE, "chain %d voxel %zu: noise variance %g not > 0", c, i, nv);
      if (!std::isfinite(data[c][i]))
        return fail(MF_E_NONFINITE, "chain %d voxel %zu: data not finite", c, i);
      tmin = std::min(tmin, nv / (rr * rr));
      ++n_obs;
    }
    if (n_obs == 0) return fail(MF_E_INVALID_ARG, "chain %d has no observed voxel", c);
    if (desc->tau > 0.0) {
      if (desc->tau > tmin)
        return fail(MF_E_TAU, "tau %g exceeds the smallest observed N / R^2 (%g) of chain %d",
                    desc->tau, tmin, c);
      tau[c] = desc->tau;
    } else {
      tau[c] = tmin;
    }
    for (int b = 0; b < nb; ++b)
      if (!std::isfinite(pk_init[c][b]) || pk_init[c][b] < 0.0)
        return fail(MF_E_NONFINITE, "chain %d: initial P of bin %d negative or not finite", c, b);
  }

  mf_problem* p = new mf_problem{};
  p->desc = *desc;
  p->L = L;
  p->sh = desc->precision == MF_PREC_FP64 ? shape_of<double>(n) : shape_of<float>(n);
  p->ws = static_cast<char*>(workspace);
  p->tau = tau;
  p->sweep = 0;
  p->xpath = (n >= 32 && n <= 256) ? kPathSplit : kPathWhole;
  p->xvar = p->default_xvar();
  hipStream_t hs = static_cast<hipStream_t>(stream);

  auto cleanup = [&](mf_status r) {
    delete p;
    return r;
  };
  // constant tables
  const std::vector<int32_t> qthr = bin_thresholds(n, nb);
  const std::vector<double> counts = bin_counts(n, nb, qthr);
  const std::vector<double> tw = twiddles(n);
  if ((st = upload_real(p, p->ws + L.tw, tw.data(), tw.size(), hs)) != MF_OK) return cleanup(st);
  if (hipMemcpyAsync(p->ws + L.qthr, qthr.data(), nb * 4, hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemcpyAsync(p->ws + L.counts, counts.data(), nb * 8, hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemcpyAsync(p->ws + L.tau, tau.data(), nch * 8, hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemsetAsync(p->ws + L.status, 0, nch * 4, hs) != hipSuccess ||
      hipMemsetAsync(p->ws + L.ctr, 0, 8, hs) != hipSuccess ||
      hipMemsetAsync(p->ws + L.partials, 0, 2 * static_cast<size_t>(nch) * L.n_wg_max * nb * 8, hs) !=
          hipSuccess ||
      hipStreamSynchronize(hs) != hipSuccess)
    return cleanup(fail(MF_E_DEVICE, "uploading tables failed"));
  // messenger coefficients in FP64 (alpha = 1 - tau R^2 / N,
  // beta = tau R d / N), rounded once and stored in the z-pass thread order
  for (int c = 0; c < nch; ++c) {
    const double* resp = response ? response[c] : nullptr;
    st = p->fp64() ? upload_coef<double>(p, c, data[c], noise_var[c], resp, tau[c], hs)
                   : upload_coef<float>(p, c, data[c], noise_var[c], resp, tau[c], hs);
    if (st != MF_OK) return cleanup(st);
  }
  // 1 / R per voxel (0 where unobserved), used by the Wiener filter only
  if (desc->has_response) {
    std::vector<double> ri(m);
    for (int c = 0; c < nch; ++c) {
      for (size_t i = 0; i < m; ++i)
        ri[i] = observed(noise_var[c], response[c], i) ? 1.0 / response[c][i] : 0.0;
      if (hipMemcpyAsync(p->ws + L.rinv + static_cast<size_t>(c) * m * 8, ri.data(), m * 8,
                         hipMemcpyHostToDevice, hs) != hipSuccess ||
          hipStreamSynchronize(hs) != hipSuccess)
        return cleanup(fail(MF_E_DEVICE, "uploading the response failed"));
    }
  }
  // initial state
  const size_t rs = p->fp64() ? 8 : 4;
  if (hipMemsetAsync(p->ws + L.spec, 0, static_cast<size_t>(nch) * L.spec_stride * 2 * rs, hs) !=
      hipSuccess)
    return cleanup(fail(MF_E_DEVICE, "clearing the spectrum failed"));
  for (int c = 0; c < nch; ++c) {
    const double* s0 = (s_init && s_init[c]) ? s_init[c] : nullptr;
    if (s0)
      for (size_t i = 0; i < m; ++i)
        if (!std::isfinite(s0[i])) return cleanup(fail(MF_E_NONFINITE, "s_init not finite"));
    if ((st = set_state(p, c, s0, pk_init[c], hs)) != MF_OK) return cleanup(st);
  }
  (void)vc;
  *out = p;
  return MF_OK;
}

mf_status mf_gibbs_sweep(mf_problem* p, int32_t n_sweeps, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (n_sweeps < 0) return fail(MF_E_INVALID_ARG, "negative sweep count");
  const mf_status room = check_sweep_room(p, n_sweeps);
  if (room != MF_OK) return room;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n_sweeps; ++i) {
    for (int k = 0; k < MF_NUM_KERNELS; ++k) {
      const mf_status st = launch_checked(p, kSweepOrder[k], 0, hs);
      if (st != MF_OK) return st;
    }
    ++p->sweep;
  }
  return MF_OK;
}

mf_status mf_mixing_sweep(mf_problem* p, int32_t n_sweeps, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (n_sweeps < 0) return fail(MF_E_INVALID_ARG, "negative sweep count");
  if (p->desc.n < 32 || p->desc.n > 256)
    return fail(MF_E_UNSUPPORTED_SIZE, "the mixing sweep supports grid sides 32 to 256 (got %d)",
                p->desc.n);
  // the mixing sweep's Metropolis-Hastings move is a move of P itself
  if (!p->desc.sample_pk)
    return fail(MF_E_INVALID_ARG, "mixing sweeps update P(k); the problem holds P fixed (sample_pk = 0)");
  const mf_status room = check_sweep_room(p, n_sweeps);
  if (room != MF_OK) return room;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const int ids[6] = {kZ, kYF, kXMixK, kMixPkK, kXMixInvK, kYI};
  for (int i = 0; i < n_sweeps; ++i) {
    for (int id : ids) {
      // the split path throughout; the inverse y-pass leaves P alone (the
      // Metropolis-Hastings move has set it and its table)
      const mf_status st = launch_checked(p, id, 0, hs, kPathSplit,
                                          id == kYI ? mf::kPkNone : mf::kPkDraw);
      if (st != MF_OK) return st;
    }
    ++p->sweep;
  }
  return MF_OK;
}

}  // extern "C"

namespace {

// Gibbs sweeps with kernel i mod MF_NUM_KERNELS of sweep i timed by one pair
// of events that skip the system-scope fence (a cache write-back and
// invalidate at every event would slow the kernels being timed).  With an
// eviction buffer, it is streamed through just before each timed kernel, so
// that the kernel starts with the fabric's last-level cache holding none of
// its data: mode 0 copies its first half onto its second half, mode 1 reads
// all of it, mode 2 does both (copy, then read).
mf_status timed_sweeps(mf_problem* p, int32_t n_sweeps, hipStream_t hs, double* kernel_ms,
                       int32_t n_kernels, void* evict, size_t evict_bytes, int evict_mode) {
  if (!p || !kernel_ms || n_kernels < 0) return fail(MF_E_INVALID_ARG, "bad argument");
  if (n_sweeps <= 0) return fail(MF_E_INVALID_ARG, "need at least one sweep");
  const mf_status room = check_sweep_room(p, n_sweeps);
  if (room != MF_OK) return room;
  const size_t half16 = evict_bytes / 32;   // 16-byte vectors per half
  // every event created is destroyed on every way out
  std::vector<hipEvent_t> ev;
  ev.reserve(static_cast<size_t>(n_sweeps) * 2);
  mf_status st = MF_OK;
  auto device_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == MF_OK) st = fail(MF_E_DEVICE, "%s failed: %s", what, hipGetErrorString(e));
    return st == MF_OK;
  };
  for (int i = 0; i < 2 * n_sweeps && st == MF_OK; ++i) {
    hipEvent_t e = nullptr;
    if (device_ok(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreateWithFlags"))
      ev.push_back(e);
  }
  for (int i = 0; i < n_sweeps && st == MF_OK; ++i) {
    const int timed = i % MF_NUM_KERNELS;
    for (int k = 0; k < MF_NUM_KERNELS && st == MF_OK; ++k) {
      if (k == timed && evict) {
        const auto* src = static_cast<const mf::v4u*>(evict);
        if (evict_mode != 1)
          hipLaunchKernelGGL(mf::stream_copy_kernel<false>, dim3(16384), dim3(mf::kStreamThreads),
                             0, hs, src, static_cast<mf::v4u*>(evict) + half16, half16);
        if (evict_mode != 0)   // one sum per workgroup lands in the buffer's first 16 KiB
          hipLaunchKernelGGL(mf::stream_read_kernel<false>, dim3(4096), dim3(mf::kStreamThreads),
                             0, hs, src + 1024, static_cast<uint32_t*>(evict), 2 * half16 - 1024);
        if (!device_ok(hipGetLastError(), "eviction stream launch")) break;
      }
      if (k == timed && !device_ok(hipEventRecord(ev[2 * i], hs), "hipEventRecord")) break;
      st = launch_checked(p, kSweepOrder[k], 0, hs);
      if (st == MF_OK && k == timed) device_ok(hipEventRecord(ev[2 * i + 1], hs), "hipEventRecord");
    }
    if (st == MF_OK) ++p->sweep;
  }
  if (st == MF_OK && device_ok(hipStreamSynchronize(hs), "hipStreamSynchronize")) {
    double sum[MF_NUM_KERNELS] = {0};
    int cnt[MF_NUM_KERNELS] = {0};
    for (int i = 0; i < n_sweeps && st == MF_OK; ++i) {
      float ms = 0.f;
      if (!device_ok(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]), "hipEventElapsedTime")) break;
      sum[i % MF_NUM_KERNELS] += ms;
      ++cnt[i % MF_NUM_KERNELS];
    }
    if (st == MF_OK)
      for (int k = 0; k < std::min<int>(n_kernels, MF_NUM_KERNELS); ++k)
        kernel_ms[k] = cnt[k] ? sum[k] / cnt[k] : std::numeric_limits<double>::quiet_NaN();
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return st;
}

}  // namespace

extern "C" {

mf_status mf_gibbs_sweep_timed(mf_problem* p, int32_t n_sweeps, void* stream, double* kernel_ms,
                               int32_t n_kernels) {
  return timed_sweeps(p, n_sweeps, static_cast<hipStream_t>(stream), kernel_ms, n_kernels,
                      nullptr, 0, 0);
}

mf_status mf_gibbs_sweep_timed_cold(mf_problem* p, int32_t n_sweeps, void* stream,
                                    double* kernel_ms, int32_t n_kernels, void* evict,
                                    size_t evict_bytes, int32_t evict_mode) {
  if (!evict || reinterpret_cast<uintptr_t>(evict) % 16 != 0 || evict_bytes < (64u << 20) ||
      evict_bytes % 32 != 0)
    return fail(MF_E_INVALID_ARG, "eviction buffer: 16-byte aligned, a multiple of 32 bytes, "
                "at least 64 MiB");
  if (evict_mode < 0 || evict_mode > 2) return fail(MF_E_INVALID_ARG, "evict_mode %d outside 0..2", evict_mode);
  return timed_sweeps(p, n_sweeps, static_cast<hipStream_t>(stream), kernel_ms, n_kernels,
                      evict, evict_bytes, evict_mode);
}

mf_status mf_get_chain_state(mf_problem* p, int32_t chain, double* s_out, double* pk_out,
                             uint64_t* sweep_out, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  if (s_out) {
    mf_status st = launch_checked(p, kZGet, chain, hs);
    if (st != MF_OK) return st;
    if ((st = download_real(p, s_out, p->ws + p->L.staging, m, hs)) != MF_OK) return st;
  }
  if (pk_out) {
    const int nb = p->desc.n_bins;
    MF_HIP(hipMemcpyAsync(pk_out, p->ws + p->L.pk + static_cast<size_t>(chain) * nb * 8, nb * 8,
                          hipMemcpyDeviceToHost, hs));
    MF_HIP(hipStreamSynchronize(hs));
    const double vc = std::pow(p->desc.box / p->desc.n, 3);
    for (int b = 0; b < nb; ++b) pk_out[b] *= vc;
  }
  uint32_t status = 0;
  MF_HIP(hipMemcpyAsync(&status, p->ws + p->L.status + chain * 4, 4, hipMemcpyDeviceToHost, hs));
  MF_HIP(hipStreamSynchronize(hs));
  if (sweep_out) *sweep_out = p->sweep;
  if (status) return fail(MF_E_NONFINITE, "chain %d: non-finite shell sum or P draw on device", chain);
  return MF_OK;
}

mf_status mf_set_chain_state(mf_problem* p, int32_t chain, const double* s, const double* pk,
                             uint64_t sweep, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  if (s)
    for (size_t i = 0; i < m; ++i)
      if (!std::isfinite(s[i])) return fail(MF_E_NONFINITE, "s not finite at %zu", i);
  const mf_status chk = check_sweep_index(sweep);
  if (chk != MF_OK) return chk;
  p->sweep = sweep;
  const mf_status st = write_counter(p, sweep, static_cast<hipStream_t>(stream));
  if (st != MF_OK) return st;
  return set_state(p, chain, s, pk, static_cast<hipStream_t>(stream));
}

namespace {
struct CheckpointHeader {
  char magic[8];        // "MFGIBBS1"
  int32_t n, n_bins, precision, reserved;
  uint64_t sweep;
};
size_t checkpoint_bytes(const mf_problem* p) {
  const size_t rs = p->fp64() ? 8 : 4;
  return sizeof(CheckpointHeader) + p->desc.n_bins * 8 + p->L.spec_elems * 2 * rs;
}
}  // namespace

mf_status mf_checkpoint_bytes(mf_problem* p, size_t* bytes) {
  if (!p || !bytes) return fail(MF_E_INVALID_ARG, "NULL argument");
  *bytes = checkpoint_bytes(p);
  return MF_OK;
}

mf_status mf_save_checkpoint(mf_problem* p, int32_t chain, void* buf, size_t bytes, void* stream) {
  if (!p || !buf) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  if (bytes < checkpoint_bytes(p)) return fail(MF_E_INVALID_ARG, "checkpoint buffer too small");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t rs = p->fp64() ? 8 : 4;
  CheckpointHeader h{};
  std::memcpy(h.magic, "MFGIBBS1", 8);
  h.n = p->desc.n;
  h.n_bins = p->desc.n_bins;
  h.precision = p->desc.precision;
  h.sweep = p->sweep;
  char* out = static_cast<char*>(buf);
  std::memcpy(out, &h, sizeof(h));
  const int nb = p->desc.n_bins;
  MF_HIP(hipMemcpyAsync(out + sizeof(h), p->ws + p->L.pk + static_cast<size_t>(chain) * nb * 8,
                        nb * 8, hipMemcpyDeviceToHost, hs));
  MF_HIP(hipMemcpyAsync(out + sizeof(h) + nb * 8,
                        p->ws + p->L.spec + static_cast<size_t>(chain) * p->L.spec_stride * 2 * rs,
                        p->L.spec_elems * 2 * rs, hipMemcpyDeviceToHost, hs));
  MF_HIP(hipStreamSynchronize(hs));
  return MF_OK;
}

mf_status mf_load_checkpoint(mf_problem* p, int32_t chain, const void* buf, size_t bytes,
                             void* stream) {
  if (!p || !buf) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  if (bytes < checkpoint_bytes(p)) return fail(MF_E_INVALID_ARG, "checkpoint buffer too small");
  CheckpointHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "MFGIBBS1", 8) != 0 || h.n != p->desc.n || h.n_bins != p->desc.n_bins ||
      h.precision != p->desc.precision)
    return fail(MF_E_INVALID_ARG, "checkpoint does not match this problem");
  if (check_sweep_index(h.sweep) != MF_OK) return MF_E_INVALID_ARG;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t rs = p->fp64() ? 8 : 4;
  const int nb = p->desc.n_bins;
  const char* in = static_cast<const char*>(buf);
  MF_HIP(hipMemcpyAsync(p->ws + p->L.pk + static_cast<size_t>(chain) * nb * 8, in + sizeof(h),
                        nb * 8, hipMemcpyHostToDevice, hs));
  MF_HIP(hipMemcpyAsync(p->ws + p->L.spec + static_cast<size_t>(chain) * p->L.spec_stride * 2 * rs,
                        in + sizeof(h) + nb * 8, p->L.spec_elems * 2 * rs, hipMemcpyHostToDevice, hs));
  MF_HIP(hipStreamSynchronize(hs));
  mf_status st = launch_checked(p, kTable, chain, hs);
  if (st != MF_OK) return st;
  p->sweep = h.sweep;
  return write_counter(p, h.sweep, hs);
}

mf_status mf_set_x_path(mf_problem* p, int32_t path) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (path != kPathSplit && path != kPathWhole) return fail(MF_E_INVALID_ARG, "unknown path %d", path);
  if (path == kPathSplit && (p->desc.n < 32 || p->desc.n > 256))
    return fail(MF_E_UNSUPPORTED_SIZE, "the split x transform needs 32 <= N <= 256");
  p->xpath = path;
  return MF_OK;
}

mf_status mf_get_x_path(const mf_problem* p, int32_t* path) {
  if (!p || !path) return fail(MF_E_INVALID_ARG, "NULL argument");
  *path = p->xpath;
  return MF_OK;
}

mf_status mf_set_tuning(mf_problem* p, const mf_tuning* t) {
  if (!p || !t) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (t->x_tile < 0 || t->x_tile >= kTileVariants || t->y_group < 0 || t->y_group >= kTileVariants)
    return fail(MF_E_INVALID_ARG, "tile variants must be 0..%d", kTileVariants - 1);
  if (t->y_radix != 0 && t->y_radix != 1)
    return fail(MF_E_INVALID_ARG, "y_radix must be 0 (schedule order) or 1 (reversed)");
  if (t->x_path == kPathSplit && p->desc.n >= 32 && p->desc.n <= 256 &&
      p->desc.n_bins > p->sh.x_max_bins[t->x_tile])
    return fail(MF_E_INVALID_ARG, "x tile %d holds histograms for at most %d bins (problem has %d)",
                t->x_tile, p->sh.x_max_bins[t->x_tile], p->desc.n_bins);
  const mf_status st = mf_set_x_path(p, t->x_path);
  if (st != MF_OK) return st;
  p->xvar = t->x_tile;
  p->yvar = t->y_group;
  p->yrad = t->y_radix;
  return MF_OK;
}

mf_status mf_get_tuning(const mf_problem* p, mf_tuning* t) {
  if (!p || !t) return fail(MF_E_INVALID_ARG, "NULL argument");
  t->x_path = p->xpath;
  t->x_tile = p->xvar;
  t->y_group = p->yvar;
  const bool split = p->xpath == kPathSplit;
  t->x_cols = split ? p->sh.x_cols[p->xvar] : 0;
  t->x_k1 = split ? p->sh.x_k1[p->xvar] : 0;
  t->x_hist = split ? p->sh.x_hist[p->xvar] : 0;
  t->y_units = split ? p->sh.y_units[p->yvar] : 0;
  t->y_radix = split ? p->yrad : 0;
  return MF_OK;
}

}  // extern "C"

namespace {

// Mean ms of `trials` Gibbs sweeps (after one warm-up sweep) with the given
// choices; restores nothing (the caller saved the chains).
mf_status time_choice(mf_problem* p, int path, int xv, int yv, int yr, int trials, void* stream,
                      hipEvent_t e0, hipEvent_t e1, double* ms) {
  hipStream_t hs = static_cast<hipStream_t>(stream);
  p->xpath = path;
  p->xvar = xv;
  p->yvar = yv;
  p->yrad = yr;
  mf_status st = mf_gibbs_sweep(p, 1, stream);
  if (st != MF_OK) return st;
  MF_HIP(hipEventRecord(e0, hs));
  if ((st = mf_gibbs_sweep(p, trials, stream)) != MF_OK) return st;
  MF_HIP(hipEventRecord(e1, hs));
  MF_HIP(hipEventSynchronize(e1));
  float t = 0.f;
  MF_HIP(hipEventElapsedTime(&t, e0, e1));
  *ms = t / trials;
  return MF_OK;
}

}  // namespace

extern "C" {

// Rounds of the autotuner's search: each stage times its candidates in turn,
// this many times, and keeps every candidate's fastest round; an alternative
// replaces the incumbent only when it is faster by more than kTuneMargin.
constexpr int kTuneRounds = 3;
constexpr double kTuneMargin = 0.01;

mf_status mf_autotune(mf_problem* p, int32_t trials, void* stream, double* ms, mf_tuning* picked) {
  if (!p || !ms) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (trials < 1) return fail(MF_E_INVALID_ARG, "need at least one trial sweep");
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int i = 0; i < MF_TUNE_SLOTS; ++i) ms[i] = nan;
  const bool can_split = p->desc.n >= 32 && p->desc.n <= 256;
  if (!can_split) {
    p->xpath = kPathWhole;
    p->xvar = p->default_xvar();
    p->yvar = 0;
    p->yrad = 0;
    return picked ? mf_get_tuning(p, picked) : MF_OK;
  }
  // every candidate's sweeps must fit below the 2^32 sweep-index bound; the
  // chains are restored afterwards
  const int warm = std::max<int>(trials, 20);
  const int64_t budget = static_cast<int64_t>(kTuneRounds) * 10 * (trials + 1) + warm;
  mf_status st = check_sweep_room(p, budget);
  if (st != MF_OK) return st;
  // Save every chain (spectrum, P, sweep index) and switch recording off, so
  // the trial sweeps leave no trace.
  const size_t cb = checkpoint_bytes(p);
  std::vector<std::vector<char>> saved(p->desc.n_chains, std::vector<char>(cb));
  for (int c = 0; c < p->desc.n_chains && st == MF_OK; ++c)
    st = mf_save_checkpoint(p, c, saved[c].data(), cb, stream);
  if (st != MF_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MF_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MF_E_DEVICE, "hipEventCreate failed");
  }
  const DiagRec diag = p->diag;
  const int path0 = p->xpath, xv0 = p->xvar, yv0 = p->yvar, yr0 = p->yrad;
  p->diag = DiagRec{};
  // candidates of a stage: (path, x tile, y group, y radix order, slot);
  // fastest round kept
  struct Cand { int path, xv, yv, yr, slot; };
  auto run_stage = [&](const std::vector<Cand>& cands) {
    for (int r = 0; r < kTuneRounds && st == MF_OK; ++r)
      for (const Cand& c : cands) {
        double t = 0.0;
        st = time_choice(p, c.path, c.xv, c.yv, c.yr, trials, stream, e0, e1, &t);
        if (st != MF_OK) return;
        if (!(ms[c.slot] <= t)) ms[c.slot] = t;   // NaN or slower: replace
      }
  };
  // index of the fastest candidate; the first (incumbent) wins ties and
  // margins below kTuneMargin
  auto pick = [&](const std::vector<Cand>& cands) {
    int best = 0;
    for (int i = 1; i < static_cast<int>(cands.size()); ++i)
      if (ms[cands[i].slot] < ms[cands[best].slot] * (1.0 - kTuneMargin)) best = i;
    return best;
  };
  p->xpath = kPathSplit;
  p->xvar = p->default_xvar();
  p->yvar = 0;
  p->yrad = 0;
  st = mf_gibbs_sweep(p, warm, stream);   // device warm-up
  // 1. x tiles on the split path, y group 0
  std::vector<Cand> xs;
  for (int v = 0; v < kTileVariants; ++v)
    if (p->desc.n_bins <= p->sh.x_max_bins[v]) xs.push_back({kPathSplit, v, 0, 0, 2 + v});
  run_stage(xs);
  const int best_x = st == MF_OK ? xs[pick(xs)].xv : 0;
  // 2. y groups with the best x tile (groups of equal size are timed once)
  std::vector<Cand> ys{{kPathSplit, best_x, 0, 0, 5}};
  for (int v = 1; v < kTileVariants; ++v)
    if (p->sh.y_units[v] != p->sh.y_units[v - 1]) ys.push_back({kPathSplit, best_x, v, 0, 5 + v});
  if (st == MF_OK) run_stage(ys);
  const int best_y = st == MF_OK ? ys[pick(ys)].yv : 0;
  // 3. the y transform's radix schedule in order or reversed, where the two
  // differ
  int best_r = 0;
  if (st == MF_OK && p->sh.y_rev_distinct) {
    std::vector<Cand> rs{{kPathSplit, best_x, best_y, 0, 8}, {kPathSplit, best_x, best_y, 1, 9}};
    run_stage(rs);
    if (st == MF_OK) best_r = rs[pick(rs)].yr;
  }
  // 4. the split path so tuned against the whole-pencil path
  std::vector<Cand> paths{{kPathSplit, best_x, best_y, best_r, 0}, {kPathWhole, 0, 0, 0, 1}};
  if (st == MF_OK) run_stage(paths);
  const bool whole = st == MF_OK && pick(paths) == 1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->diag = diag;
  p->xpath = path0;
  p->xvar = xv0;
  p->yvar = yv0;
  p->yrad = yr0;
  for (int c = 0; c < p->desc.n_chains; ++c) {
    const mf_status r = mf_load_checkpoint(p, c, saved[c].data(), cb, stream);
    if (st == MF_OK) st = r;
  }
  if (st != MF_OK) return st;
  p->xpath = whole ? kPathWhole : kPathSplit;
  p->xvar = whole ? p->default_xvar() : best_x;
  p->yvar = whole ? 0 : best_y;
  p->yrad = whole ? 0 : best_r;
  return picked ? mf_get_tuning(p, picked) : MF_OK;
}

mf_status mf_sweep_bytes(const mf_problem* p, size_t* bytes) {
  if (!p || !bytes) return fail(MF_E_INVALID_ARG, "NULL argument");
  const size_t rs = p->fp64() ? 8 : 4, n = p->desc.n, m = n * n * n, nb = p->desc.n_bins;
  const size_t spec = (n / 2 + 1) * n * n * 2 * rs;
  const size_t part = static_cast<size_t>(p->n_wg(p->xpath, p->xvar)) * nb * 8;
  for (int k = 0; k < MF_NUM_KERNELS; ++k) bytes[k] = 0;
  for (int c = 0; c < p->desc.n_chains; ++c) {
    const size_t coef = 2 * m * rs * static_cast<size_t>(p->obs_chunks[c]) / (p->sh.ztiles * p->sh.zept);
    bytes[0] += 2 * spec + coef;
    bytes[1] += 2 * spec;
    bytes[2] += 2 * spec + part;
    bytes[3] += 2 * spec + part + nb * (16 + 2 * rs);
  }
  return MF_OK;
}

mf_status mf_get_tau(mf_problem* p, int32_t chain, double* tau_out) {
  if (!p || !tau_out) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  *tau_out = p->tau[chain];
  return MF_OK;
}

mf_status mf_debug_run_kernel(mf_problem* p, int32_t kernel, uint64_t sweep, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (kernel < 0 || kernel >= MF_NUM_KERNELS) return fail(MF_E_INVALID_ARG, "bad kernel id");
  if (check_sweep_index(sweep) != MF_OK) return MF_E_INVALID_ARG;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const mf_status st = write_counter(p, sweep, hs);
  if (st != MF_OK) return st;
  return launch_checked(p, kSweepOrder[kernel], 0, hs);
}

mf_status mf_debug_spectrum(mf_problem* p, int32_t chain, double* buf, int32_t to_device,
                            void* stream) {
  if (!p || !buf) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t count = 2 * p->L.spec_elems;
  const size_t rs = p->fp64() ? 8 : 4;
  char* dev = p->ws + p->L.spec + static_cast<size_t>(chain) * p->L.spec_stride * 2 * rs;
  if (to_device) return upload_real(p, dev, buf, count, hs);
  return download_real(p, buf, dev, count, hs);
}

void mf_destroy_problem(mf_problem* p) { delete p; }

}  // extern "C"

struct mf_graph {
  std::vector<mf_problem*> probs;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool counted = false;   // probs' graph counts include this graph
  ~mf_graph() {
    if (counted)
      for (auto* p : probs) --p->graphs;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto s : side) (void)hipStreamDestroy(s);
  }
};

extern "C" {

mf_status mf_graph_create(mf_problem* const* problems, int32_t n, void* stream, mf_graph** out) {
  if (!out) return fail(MF_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!problems || n < 1) return fail(MF_E_INVALID_ARG, "need at least one problem");
  for (int i = 0; i < n; ++i)
    if (!problems[i]) return fail(MF_E_INVALID_ARG, "problem %d is NULL", i);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  mf_graph* g = new mf_graph{};
  g->probs.assign(problems, problems + n);
  auto bail = [&](const char* what, hipError_t e) {
    delete g;
    return fail(MF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  for (int i = 0; i < n; ++i) {
    hipStream_t s2;
    if ((e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking)) != hipSuccess)
      return bail("hipStreamCreateWithFlags", e);
    g->side.push_back(s2);
  }
  for (int i = 0; i < n + 1; ++i) {
    hipEvent_t ev;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return bail("hipEventCreate", e);
    g->events.push_back(ev);
  }
  // Capture on a stream of the graph's own (the caller's may be the legacy
  // default stream, which cannot be captured); replays go to the caller's.
  (void)hs;
  hipStream_t cap;
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
    return bail("hipStreamCreateWithFlags", e);
  g->side.push_back(cap);
  hs = cap;
  if ((e = hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return bail("hipStreamBeginCapture", e);
  mf_status st = MF_OK;
  (void)hipEventRecord(g->events[n], hs);             // fork point
  for (int i = 0; i < n && st == MF_OK; ++i) {
    hipStream_t s2 = g->side[i];
    (void)hipStreamWaitEvent(s2, g->events[n], 0);
    for (int k = 0; k < MF_NUM_KERNELS && st == MF_OK; ++k)
      st = launch_checked(problems[i], kSweepOrder[k], 0, s2);
    (void)hipEventRecord(g->events[i], s2);
    (void)hipStreamWaitEvent(hs, g->events[i], 0);     // join
  }
  e = hipStreamEndCapture(hs, &g->graph);
  if (st != MF_OK) {
    delete g;
    return st;
  }
  if (e != hipSuccess) return bail("hipStreamEndCapture", e);
  if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
    return bail("hipGraphInstantiate", e);
  // the graph holds the diagnostic buffers' addresses as captured
  for (auto* p : g->probs) ++p->graphs;
  g->counted = true;
  *out = g;
  return MF_OK;
}

mf_status mf_graph_launch(mf_graph* g, int32_t n_sweeps, void* stream) {
  if (!g) return fail(MF_E_INVALID_ARG, "graph is NULL");
  if (n_sweeps < 0) return fail(MF_E_INVALID_ARG, "negative sweep count");
  for (auto* p : g->probs) {
    const mf_status room = check_sweep_room(p, n_sweeps);
    if (room != MF_OK) return room;
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n_sweeps; ++i) MF_HIP(hipGraphLaunch(g->exec, hs));
  for (auto* p : g->probs) p->sweep += static_cast<uint64_t>(n_sweeps);
  return MF_OK;
}

void mf_graph_destroy(mf_graph* g) { delete g; }

const char* mf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------- Wiener filter
namespace {

// Wiener workspace for nc chains processed together; every buffer holds the
// chains one after another, each 256-byte aligned.
struct WLayout {
  size_t partial, pkg, gacc, table, wcoef, fwd, adj, ckpt, aux, acc, dr, total;
  size_t spec_bytes;   // one chain's spectrum (with the problem's stride)
  int nblk, n_ckpt, nc;
};

WLayout wiener_layout(const mf_problem* p, int n_iter, int every, int nc) {
  const size_t rs = p->fp64() ? 8 : 4;
  const size_t n = p->desc.n, m = n * n * n, nb = p->desc.n_bins;
  WLayout W{};
  W.nc = nc;
  W.nblk = static_cast<int>((m / 2 + mf::kWienerThreads - 1) / mf::kWienerThreads);
  W.n_ckpt = (n_iter + every - 1) / every;
  W.spec_bytes = p->L.spec_stride * 2 * rs;
  const size_t specs = static_cast<size_t>(nc) * W.spec_bytes;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  W.partial = take(static_cast<size_t>(nc) * W.nblk * 8);
  W.pkg = take(nc * nb * 8);
  W.gacc = take(nc * nb * 8);
  W.table = take(nc * nb * 2 * rs);
  W.wcoef = take(nc * 2 * m * rs);
  W.fwd = take(specs);
  W.adj = take(specs);
  W.ckpt = take(static_cast<size_t>(W.n_ckpt) * specs);
  W.aux = take(static_cast<size_t>(every) * specs);
  W.acc = take(nc * m * rs);
  W.dr = take(p->desc.has_response ? nc * m * 8 : 0);   // d / R
  W.total = off;
  return W;
}

// chain = -1: all chains of the problem; else that one chain.
mf_status wiener_chains(const mf_problem* p, int chain, int* c0, int* nc) {
  if (chain == -1) {
    *c0 = 0;
    *nc = p->desc.n_chains;
    return MF_OK;
  }
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  *c0 = chain;
  *nc = 1;
  return MF_OK;
}

mf_status check_wiener(const mf_problem* p, int chain, int n_iter, int every, const void* gws,
                       size_t gws_bytes, WLayout* W, int* c0) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (p->desc.n < 32 || p->desc.n > 256)
    return fail(MF_E_UNSUPPORTED_SIZE, "the Wiener iteration supports grid sides 32 to 256 (got %d)",
                p->desc.n);
  int nc = 0;
  mf_status r = wiener_chains(p, chain, c0, &nc);
  if (r != MF_OK) return r;
  if (n_iter < 1 || every < 1 || every > n_iter)
    return fail(MF_E_INVALID_ARG, "need n_iter >= 1 and 1 <= ckpt_every <= n_iter");
  *W = wiener_layout(p, n_iter, every, nc);
  if (!gws || reinterpret_cast<uintptr_t>(gws) % kAlign != 0)
    return fail(MF_E_WORKSPACE, "Wiener workspace NULL or not 256-byte aligned");
  if (gws_bytes < W->total)
    return fail(MF_E_WORKSPACE, "Wiener workspace too small: %zu < %zu", gws_bytes, W->total);
  return MF_OK;
}

template <typename F>
void with_n(int n, F&& f) {
  switch (n) {
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 48: f(std::integral_constant<int, 48>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 80: f(std::integral_constant<int, 80>{}); break;
    case 96: f(std::integral_constant<int, 96>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    default: break;
  }
}

// o = tau R^2 / N of problem chain c, z-pass entry order.
template <typename R>
const R* omw_of(const mf_problem* p, int c) {
  const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  return reinterpret_cast<const R*>(p->ws + p->L.omw) + static_cast<size_t>(c) * m;
}

// Sweep arguments of the deterministic iteration of chains c0 .. c0 + nc - 1
// (grid z = nc; chain c of the launch is problem chain c0 + c).
template <typename R>
mf::SweepArgs<R> wiener_args(const mf_problem* p, int c0, const R* coef, R* table, double* pkg,
                             double* gacc) {
  mf::SweepArgs<R> a = args_of<R>(p, kPathSplit, 1);
  a.coef = coef;
  a.table = table;
  a.pk = pkg;
  a.gacc = gacc;
  a.tau = reinterpret_cast<const double*>(p->ws + p->L.tau) + c0;
  a.status = reinterpret_cast<uint32_t*>(p->ws + p->L.status) + c0;
  a.tile_obs = reinterpret_cast<const uint32_t*>(p->ws + p->L.tobs) + static_cast<size_t>(c0) * p->sh.ztiles;
  a.chain0 = p->desc.chain_id + c0;
  a.advance = 0;
  a.staging_chain = 0;
  a.trace = nullptr;
  a.mom = nullptr;
  return a;
}

template <typename R>
mf::SweepArgs<R> wiener_args(const mf_problem* p, int c0, char* g, const WLayout& W) {
  return wiener_args<R>(p, c0, reinterpret_cast<const R*>(g + W.wcoef),
                        reinterpret_cast<R*>(g + W.table), reinterpret_cast<double*>(g + W.pkg),
                        reinterpret_cast<double*>(g + W.gacc));
}

mf_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MF_E_DEVICE, "%s launch failed: %s", what, hipGetErrorString(e));
  return MF_OK;
}

// One iteration s' = C (cs alpha s + cb beta) of every chain on `spec`.
// Forward (adj = false): t^ goes to aux when aux is set.  Adjoint (adj =
// true): the per-bin sums of Re(conj(t^) aux) are added to gacc, and s is
// added to acc when set.
template <typename R>
mf_status wiener_iter(mf_problem* p, mf::SweepArgs<R> a, int nc, mf::cx<R>* spec, mf::cx<R>* aux,
                      bool adj, R cs, R cb, R* acc, hipStream_t st) {
  a.spec = spec;
  a.aux = aux;
  a.acc = acc;
  a.cs = cs;
  a.cb = cb;
  a.pk_mode = adj ? mf::kPkGrad : mf::kPkNone;
  const int ids[4] = {kZDetK, kYF, adj ? kXAdjK : kXDetK, kYI};
  for (int id : ids) {
    launch<R>(id, a, p->desc.n, nc, st);
    const mf_status r = check_launch("Wiener iteration");
    if (r != MF_OK) return r;
  }
  return MF_OK;
}

// y = x / R for chains c0 .. c0 + nc - 1 (y may be x).  A problem with a
// response R is the problem with data d / R and noise N / R^2, voxel by
// voxel: the iteration, s_K and chi2_K coincide, and d chi2 / d d is
// d chi2 / d (d / R) divided by R.
void scale_by_rinv(const mf_problem* p, int c0, int nc, const double* x, double* y, hipStream_t st) {
  const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  const double* rinv = reinterpret_cast<const double*>(p->ws + p->L.rinv) + static_cast<size_t>(c0) * m;
  hipLaunchKernelGGL(mf::scale_kernel, dim3(1024), dim3(256), 0, st, x, rinv, y,
                     static_cast<size_t>(nc) * m);
}

template <typename R>
mf_status wiener_forward(mf_problem* p, int c0, const double* d, const double* pk, int n_iter,
                         int every, char* g, const WLayout& W, double* chi2, double* s_out,
                         hipStream_t st) {
  const int n = p->desc.n, nb = p->desc.n_bins, nc = W.nc;
  const size_t m = static_cast<size_t>(n) * n * n, entries = m / 2;
  if (p->desc.has_response) {
    double* dr = reinterpret_cast<double*>(g + W.dr);
    scale_by_rinv(p, c0, nc, d, dr, st);
    d = dr;
  }
  const double vcell = std::pow(p->desc.box / n, 3);
  auto a = wiener_args<R>(p, c0, g, W);
  const size_t specs = static_cast<size_t>(nc) * W.spec_bytes;
  for (int c = 0; c < nc; ++c) {
    const R* coef = reinterpret_cast<const R*>(p->ws + p->L.coef) + static_cast<size_t>(c0 + c) * 2 * m;
    R* wcoef = reinterpret_cast<R*>(g + W.wcoef) + static_cast<size_t>(c) * 2 * m;
    with_n(n, [&](auto nn) {
      constexpr int N = decltype(nn)::value;
      hipLaunchKernelGGL((mf::wiener_coef_kernel<R, N>), dim3(W.nblk), dim3(mf::kWienerThreads), 0,
                         st, coef, omw_of<R>(p, c0 + c), wcoef, d + c * m, entries);
    });
    hipLaunchKernelGGL((mf::wiener_table_kernel<R>), dim3((nb + 63) / 64), dim3(64), 0, st,
                       pk + c * nb, reinterpret_cast<double*>(g + W.pkg) + c * nb,
                       reinterpret_cast<R*>(g + W.table) + c * 2 * nb, p->tau[c0 + c], vcell,
                       static_cast<double>(m), nb);
  }
  hipLaunchKernelGGL((mf::fill_zero_kernel<R>), dim3(1024), dim3(256), 0, st,
                     reinterpret_cast<R*>(g + W.fwd), specs / sizeof(R));
  mf_status r = check_launch("Wiener set-up");
  if (r != MF_OK) return r;
  auto* fwd = reinterpret_cast<mf::cx<R>*>(g + W.fwd);
  for (int k = 0; k < n_iter; ++k) {
    if (k % every == 0)
      MF_HIP(hipMemcpyAsync(g + W.ckpt + static_cast<size_t>(k / every) * specs, fwd, specs,
                            hipMemcpyDeviceToDevice, st));
    if ((r = wiener_iter<R>(p, a, nc, fwd, nullptr, false, R(1), R(1), nullptr, st)) != MF_OK)
      return r;
  }
  const R* s = reinterpret_cast<const R*>(p->ws + p->L.staging);
  for (int c = 0; c < nc; ++c) {   // s_K of chain c through the state staging buffer
    auto ag = a;
    ag.spec = fwd;
    ag.staging_chain = c;
    launch<R>(kZGet, ag, n, 1, st);
    with_n(n, [&](auto nn) {
      constexpr int N = decltype(nn)::value;
      hipLaunchKernelGGL((mf::wiener_chi2_kernel<R, N>), dim3(W.nblk), dim3(mf::kWienerThreads), 0,
                         st, omw_of<R>(p, c0 + c), d + c * m, s,
                         p->tau[c0 + c], reinterpret_cast<double*>(g + W.partial) + c * W.nblk,
                         s_out ? s_out + c * m : nullptr, entries);
    });
    hipLaunchKernelGGL(mf::sum_partials_kernel, dim3(1), dim3(mf::kWienerThreads), 0, st,
                       reinterpret_cast<const double*>(g + W.partial) + c * W.nblk, W.nblk, chi2 + c);
  }
  return check_launch("Wiener chi2");
}

template <typename R>
mf_status wiener_backward(mf_problem* p, int c0, const double* d, char* g, const WLayout& W,
                          double* grad_d, double* grad_pk, hipStream_t st) {
  const int n = p->desc.n, nb = p->desc.n_bins, nc = W.nc;
  const int n_iter = p->wiener.n_iter, every = p->wiener.every;
  const size_t m = static_cast<size_t>(n) * n * n, entries = m / 2;
  const double vcell = std::pow(p->desc.box / n, 3);
  auto a = wiener_args<R>(p, c0, g, W);
  const size_t specs = static_cast<size_t>(nc) * W.spec_bytes;
  auto* fwd = reinterpret_cast<mf::cx<R>*>(g + W.fwd);
  auto* adj = reinterpret_cast<mf::cx<R>*>(g + W.adj);
  R* acc = reinterpret_cast<R*>(g + W.acc);
  auto slot = [&](int j) { return reinterpret_cast<mf::cx<R>*>(g + W.aux + static_cast<size_t>(j) * specs); };
  const R* s = reinterpret_cast<const R*>(p->ws + p->L.staging);
  if (p->desc.has_response) {
    double* dr = reinterpret_cast<double*>(g + W.dr);
    scale_by_rinv(p, c0, nc, d, dr, st);
    d = dr;
  }
  hipLaunchKernelGGL((mf::fill_zero_kernel<double>), dim3(1), dim3(256), 0, st,
                     reinterpret_cast<double*>(g + W.gacc), static_cast<size_t>(nc) * nb);
  hipLaunchKernelGGL((mf::fill_zero_kernel<R>), dim3(1024), dim3(256), 0, st, acc, nc * m);
  hipLaunchKernelGGL((mf::fill_zero_kernel<R>), dim3(1024), dim3(256), 0, st,
                     reinterpret_cast<R*>(adj), specs / sizeof(R));
  mf_status r = check_launch("Wiener adjoint set-up");
  if (r != MF_OK) return r;
  for (int sg = W.n_ckpt - 1; sg >= 0; --sg) {
    const int k0 = sg * every, k1 = std::min(n_iter, k0 + every);
    MF_HIP(hipMemcpyAsync(fwd, g + W.ckpt + static_cast<size_t>(sg) * specs, specs,
                          hipMemcpyDeviceToDevice, st));
    for (int k = k0; k < k1; ++k)
      if ((r = wiener_iter<R>(p, a, nc, fwd, slot(k - k0), false, R(1), R(1), nullptr, st)) != MF_OK)
        return r;
    if (sg == W.n_ckpt - 1) {   // fwd holds s_K: the direct term w (2 d - s_K) of d chi2 / d d
      for (int c = 0; c < nc; ++c) {
        auto ag = a;
        ag.spec = fwd;
        ag.staging_chain = c;
        launch<R>(kZGet, ag, n, 1, st);
        with_n(n, [&](auto nn) {
          constexpr int N = decltype(nn)::value;
          hipLaunchKernelGGL((mf::wiener_grad_direct_kernel<R, N>), dim3(W.nblk),
                             dim3(mf::kWienerThreads), 0, st, omw_of<R>(p, c0 + c), d + c * m, s,
                             p->tau[c0 + c], grad_d + c * m, entries);
        });
      }
    }
    for (int k = k1 - 1; k >= k0; --k) {
      // step k maps g_{k+1} to r_k = C g_{k+1}: g_K = -w d = -beta / tau (of
      // each chain), and g_{k+1} = alpha r_{k+1} otherwise (r_{k+1} then
      // joins the sum)
      if (k == n_iter - 1) {
        auto af = a;
        af.cb_over_tau = 1;
        r = wiener_iter<R>(p, af, nc, adj, slot(k - k0), true, R(0), R(-1), nullptr, st);
      } else {
        r = wiener_iter<R>(p, a, nc, adj, slot(k - k0), true, R(1), R(0), acc, st);
      }
      if (r != MF_OK) return r;
    }
  }
  a.spec = adj;
  a.acc = acc;
  launch<R>(kZAccK, a, n, nc, st);   // adds r_0
  for (int c = 0; c < nc; ++c) {
    with_n(n, [&](auto nn) {
      constexpr int N = decltype(nn)::value;
      hipLaunchKernelGGL((mf::wiener_grad_adjoint_kernel<R, N>), dim3(W.nblk),
                         dim3(mf::kWienerThreads), 0, st, omw_of<R>(p, c0 + c), acc + c * m,
                         grad_d + c * m, entries);
    });
    hipLaunchKernelGGL(mf::wiener_grad_pk_kernel, dim3((nb + 63) / 64), dim3(64), 0, st,
                       reinterpret_cast<const double*>(g + W.gacc) + c * nb,
                       reinterpret_cast<const double*>(g + W.pkg) + c * nb, p->tau[c0 + c], vcell,
                       nb, grad_pk + c * nb);
  }
  if (p->desc.has_response) scale_by_rinv(p, c0, nc, grad_d, grad_d, st);
  return check_launch("Wiener gradient");
}

}  // namespace

extern "C" {

mf_status mf_wiener_workspace_bytes(const mf_problem* p, int32_t chain, int32_t n_iter,
                                    int32_t ckpt_every, size_t* bytes) {
  if (!p || !bytes) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (n_iter < 1 || ckpt_every < 1 || ckpt_every > n_iter)
    return fail(MF_E_INVALID_ARG, "need n_iter >= 1 and 1 <= ckpt_every <= n_iter");
  int c0 = 0, nc = 0;
  const mf_status r = wiener_chains(p, chain, &c0, &nc);
  if (r != MF_OK) return r;
  *bytes = wiener_layout(p, n_iter, ckpt_every, nc).total;
  return MF_OK;
}

mf_status mf_wiener_forward(mf_problem* p, int32_t chain, const double* d, const double* pk,
                            int32_t n_iter, int32_t ckpt_every, void* workspace, size_t ws_bytes,
                            double* chi2, double* s_out, void* stream) {
  WLayout W{};
  int c0 = 0;
  mf_status r = check_wiener(p, chain, n_iter, ckpt_every, workspace, ws_bytes, &W, &c0);
  if (r != MF_OK) return r;
  if (!d || !pk || !chi2) return fail(MF_E_INVALID_ARG, "d, pk and chi2 must be device pointers");
  p->wiener = WienerRun{};
  hipStream_t hs = static_cast<hipStream_t>(stream);
  char* g = static_cast<char*>(workspace);
  r = p->fp64() ? wiener_forward<double>(p, c0, d, pk, n_iter, ckpt_every, g, W, chi2, s_out, hs)
                : wiener_forward<float>(p, c0, d, pk, n_iter, ckpt_every, g, W, chi2, s_out, hs);
  if (r == MF_OK) p->wiener = WienerRun{workspace, chain, n_iter, ckpt_every};
  return r;
}

mf_status mf_wiener_backward(mf_problem* p, int32_t chain, const double* d, void* workspace,
                             size_t ws_bytes, double* grad_d, double* grad_pk, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (p->wiener.gws == nullptr || p->wiener.gws != workspace || p->wiener.chain != chain)
    return fail(MF_E_STATE, "no Wiener forward run of chain %d with this workspace", chain);
  WLayout W{};
  int c0 = 0;
  mf_status r = check_wiener(p, chain, p->wiener.n_iter, p->wiener.every, workspace, ws_bytes, &W, &c0);
  if (r != MF_OK) return r;
  if (!d || !grad_d || !grad_pk) return fail(MF_E_INVALID_ARG, "d, grad_d and grad_pk must be device pointers");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  char* g = static_cast<char*>(workspace);
  return p->fp64() ? wiener_backward<double>(p, c0, d, g, W, grad_d, grad_pk, hs)
                   : wiener_backward<float>(p, c0, d, g, W, grad_d, grad_pk, hs);
}

}  // extern "C"

// ---------------------------------------------------------------- log-determinant trace
namespace {

// Workspace of the trace estimator for nc chains: the filter table, two sets
// of bin sums, the probe coefficients and four spectra (s_K, s_{K-1}, the
// transform of beta_z, scratch).
struct LLayout {
  size_t pkg, table, g1, g0, wcoef, fwd, prev, aux, scr, total;
  size_t specs;   // bytes of nc spectra
  int nc;
};

LLayout logdet_layout(const mf_problem* p, int nc) {
  const size_t rs = p->fp64() ? 8 : 4;
  const size_t n = p->desc.n, m = n * n * n, nb = p->desc.n_bins;
  LLayout L{};
  L.nc = nc;
  L.specs = static_cast<size_t>(nc) * p->L.spec_stride * 2 * rs;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.pkg = take(nc * nb * 8);
  L.table = take(nc * nb * 2 * rs);
  L.g1 = take(nc * nb * 8);
  L.g0 = take(nc * nb * 8);
  L.wcoef = take(nc * 2 * m * rs);
  L.fwd = take(L.specs);
  L.prev = take(L.specs);
  L.aux = take(L.specs);
  L.scr = take(L.specs);
  L.total = off;
  return L;
}

// One probe j: K iterations on beta_z from s_0 = 0 (s_{K-1} kept), the
// transform b^ of beta_z stored by a pass with t = beta_z, then the bin sums
// G1 = (1/M) sum Re(conj(t^_K) b^) and G0 (the same with t_{K-1}) from two
// adjoint-mode passes; T_b += (G1 - f G0) / (tau^2 V_cell) / n_probes.
template <typename R>
mf_status logdet_run(mf_problem* p, int c0, const double* pk, int n_iter, int n_probes,
                     uint32_t probe0, char* g, const LLayout& L, double* out, hipStream_t st) {
  const int n = p->desc.n, nb = p->desc.n_bins, nc = L.nc;
  const size_t m = static_cast<size_t>(n) * n * n, entries = m / 2;
  const double vcell = std::pow(p->desc.box / n, 3);
  const int nblk = static_cast<int>((entries + mf::kWienerThreads - 1) / mf::kWienerThreads);
  R* wcoef = reinterpret_cast<R*>(g + L.wcoef);
  double* pkg = reinterpret_cast<double*>(g + L.pkg);
  double* g1 = reinterpret_cast<double*>(g + L.g1);
  double* g0 = reinterpret_cast<double*>(g + L.g0);
  auto a = wiener_args<R>(p, c0, wcoef, reinterpret_cast<R*>(g + L.table), pkg, g1);
  auto a0 = a;
  a0.gacc = g0;
  auto* fwd = reinterpret_cast<mf::cx<R>*>(g + L.fwd);
  auto* prev = reinterpret_cast<mf::cx<R>*>(g + L.prev);
  auto* aux = reinterpret_cast<mf::cx<R>*>(g + L.aux);
  auto* scr = reinterpret_cast<mf::cx<R>*>(g + L.scr);
  for (int c = 0; c < nc; ++c)
    hipLaunchKernelGGL((mf::wiener_table_kernel<R>), dim3((nb + 63) / 64), dim3(64), 0, st,
                       pk + c * nb, pkg + c * nb, reinterpret_cast<R*>(g + L.table) + c * 2 * nb,
                       p->tau[c0 + c], vcell, static_cast<double>(m), nb);
  hipLaunchKernelGGL((mf::fill_zero_kernel<double>), dim3(1), dim3(256), 0, st, out,
                     static_cast<size_t>(nc) * nb);
  mf_status r = check_launch("log-determinant set-up");
  if (r != MF_OK) return r;
  for (int j = 0; j < n_probes; ++j) {
    for (int c = 0; c < nc; ++c) {
      const R* coef = reinterpret_cast<const R*>(p->ws + p->L.coef) + static_cast<size_t>(c0 + c) * 2 * m;
      with_n(n, [&](auto nn) {
        constexpr int N = decltype(nn)::value;
        hipLaunchKernelGGL((mf::probe_coef_kernel<R, N>), dim3(nblk), dim3(mf::kWienerThreads), 0,
                           st, coef, omw_of<R>(p, c0 + c), wcoef + static_cast<size_t>(c) * 2 * m,
                           p->tau[c0 + c],
                           probe0 + static_cast<uint32_t>(j), p->desc.chain_id + c0 + c, a.key0,
                           a.key1, entries);
      });
    }
    hipLaunchKernelGGL((mf::fill_zero_kernel<R>), dim3(1024), dim3(256), 0, st,
                       reinterpret_cast<R*>(fwd), L.specs / sizeof(R));
    if ((r = check_launch("log-determinant probe")) != MF_OK) return r;
    for (int k = 0; k < n_iter; ++k) {
      if (k == n_iter - 1)
        MF_HIP(hipMemcpyAsync(prev, fwd, L.specs, hipMemcpyDeviceToDevice, st));
      if ((r = wiener_iter<R>(p, a, nc, fwd, nullptr, false, R(1), R(1), nullptr, st)) != MF_OK)
        return r;
    }
    MF_HIP(hipMemcpyAsync(scr, fwd, L.specs, hipMemcpyDeviceToDevice, st));
    if ((r = wiener_iter<R>(p, a, nc, scr, aux, false, R(0), R(1), nullptr, st)) != MF_OK) return r;
    hipLaunchKernelGGL((mf::fill_zero_kernel<double>), dim3(1), dim3(256), 0, st, g1,
                       static_cast<size_t>(nc) * nb);
    hipLaunchKernelGGL((mf::fill_zero_kernel<double>), dim3(1), dim3(256), 0, st, g0,
                       static_cast<size_t>(nc) * nb);
    MF_HIP(hipMemcpyAsync(scr, fwd, L.specs, hipMemcpyDeviceToDevice, st));
    if ((r = wiener_iter<R>(p, a, nc, scr, aux, true, R(1), R(1), nullptr, st)) != MF_OK) return r;
    MF_HIP(hipMemcpyAsync(scr, prev, L.specs, hipMemcpyDeviceToDevice, st));
    if ((r = wiener_iter<R>(p, a0, nc, scr, aux, true, R(1), R(1), nullptr, st)) != MF_OK) return r;
    for (int c = 0; c < nc; ++c)
      hipLaunchKernelGGL(mf::logdet_combine_kernel, dim3((nb + 63) / 64), dim3(64), 0, st,
                         g1 + c * nb, g0 + c * nb, pkg + c * nb, p->tau[c0 + c], vcell,
                         1.0 / n_probes, nb, out + c * nb);
    if ((r = check_launch("log-determinant sums")) != MF_OK) return r;
  }
  return MF_OK;
}

}  // namespace

extern "C" {

mf_status mf_wiener_logdet_workspace_bytes(const mf_problem* p, int32_t chain, size_t* bytes) {
  if (!p || !bytes) return fail(MF_E_INVALID_ARG, "NULL argument");
  int c0 = 0, nc = 0;
  const mf_status r = wiener_chains(p, chain, &c0, &nc);
  if (r != MF_OK) return r;
  *bytes = logdet_layout(p, nc).total;
  return MF_OK;
}

mf_status mf_wiener_logdet_trace(mf_problem* p, int32_t chain, const double* pk, int32_t n_iter,
                                 int32_t n_probes, uint32_t probe0, void* workspace,
                                 size_t ws_bytes, double* trace_out, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (p->desc.n < 32 || p->desc.n > 256)
    return fail(MF_E_UNSUPPORTED_SIZE, "the Wiener iteration supports grid sides 32 to 256 (got %d)",
                p->desc.n);
  int c0 = 0, nc = 0;
  mf_status r = wiener_chains(p, chain, &c0, &nc);
  if (r != MF_OK) return r;
  if (n_iter < 1 || n_probes < 1) return fail(MF_E_INVALID_ARG, "need n_iter >= 1 and n_probes >= 1");
  if (!pk || !trace_out) return fail(MF_E_INVALID_ARG, "pk and trace_out must be device pointers");
  const LLayout L = logdet_layout(p, nc);
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(MF_E_WORKSPACE, "log-determinant workspace NULL or not 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(MF_E_WORKSPACE, "log-determinant workspace too small: %zu < %zu", ws_bytes, L.total);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  char* g = static_cast<char*>(workspace);
  return p->fp64() ? logdet_run<double>(p, c0, pk, n_iter, n_probes, probe0, g, L, trace_out, hs)
                   : logdet_run<float>(p, c0, pk, n_iter, n_probes, probe0, g, L, trace_out, hs);
}

}  // extern "C"

// ------------------------------------------- log-determinant trace without allocation
namespace {

// Scratch of mf_wiener_logdet_trace_noalloc: the estimator's workspace in a
// device array of the library's own, so that the call allocates nothing.
// Every device the library runs on holds its own copy until the process
// ends.  In host code `scratch` names a host-side stand-in, never the
// device's memory: kernels and copies take the address from
// hipGetSymbolAddress (scratch_address), kept per device.
static __device__ __align__(256) unsigned char scratch[MF_LOGDET_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the calling thread's current device, looked
// up on that device's first call and kept.
mf_status scratch_address(void** out) {
  int dev = -1;
  MF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(MF_E_DEVICE, "device %d outside the %d devices the scratch table covers", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    MF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign != 0)
      return fail(MF_E_DEVICE, "scratch array of device %d has no usable address", dev);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MF_OK;
}

}  // namespace

extern "C" {

mf_status mf_wiener_logdet_trace_noalloc(mf_problem* p, int32_t chain, const double* pk,
                                         int32_t n_iter, int32_t n_probes, uint32_t probe0,
                                         double* trace_out, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (p->desc.n < 32 || p->desc.n > 256)
    return fail(MF_E_UNSUPPORTED_SIZE, "the Wiener iteration supports grid sides 32 to 256 (got %d)",
                p->desc.n);
  int c0 = 0, nc = 0;
  mf_status r = wiener_chains(p, chain, &c0, &nc);
  if (r != MF_OK) return r;
  if (n_iter < 1 || n_probes < 1) return fail(MF_E_INVALID_ARG, "need n_iter >= 1 and n_probes >= 1");
  if (!pk || !trace_out) return fail(MF_E_INVALID_ARG, "pk and trace_out must be device pointers");
  const LLayout L = logdet_layout(p, nc);
  if (L.total > static_cast<size_t>(MF_LOGDET_SCRATCH_BYTES))
    return fail(MF_E_WORKSPACE, "this estimate needs %zu bytes of scratch; the library's static "
                "scratch holds %zu (use mf_wiener_logdet_trace with a workspace)", L.total,
                static_cast<size_t>(MF_LOGDET_SCRATCH_BYTES));
  void* g = nullptr;
  if ((r = scratch_address(&g)) != MF_OK) return r;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  char* gc = static_cast<char*>(g);
  return p->fp64() ? logdet_run<double>(p, c0, pk, n_iter, n_probes, probe0, gc, L, trace_out, hs)
                   : logdet_run<float>(p, c0, pk, n_iter, n_probes, probe0, gc, L, trace_out, hs);
}

}  // extern "C"

// ---------------------------------------------------------------- diagnostics
namespace {

// Samples n in [start, sweep) with (n - start) % thin == 0.
uint64_t recorded_count(const mf_problem* p) {
  const DiagRec& d = p->diag;
  if (d.thin <= 0 || p->sweep <= d.start) return 0;
  return (p->sweep - d.start - 1) / static_cast<uint64_t>(d.thin) + 1;
}

template <typename R>
void launch_moments(const mf_problem* p, int chain, double count, double* mean, double* var,
                    hipStream_t st) {
  const int n = p->desc.n;
  const size_t m = static_cast<size_t>(n) * n * n, entries = m / 2;
  const double* mom = p->diag.mom + static_cast<size_t>(chain) * 2 * m;
  const int nblk = static_cast<int>((entries + mf::kWienerThreads - 1) / mf::kWienerThreads);
  auto go = [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    hipLaunchKernelGGL((mf::moments_kernel<R, N>), dim3(nblk), dim3(mf::kWienerThreads), 0, st, mom,
                       count, mean, var, entries);
  };
  switch (n) {
    case 8: go(std::integral_constant<int, 8>{}); break;
    case 16: go(std::integral_constant<int, 16>{}); break;
    case 512: go(std::integral_constant<int, 512>{}); break;
    default: with_n(n, go); break;
  }
}

}  // namespace

extern "C" {

mf_status mf_diagnostics_bytes(const mf_problem* p, int32_t trace_cap, size_t* trace_bytes,
                               size_t* moments_bytes) {
  if (!p || !trace_bytes || !moments_bytes) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (trace_cap < 0) return fail(MF_E_INVALID_ARG, "negative trace capacity");
  const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
  *trace_bytes = static_cast<size_t>(p->desc.n_chains) * trace_cap * p->desc.n_bins * 8;
  *moments_bytes = static_cast<size_t>(p->desc.n_chains) * 2 * m * 8;
  return MF_OK;
}

mf_status mf_set_diagnostics(mf_problem* p, uint64_t start, int32_t thin, double* trace,
                             int32_t trace_cap, double* moments, void* stream) {
  if (!p) return fail(MF_E_INVALID_ARG, "problem is NULL");
  if (thin < 1) return fail(MF_E_INVALID_ARG, "thin must be >= 1");
  if (trace && trace_cap < 1) return fail(MF_E_INVALID_ARG, "trace capacity must be >= 1");
  if (start > kMaxSweep) return fail(MF_E_INVALID_ARG, "start sweep beyond 2^32 - 1");
  // a graph replays the recording settings it captured, buffers included
  if (p->graphs > 0)
    return fail(MF_E_STATE, "%d live graph(s) captured this problem's sweep; destroy them "
                "before changing the diagnostics", p->graphs);
  for (const void* q : {static_cast<const void*>(trace), static_cast<const void*>(moments)})
    if (q && reinterpret_cast<uintptr_t>(q) % 8 != 0)
      return fail(MF_E_INVALID_ARG, "diagnostic buffers must be 8-byte aligned");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (moments) {
    const size_t m = static_cast<size_t>(p->desc.n) * p->desc.n * p->desc.n;
    hipLaunchKernelGGL((mf::fill_zero_kernel<double>), dim3(1024), dim3(256), 0, hs, moments,
                       static_cast<size_t>(p->desc.n_chains) * 2 * m);
    const mf_status r = check_launch("moment buffer clear");
    if (r != MF_OK) return r;
  }
  p->diag = DiagRec{trace, moments, start, thin, trace ? trace_cap : 0};
  if (!trace && !moments) p->diag = DiagRec{};
  return MF_OK;
}

mf_status mf_recorded_samples(const mf_problem* p, uint64_t* count) {
  if (!p || !count) return fail(MF_E_INVALID_ARG, "NULL argument");
  *count = recorded_count(p);
  return MF_OK;
}

mf_status mf_get_moments(mf_problem* p, int32_t chain, double* mean, double* var, void* stream) {
  if (!p || !mean || !var) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (chain < 0 || chain >= p->desc.n_chains) return fail(MF_E_STATE, "chain %d out of range", chain);
  if (!p->diag.mom) return fail(MF_E_STATE, "no moment buffer set (mf_set_diagnostics)");
  const uint64_t k = recorded_count(p);
  if (k == 0) return fail(MF_E_STATE, "no sample recorded yet");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (p->fp64()) launch_moments<double>(p, chain, static_cast<double>(k), mean, var, hs);
  else launch_moments<float>(p, chain, static_cast<double>(k), mean, var, hs);
  return check_launch("moments");
}

mf_status mf_acf(const double* trace, int32_t t, int32_t n_bins, int32_t max_lag, double* acf,
                 int32_t* nc, void* stream) {
  if (!trace || !acf || !nc) return fail(MF_E_INVALID_ARG, "NULL argument");
  if (t < 2 || n_bins < 1 || max_lag < 0 || max_lag >= t)
    return fail(MF_E_INVALID_ARG, "need t >= 2, n_bins >= 1 and 0 <= max_lag < t");
  hipLaunchKernelGGL(mf::acf_kernel, dim3(n_bins), dim3(mf::kWienerThreads), 0,
                     static_cast<hipStream_t>(stream), trace, t, n_bins, max_lag, acf, nc);
  return check_launch("acf");
}

mf_status mf_stream_reference(const void* src, void* dst, size_t bytes, int32_t mode,
                              int32_t blocks, void* stream) {
  if (!src || !dst) return fail(MF_E_INVALID_ARG, "src and dst must be device pointers");
  if (mode < 0 || mode > 3) return fail(MF_E_INVALID_ARG, "mode %d outside 0..3", mode);
  if (bytes == 0 || bytes % 16 != 0) return fail(MF_E_INVALID_ARG, "bytes must be a positive multiple of 16");
  if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return fail(MF_E_INVALID_ARG, "src and dst must be 16-byte aligned");
  if (blocks < 1 || blocks > 65536) return fail(MF_E_INVALID_ARG, "blocks %d outside 1..65536", blocks);
  const auto* s16 = static_cast<const mf::v4u*>(src);
  const size_t n16 = bytes / 16;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const dim3 grid(static_cast<unsigned>(blocks)), block(mf::kStreamThreads);
  switch (mode) {
    case 0: hipLaunchKernelGGL(mf::stream_copy_kernel<false>, grid, block, 0, hs, s16, static_cast<mf::v4u*>(dst), n16); break;
    case 1: hipLaunchKernelGGL(mf::stream_copy_kernel<true>, grid, block, 0, hs, s16, static_cast<mf::v4u*>(dst), n16); break;
    case 2: hipLaunchKernelGGL(mf::stream_read_kernel<false>, grid, block, 0, hs, s16, static_cast<uint32_t*>(dst), n16); break;
    default: hipLaunchKernelGGL(mf::stream_read_kernel<true>, grid, block, 0, hs, s16, static_cast<uint32_t*>(dst), n16); break;
  }
  return check_launch("stream reference");
}

}  // extern "C"
