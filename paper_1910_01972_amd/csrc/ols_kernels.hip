// Fused overlap-and-save kernels for gfx950 and the C ABI declared in ols.h.
//
// ols_forward_kernel<N>: one persistent workgroup processes a contiguous range
// of (segment tile, filter) work units.  A tile is SEGS consecutive segments,
// one N-point transform per G = N/16 lanes.  When the range enters a new tile
// the workgroup loads its segments and forward transforms them once; the
// spectra stay in registers for every filter of the range (sec. 3.4: the
// segment samples are reused throughout).  Each unit multiplies by one filter
// spectrum, inverse transforms, and writes only the unaliased samples
// (sec. 3.2, Alg. 2).  HBM sees the signal once (plus the D-sample overlaps)
// and every output sample once.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/ols.h"
#include "ols_fft.hpp"
#include "ols_ops.hpp"
#include "ols_twiddle.hpp"

namespace ols {

// ---------------------------------------------------------------------------
// Transform drivers (device): passes in registers, exchanges through LDS.
// ---------------------------------------------------------------------------
// Synchronisation of an exchange.  When a transform spans several waves
// (G > 64) the exchange crosses waves and needs a workgroup barrier.  When
// every transform lives inside one wave (G <= 64), a wave only ever touches
// the LDS interval of its own transforms, in every exchange and every buffer,
// and the LDS completes a wave's operations in program order: no barrier is
// needed, only a fence that keeps the compiler from reordering the reads of
// other lanes' data before the writes.
template <int N>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (Geo<N>::G <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  } else {
    __syncthreads();
  }
}

// Exchanges alternate between two LDS buffers of Geo<N>::LDS elements.  All
// lanes of the workgroup see the same sequence of exchanges, so one barrier
// per exchange suffices: a lane that passes the barrier of exchange n+1 knows
// every lane has finished reading exchange n (program order), and exchange n+2
// reuses exchange n's buffer.  `par` selects the buffer of the next exchange.
// Single-wave transforms need no second buffer (their exchanges are
// wave-private and in order), so they keep using the first.
template <int N, int E, int KW, int KR>
__device__ __forceinline__ void exchange(float2 (&x)[16], float2* lds, int& par, int grp, int g) {
  float2* buf = lds + ((Geo<N>::G > 64 && par) ? Geo<N>::LDS : 0);
  par ^= 1;
  lds_store<N, E, KW>(buf, x, grp, g);
  exchange_sync<N>();
  lds_load<N, E, KR>(buf, x, grp, g);
}

// NF independent transforms exchanged together: one buffer each, written
// before one barrier and read after it; the second barrier protects the
// buffers from the next exchange's writes.  The last exchange of the
// transform (between passes P-2 and P-1) keeps every value inside the wave
// that wrote it (both layouts put position bits 10 and up in the wave index;
// the host emulator checks this for every N), so its first barrier is
// replaced by a wave-scope fence; the second still guards the next exchange,
// whose writes cross waves.
template <int N, int NF, int E, int KW, int KR>
__device__ __forceinline__ void exchange_nf(float2 (&x)[NF][16], float2* lds, int& par, int grp, int g) {
  if constexpr (NF == 1) {
    exchange<N, E, KW, KR>(x[0], lds, par, grp, g);
  } else {
#pragma unroll
    for (int f = 0; f < NF; ++f) lds_store<N, E, KW>(lds + f * Geo<N>::LDS, x[f], grp, g);
    if constexpr (E == Geo<N>::P - 2) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    else exchange_sync<N>();
#pragma unroll
    for (int f = 0; f < NF; ++f) lds_load<N, E, KR>(lds + f * Geo<N>::LDS, x[f], grp, g);
    exchange_sync<N>();
  }
}

template <int N, int K>
__device__ __forceinline__ void fwd_from(float2 (&x)[16], float2* lds, int& par, const float2* tw, int grp, int g) {
  run_pass<N, K, false>(x, tw + Geo<N>::lane_tw_offset(K));
  if constexpr (K + 1 < Geo<N>::P) {
    exchange<N, K, K, K + 1>(x, lds, par, grp, g);
    fwd_from<N, K + 1>(x, lds, par, tw, grp, g);
  }
}

template <int N, int K>
__device__ __forceinline__ void inv_from(float2 (&x)[16], float2* lds, int& par, const float2* tw, int grp, int g) {
  inverse_pass<N, K>(x, tw + Geo<N>::lane_tw_offset(K));
  if constexpr (K > 0) {
    exchange<N, K - 1, K, K - 1>(x, lds, par, grp, g);
    inv_from<N, K - 1>(x, lds, par, tw, grp, g);
  }
}

template <int N, int NF, int K>
__device__ __forceinline__ void inv_from_nf(float2 (&x)[NF][16], float2* lds, int& par, const float2* tw, int grp,
                                            int g) {
#pragma unroll
  for (int f = 0; f < NF; ++f) inverse_pass<N, K>(x[f], tw + Geo<N>::lane_tw_offset(K));
  if constexpr (K > 0) {
    exchange_nf<N, NF, K - 1, K, K - 1>(x, lds, par, grp, g);
    inv_from_nf<N, NF, K - 1>(x, lds, par, tw, grp, g);
  }
}

// x[f] holds a filter spectrum on entry and the inverse FFT of A * spectrum
// (natural order) on exit, for NF filters at once; the product is fused into
// the first inverse pass.
template <int N, int NF>
__device__ __forceinline__ void inverse_of_products(float2 (&x)[NF][16], const float2 (&A)[16], float2* lds,
                                                    int& par, const float2* tw, int grp, int g) {
  constexpr int P = Geo<N>::P;
#pragma unroll
  for (int f = 0; f < NF; ++f) product_pass<N>(x[f], A);
  exchange_nf<N, NF, P - 2, P - 1, P - 2>(x, lds, par, grp, g);
  inv_from_nf<N, NF, P - 2>(x, lds, par, tw, grp, g);
}

// ---------------------------------------------------------------------------
// Filter spectra (plan step): F_r = FFT_N(pad(h_r)) / N in kernel order;
// h is complex64, or float32 for R2R plans (real != 0).
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Geo<N>::WG) void ols_filter_spectra_kernel(const void* __restrict__ h, int K, int M,
                                                                        float2* __restrict__ F,
                                                                        const float2* __restrict__ twt, int diff,
                                                                        int real) {
  using GE = Geo<N>;
  __shared__ float2 lds[2 * GE::LDS];
  const int tid = threadIdx.x;
  const int grp = tid / GE::G, g = tid - grp * GE::G;
  const int r = blockIdx.x * GE::SEGS + grp;
  int par = 0;
  float2 tw[GE::TWR];
  load_lane_twiddles<N>(tw, twt, g);
  float2 x[16];
  const bool valid = r < K;
  const int64_t row = (int64_t)(valid ? r : 0) * M;
  if (real) load_filter_real<N>(x, (const float*)h + row, M, valid, diff != 0, g);
  else if (diff) load_filter_diff<N>(x, (const float2*)h + row, M, valid, g);
  else load_filter<N>(x, (const float2*)h + row, M, valid, g);
  fwd_from<N, 0>(x, lds, par, tw, grp, g);
  if (valid) store_spectrum<N>(x, F, r, g, 1.0f / (float)N);
}

// Natural-order copy of the spectra: out[r][k] = F[r][spectrum_offset(reg, g)]
// with k = spectrum_index(g, reg).
template <int N>
__global__ void ols_spectra_natural_kernel(const float2* __restrict__ F, int K, float2* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over K * N
  if (i >= (int64_t)K * N) return;
  const int r = (int)(i / N);
  const int rem = (int)(i - (int64_t)r * N);  // = spectrum_offset(reg, g)
  const int pair = rem >> 1, j = pair / Geo<N>::G, g = pair - j * Geo<N>::G;
  const int reg = 2 * j + (rem & 1);
  out[(int64_t)r * N + spectrum_index<N>(g, reg)] = F[i];
}

// ---------------------------------------------------------------------------
// Forward overlap-and-save: persistent, balanced static partition of the
// ntiles * ceil(K / NF) work units over the grid.  A unit is one tile of
// segments and NF consecutive filters, whose NF inverse transforms run
// interleaved (independent instruction streams; one barrier pair per exchange
// serves all NF).
// ---------------------------------------------------------------------------
// Units [u0, u1) of one signal: the body shared by the single-signal kernel
// and the batched kernel.  `par` carries the LDS buffer parity across calls.
// REAL (R2R): s and y are float32 and a transform carries a pair of segments
// (real part 2q, imaginary part 2q+1), so a tile is SEGS pairs.  POWER
// stores |y|^2 (float32) instead of y.
// tw: this lane's twiddles (load_lane_twiddles).
template <int N, int NF, bool POWER = false, bool REAL = false, int SMODE = STORE_NT_WHOLE>
__device__ __forceinline__ void forward_units(const void* __restrict__ sv, int64_t Ns, const float2* __restrict__ F,
                                              void* __restrict__ yv, int K, int D, int H,
                                              const float2 (&tw)[Geo<N>::TWR], int64_t u0, int64_t u1, float2* lds,
                                              int& par) {
  using GE = Geo<N>;
  const int tid = threadIdx.x;
  const int grp = tid / GE::G, g = tid - grp * GE::G;
  const int KG = (K + NF - 1) / NF;  // filter groups
  const int64_t step = REAL ? 2 * (int64_t)H : H;  // signal advance per transform

  int64_t tile = u0 / KG;
  int rg = (int)(u0 - tile * KG);
  float2 A[16], x[NF][16];

  // Transform index of this lane (a segment, or a segment pair for REAL);
  // uniform over a wave when a transform spans whole waves (G >= 64).
  auto segment_of = [&](int64_t t) -> int64_t {
    const int64_t sg = t * GE::SEGS + grp;
    return GE::G >= 64 ? wave_uniform64(sg) : sg;
  };
  auto load = [&](int64_t sg) {
    if constexpr (REAL) load_segment_pair<N>(x[0], (const float*)sv, Ns, sg * step - D, H, g);
    else load_segment<N>(x[0], (const float2*)sv, Ns, sg * step - D, g);
  };

  int64_t seg = segment_of(tile);
  load(seg);
  fwd_from<N, 0>(x[0], lds, par, tw, grp, g);
#pragma unroll
  for (int i = 0; i < 16; ++i) A[i] = x[0][i];

  for (int64_t u = u0; u < u1; ++u) {
    if (rg == KG) {  // next tile: new segments, one forward transform each
      rg = 0;
      ++tile;
      seg = segment_of(tile);
      load(seg);
      fwd_from<N, 0>(x[0], lds, par, tw, grp, g);
#pragma unroll
      for (int i = 0; i < 16; ++i) A[i] = x[0][i];
    }
    // spectra of this unit's filters; filters past K (a ragged last group)
    // reuse the last filter's spectrum and are not stored
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int r = rg * NF + f;
      load_spectrum<N>(x[f], F, r < K ? r : K - 1, g);
    }
    inverse_of_products<N, NF>(x, A, lds, par, tw, grp, g);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int r = rg * NF + f;
      if (NF == 1 || r < K) {
        if constexpr (REAL)
          store_valid_pair<N, POWER, SMODE>(x[f], (float*)yv + (int64_t)r * Ns, Ns, seg * step, D, H, g);
        else if constexpr (POWER)
          store_valid_power<N, SMODE>(x[f], (float*)yv + (int64_t)r * Ns, Ns, seg * step, D, H, g);
        else
          store_valid<N, SMODE>(x[f], (float2*)yv + (int64_t)r * Ns, Ns, seg * step, D, H, g);
      }
    }
    ++rg;
  }
}

template <int N, int NF, bool POWER = false, bool REAL = false, int SMODE = STORE_NT_WHOLE>
__device__ __forceinline__ void forward_range(const void* __restrict__ sv, int64_t Ns, const float2* __restrict__ F,
                                              void* __restrict__ yv, int K, int D, int H,
                                              const float2* __restrict__ twt, int64_t u0, int64_t u1, float2* lds,
                                              int& par) {
  float2 tw[Geo<N>::TWR];
  load_lane_twiddles<N>(tw, twt, threadIdx.x % Geo<N>::G);
  forward_units<N, NF, POWER, REAL, SMODE>(sv, Ns, F, yv, K, D, H, tw, u0, u1, lds, par);
}

template <int N, int NF, bool POWER, bool REAL>
__global__ __launch_bounds__(Geo<N>::WG) void ols_forward_kernel(const void* __restrict__ s, int64_t Ns,
                                                                 const float2* __restrict__ F, void* __restrict__ y,
                                                                 int K, int D, int H, int64_t ntiles,
                                                                 const float2* __restrict__ twt) {
  using GE = Geo<N>;
  constexpr int BUFS = (NF == 1 && GE::G > 64) ? 2 : NF;  // double-buffered only across waves
  __shared__ float2 lds[BUFS * GE::LDS];
  const int64_t U = ntiles * ((K + NF - 1) / NF);
  const int64_t u0 = first_unit(U, gridDim.x, blockIdx.x);
  const int64_t u1 = first_unit(U, gridDim.x, blockIdx.x + 1);
  if (u0 >= u1) return;  // uniform over the workgroup
  int par = 0;
  forward_range<N, NF, POWER, REAL>(s, Ns, F, y, K, D, H, twt, u0, u1, lds, par);
}

// ---------------------------------------------------------------------------
// Batched forward: many signals, each with its own filters (K_i, M_i), FFT
// length N_i in {256, ..., 4096} and hop, in one persistent launch.  The
// items' segment tiles are numbered consecutively (item i owns tiles
// [tile_begin_i, tile_begin_i + ntiles_i)) and dealt round-robin to the
// workgroups; for each tile a workgroup switches on its item's (N, filters
// per unit) to the same range body as the single-signal kernel, over all of
// the tile's units.  Every N <= 4096 uses 256 threads and the same LDS
// footprint, so one launch covers them all.
// ---------------------------------------------------------------------------
struct BatchItem {
  const float2* s;
  float2* y;
  const float2* spectra;  // [K][N] in transform order, scaled by 1/N
  int64_t Ns;
  int64_t unit_begin;
  int64_t units;
  int32_t K, M, N, D, H, nf;
  int64_t tile_begin;  // first tile of this item in the batch's tile list
  int64_t ntiles;      // tiles of this item (units = ntiles * units per tile)
};

// Each (N, filters per unit) body is its own non-inlined function, so its
// registers are allocated on their own and the kernel needs only the
// maximum, not the sum, over the branches it may take.  A body runs the
// workgroup's tiles t, t + P, t + 2P, ... for as long as their items keep its
// (N, filters per unit): the lane twiddles are loaded once per run, and
// consecutive tiles of one class need no barrier between them (the same
// exchange protocol as consecutive tiles of the single-signal kernel).  The
// batch plan orders the items by class, so a workgroup meets each class in
// one run.  Returns the workgroup's first tile of another class (or past the
// end); i follows the item walk.
template <int N, int NF>
__device__ __attribute__((noinline)) int64_t batched_run(const BatchItem* __restrict__ items, int nitems, int& i,
                                                         int64_t t, int64_t total_tiles,
                                                         const float2* __restrict__ twt, float2* lds, int& par) {
  float2 tw[Geo<N>::TWR];
  load_lane_twiddles<N>(tw, twt, threadIdx.x % Geo<N>::G);
  for (;;) {
    const BatchItem& it = items[i];
    const int64_t per_tile = it.units / it.ntiles;
    const int64_t a = (t - it.tile_begin) * per_tile;
    forward_units<N, NF, false, false, STORE_NT>(it.s, it.Ns, it.spectra, it.y, it.K, it.D, it.H, tw, a,
                                                  a + per_tile, lds, par);
    t += gridDim.x;
    if (t >= total_tiles) return t;
    // t grows, so the item walk only moves forward (items without tiles are skipped)
    while (i + 1 < nitems && items[i + 1].tile_begin <= t) ++i;
    if (items[i].N != N || items[i].nf != NF) return t;
  }
}

// Two filters per unit only up to N = 2048 here (BATCH_NF2_MAX_N): the
// N = 4096 two-filter body needs more than 256 registers as a separate
// function, which would drop the whole kernel to one wave per SIMD.

template <int N>
__device__ __forceinline__ int64_t batched_class(const BatchItem* __restrict__ items, int nitems, int& i, int64_t t,
                                                 int64_t total_tiles, const float2* __restrict__ twt, float2* lds,
                                                 int& par) {
  if constexpr (N <= BATCH_NF2_MAX_N) {
    if (items[i].nf == 2) return batched_run<N, 2>(items, nitems, i, t, total_tiles, twt, lds, par);
  }
  return batched_run<N, 1>(items, nitems, i, t, total_tiles, twt, lds, par);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ols_batched_kernel(const BatchItem* __restrict__ items, int nitems,
                                                          int64_t total_tiles, const float2* __restrict__ tw256,
                                                          const float2* __restrict__ tw512,
                                                          const float2* __restrict__ tw1024,
                                                          const float2* __restrict__ tw2048,
                                                          const float2* __restrict__ tw4096) {
  __shared__ float2 lds[2 * Geo<4096>::LDS];
  static_assert(Geo<256>::LDS == Geo<4096>::LDS && Geo<2048>::LDS == Geo<4096>::LDS, "same LDS footprint");
  // Tiles of all items, in the plan's item order, dealt round-robin to the
  // workgroups: workgroup b takes tiles b, b + P, b + 2P, ... with all of
  // each tile's filters.  At any moment the whole grid works on neighbouring
  // tiles of one or two items, so every XCD keeps those items' filter
  // spectra in its L2 (balanced contiguous unit ranges spread the grid over
  // all items at once and re-read the spectra from HBM: 19 % slower on the
  // uneven batch).  The imbalance is at most one tile per workgroup.
  int par = 0;
  int i = 0;
  int64_t t = blockIdx.x;
  while (t < total_tiles) {
    while (i + 1 < nitems && items[i + 1].tile_begin <= t) ++i;
    // items of another class lay out the LDS buffers differently, and
    // single-wave transforms exchange without barriers: every wave must have
    // finished with the previous run's buffers
    __syncthreads();
    switch (items[i].N) {
      case 256: t = batched_class<256>(items, nitems, i, t, total_tiles, tw256, lds, par); break;
      case 512: t = batched_class<512>(items, nitems, i, t, total_tiles, tw512, lds, par); break;
      case 1024: t = batched_class<1024>(items, nitems, i, t, total_tiles, tw1024, lds, par); break;
      case 2048: t = batched_class<2048>(items, nitems, i, t, total_tiles, tw2048, lds, par); break;
      default: t = batched_class<4096>(items, nitems, i, t, total_tiles, tw4096, lds, par); break;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of eq. (1), by overlap-and-save.  For upstream gradients g_r:
//   ds[m]   = sum_r sum_k conj(h_r[k]) g_r[m+k]
//   dh_r[k] = sum_m conj(s[m]) g_r[m+k]
// Segment j's window is g_r[jH .. jH+N-1] (future samples; the aliased
// positions are the last M-1, footnote to eq. 2).  Per segment and filter one
// forward transform G_r serves both gradients:
//   ds window = IFFT(sum_r conj(F_r) G_r), positions 0 .. H-1
//   dh_r     += first M lags of IFFT(conj(S_j)/N * G_r), S_j = FFT(s[jH .. jH+H-1])
// Units are (tile, filter) with the filter inner, split into balanced ranges.
// A tile whose filters are split between workgroups leaves partial ds windows
// in ws_ds (slot 0 for a range's first tile, 1 for its last); a fixup kernel
// adds them in workgroup order.  dh lags accumulate in each workgroup's own
// slot of part_dh ([grid][SEGS][K][M]) and are reduced in a fixed order.
// Nothing is atomic, so the result is deterministic.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(Geo<N>::WG) void ols_backward_kernel(
    const float2* __restrict__ s, const float2* __restrict__ gy, int64_t Ns, const float2* __restrict__ F, int K,
    int M, int H, int64_t ntiles, const float2* __restrict__ twt, float2* __restrict__ ds,
    float2* __restrict__ ws_ds, float2* __restrict__ part_dh, int want_ds, int want_dh) {
  using GE = Geo<N>;
  __shared__ float2 lds[2 * GE::LDS];
  const int tid = threadIdx.x;
  const int grp = tid / GE::G, g = tid - grp * GE::G;
  const int64_t P = gridDim.x, b = blockIdx.x;
  const int64_t U = ntiles * K;
  const int64_t u0 = first_unit(U, P, b), u1 = first_unit(U, P, b + 1);
  if (u0 >= u1) return;  // uniform over the workgroup

  float2 tw[GE::TWR];
  load_lane_twiddles<N>(tw, twt, g);
  float2* part = part_dh + (b * GE::SEGS + grp) * (int64_t)K * M;
  if (want_dh)
    for (int r = 0; r < K; ++r) zero_lags<N>(part + (int64_t)r * M, M, g);

  const int64_t t_first = u0 / K;
  int64_t tile = t_first;
  int r = (int)(u0 - tile * K);
  int par = 0;
  float2 A[16], acc[16], x[16], f[16];
  auto segment_of = [&](int64_t t) -> int64_t {
    const int64_t sg = t * GE::SEGS + grp;
    return GE::G >= 64 ? wave_uniform64(sg) : sg;
  };
  int64_t seg = segment_of(tile);

  auto start_tile = [&]() {
    seg = segment_of(tile);
    if (want_dh) {
      load_window<N>(x, s, Ns, seg * H, H, g);
      fwd_from<N, 0>(x, lds, par, tw, grp, g);
      conj_scaled(A, x, 1.0f / (float)N);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = make_float2(0.f, 0.f);
  };
  auto finish_tile = [&]() {
    if (!want_ds) return;
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = acc[i];
    inv_from<N, GE::P - 1>(x, lds, par, tw, grp, g);
    const bool complete = tile * K >= u0 && (tile + 1) * K <= u1;
    if (complete) {
      store_valid<N>(x, ds, Ns, seg * H, 0, H, g);
    } else {
      const int slot = tile == t_first ? 0 : 1;
      float2* w = ws_ds + ((b * 2 + slot) * GE::SEGS + grp) * (int64_t)N;
      store_valid<N>(x, w, (int64_t)H, 0, 0, H, g);
    }
  };

  start_tile();
  for (int64_t u = u0; u < u1; ++u) {
    if (r == K) {
      finish_tile();
      r = 0;
      ++tile;
      start_tile();
    }
    load_window<N>(x, gy + (int64_t)r * Ns, Ns, seg * H, N, g);
    fwd_from<N, 0>(x, lds, par, tw, grp, g);
    if (want_ds) {
      load_spectrum<N>(f, F, r, g);
      acc_conj_product(acc, x, f);
    }
    if (want_dh) {
      product_pass<N>(x, A);
      exchange<N, GE::P - 2, GE::P - 1, GE::P - 2>(x, lds, par, grp, g);
      inv_from<N, GE::P - 2>(x, lds, par, tw, grp, g);
      add_lags<N>(part + (int64_t)r * M, x, M, g);
    }
    ++r;
  }
  finish_tile();
}

// Sums the partial ds windows of tiles split between workgroups; block b-1
// handles the boundary between workgroups b-1 and b (the first boundary
// inside a tile does the whole tile).
template <int N>
__global__ void ols_ds_fixup_kernel(const float2* __restrict__ ws_ds, float2* __restrict__ ds, int64_t Ns, int K,
                                    int H, int64_t ntiles, int64_t P) {
  using GE = Geo<N>;
  const int64_t b = (int64_t)blockIdx.x + 1;
  const int64_t U = ntiles * K;
  const int64_t ub = first_unit(U, P, b);
  if (ub % K == 0) return;
  const int64_t t = ub / K;
  if (first_unit(U, P, b - 1) > t * K) return;
  const int64_t blo = owner_of_unit(U, P, t * K), bhi = owner_of_unit(U, P, (t + 1) * K - 1);
  // Slot of each sharing workgroup's window (0: the tile is its first, 1: its
  // last): every workgroup after blo starts inside tile t; blo may have
  // started in an earlier tile.  Hoisted out of the element loop (64-bit
  // divisions).
  const int64_t slot_lo = first_unit(U, P, blo) / K == t ? 0 : 1;
  // blockIdx.y splits the window between workgroups: few outputs per lane,
  // so the lanes' loads are all in flight at once
  const int stride = blockDim.x * gridDim.y;
  for (int sg = 0; sg < GE::SEGS; ++sg) {
    const int64_t o0 = (t * GE::SEGS + sg) * H;
    for (int p = threadIdx.x + blockIdx.y * blockDim.x; p < H; p += stride) {
      if (o0 + p >= Ns) break;
      float2 a = make_float2(0.f, 0.f);
      for (int64_t bb = blo; bb <= bhi; ++bb) {
        const int64_t slot = bb == blo ? slot_lo : 0;
        a = cadd(a, ws_ds[((bb * 2 + slot) * GE::SEGS + sg) * (int64_t)N + p]);
      }
      ds[o0 + p] = a;
    }
  }
}

// First level of the dh reduction: sums[c][i] = sum of part[slot][i] over
// the slots of chunk c = blockIdx.y, in slot order.
__global__ void ols_dh_chunk_kernel(const float2* __restrict__ part, int64_t nslots, int64_t KM,
                                    float2* __restrict__ sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KM) return;
  const int64_t c = blockIdx.y;
  const int64_t s0 = c * DH_CHUNK, s1 = s0 + DH_CHUNK < nslots ? s0 + DH_CHUNK : nslots;
  float2 a = make_float2(0.f, 0.f);
  for (int64_t sl = s0; sl < s1; ++sl) a = cadd(a, part[sl * KM + i]);
  sums[c * KM + i] = a;
}

// dh[i] = sum over slots of part[slot][i], in slot order (second level: the
// chunk sums in chunk order).
__global__ void ols_dh_reduce_kernel(const float2* __restrict__ part, int64_t nslots, int64_t KM,
                                     float2* __restrict__ dh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KM) return;
  float2 a = make_float2(0.f, 0.f);
  for (int64_t sl = 0; sl < nslots; ++sl) a = cadd(a, part[sl * KM + i]);
  dh[i] = a;
}

// Plain fill with zero (used instead of a memset so callers may capture it).
__global__ void ols_zero_kernel(float2* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = make_float2(0.f, 0.f);
}

// Plain copy, the known-size workload for HBM counter calibration.
__global__ void ols_copy_kernel(float4* __restrict__ dst, const float4* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace ols

// ===========================================================================
// Host side
// ===========================================================================
using namespace ols;

struct ols_plan_s {
  int K = 0, M = 0, N = 0, D = 0, H = 0;
  int device = 0;
  int cus = 0;
  int grid = 0;   // persistent workgroups of the forward kernel
  int block = 0;  // threads per workgroup
  int segs = 0;   // segments per tile
  int nf = 1;     // filters per work unit of the forward kernel
  int flags = 0;  // OLS_POST_* and OLS_REAL
  int bwd_grid = 0;           // persistent workgroups of the adjoint kernel
  float2* ws_ds = nullptr;    // [bwd_grid][2][SEGS][N] partial ds windows
  float2* part_dh = nullptr;  // [bwd_grid][SEGS][K][M] dh lag partials
  float2* sum_dh = nullptr;   // [dh_chunks(bwd_grid * SEGS)][K][M] chunk sums of part_dh
  float2* spectra = nullptr;
  float2* twiddles = nullptr;
};

struct ols_batch_s {
  int n = 0;
  int64_t total_units = 0;
  int grid = 0;
  int cus = 0;
  BatchItem* items_dev = nullptr;       // in kernel order (items_sorted)
  std::vector<BatchItem> items_host;    // in the caller's order
  std::vector<BatchItem> items_sorted;  // by class (N, filters per unit)
  std::vector<int> order;               // items_sorted[k] = items_host[order[k]]
  float2* spectra = nullptr;
  float2* tw[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // N = 256 .. 4096
  int64_t total_tiles = 0;
};

namespace {

thread_local std::string g_last_error;

ols_status_t fail(ols_status_t st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ols_status_t hip_fail(hipError_t e, const char* what) {
  return fail(OLS_ERROR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int default_delay(int N, int M) {
  const int d = ((M - 1) + 15) / 16 * 16;
  return d <= N - 1 ? d : M - 1;
}

// Approximate FFT work per valid output sample for FFT length N; used when
// the caller passes N = 0.
double cost_per_output(int N, int M, int K) {
  const int D = default_delay(N, M);
  const int H = N - D;
  if (H < 1) return 1e300;
  const double lg = std::log2((double)N);
  const double per_fft = 3.2 * N * lg;
  const double work = (K + 1.0) * per_fft + K * 4.0 * N;
  return work / ((double)K * H);
}


template <int N>
struct Kern {
  using GE = Geo<N>;
  static constexpr bool HAS_NF2 = N <= 4096;

  static hipError_t spectra(const void* h, int K, int M, float2* F, const float2* tw, hipStream_t st, int diff,
                            int real) {
    const int blocks = (K + GE::SEGS - 1) / GE::SEGS;
    hipLaunchKernelGGL(ols_filter_spectra_kernel<N>, dim3(blocks), dim3(GE::WG), 0, st, h, K, M, F, tw, diff, real);
    return hipGetLastError();
  }
  static hipError_t natural(const float2* F, int K, float2* out, hipStream_t st) {
    const int64_t total = (int64_t)K * N;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(ols_spectra_natural_kernel<N>, dim3((unsigned)blocks), dim3(threads), 0, st, F, K, out);
    return hipGetLastError();
  }
  // Forward kernel instance for (filters per unit, power epilogue, R2R).
  using ForwardFn = void (*)(const void*, int64_t, const float2*, void*, int, int, int, int64_t, const float2*);
  template <int NF>
  static ForwardFn forward_fn_nf(bool power, bool real) {
    if (real) {
      // R2R takes two filters per unit only up to N = 2048 (choose_nf_real)
      constexpr int NFR = N <= BATCH_NF2_MAX_N ? NF : 1;
      return power ? ols_forward_kernel<N, NFR, true, true> : ols_forward_kernel<N, NFR, false, true>;
    }
    return power ? ols_forward_kernel<N, NF, true, false> : ols_forward_kernel<N, NF, false, false>;
  }
  static ForwardFn forward_fn(int nf, int flags) {
    const bool power = (flags & OLS_POST_POWER) != 0, real = (flags & OLS_REAL) != 0;
    if constexpr (HAS_NF2) {
      if (nf == 2) return forward_fn_nf<2>(power, real);
    }
    return forward_fn_nf<1>(power, real);
  }
  static hipError_t forward(const ols_plan_s* p, const void* s, int64_t Ns, void* y, hipStream_t st) {
    const int64_t nseg = (Ns + p->H - 1) / p->H;
    const int64_t ntrans = (p->flags & OLS_REAL) ? (nseg + 1) / 2 : nseg;  // R2R: segment pairs
    const int64_t ntiles = (ntrans + GE::SEGS - 1) / GE::SEGS;
    const int64_t units = ntiles * ((p->K + p->nf - 1) / p->nf);
    const int64_t grid = units < p->grid ? units : p->grid;
    hipLaunchKernelGGL(forward_fn(p->nf, p->flags), dim3((unsigned)grid), dim3(GE::WG), 0, st, s, Ns, p->spectra, y,
                       p->K, p->D, p->H, ntiles, p->twiddles);
    return hipGetLastError();
  }
  static hipError_t occupancy(int nf, int flags, int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, forward_fn(nf, flags), GE::WG, 0);
  }
  static hipError_t bwd_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, ols_backward_kernel<N>, GE::WG, 0);
  }
  static hipError_t backward(const ols_plan_s* p, const float2* s, const float2* gy, int64_t Ns, float2* ds,
                             float2* dh, hipStream_t st) {
    const int64_t nseg = (Ns + p->H - 1) / p->H;
    const int64_t ntiles = (nseg + GE::SEGS - 1) / GE::SEGS;
    const int64_t units = ntiles * p->K;
    const int64_t grid = units < p->bwd_grid ? units : p->bwd_grid;
    hipLaunchKernelGGL(ols_backward_kernel<N>, dim3((unsigned)grid), dim3(GE::WG), 0, st, s, gy, Ns, p->spectra, p->K,
                       p->M, p->H, ntiles, p->twiddles, ds, p->ws_ds, p->part_dh, ds ? 1 : 0, dh ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ds && grid > 1) {
      // one workgroup per (tile boundary, eighth of the window): H <= 8192 outputs, at most 4 per lane
      hipLaunchKernelGGL(ols_ds_fixup_kernel<N>, dim3((unsigned)(grid - 1), 8), dim3(256), 0, st, p->ws_ds, ds, Ns,
                         p->K, p->H, ntiles, grid);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (dh) {
      const int64_t KM = (int64_t)p->K * p->M;
      const int64_t nslots = grid * GE::SEGS, nch = dh_chunks(nslots);
      const unsigned bx = (unsigned)((KM + 255) / 256);
      hipLaunchKernelGGL(ols_dh_chunk_kernel, dim3(bx, (unsigned)nch), dim3(256), 0, st, p->part_dh, nslots, KM,
                         p->sum_dh);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(ols_dh_reduce_kernel, dim3(bx), dim3(256), 0, st, p->sum_dh, nch, KM, dh);
      e = hipGetLastError();
    }
    return e;
  }
  static std::vector<float2> twiddles() { return build_twiddles<N>(); }
  static int block() { return GE::WG; }
  static int segs() { return GE::SEGS; }
};

template <template <int> class F, typename... Args>
auto dispatch(int N, Args&&... args) -> decltype(F<256>::run(args...)) {
  switch (N) {
    case 256: return F<256>::run(args...);
    case 512: return F<512>::run(args...);
    case 1024: return F<1024>::run(args...);
    case 2048: return F<2048>::run(args...);
    case 4096: return F<4096>::run(args...);
    default: return F<8192>::run(args...);
  }
}

template <int N>
struct RunSpectra {
  static hipError_t run(const void* h, int K, int M, float2* F, const float2* tw, hipStream_t st, int diff, int real) {
    return Kern<N>::spectra(h, K, M, F, tw, st, diff, real);
  }
};
template <int N>
struct RunNatural {
  static hipError_t run(const float2* F, int K, float2* out, hipStream_t st) { return Kern<N>::natural(F, K, out, st); }
};
template <int N>
struct RunForward {
  static hipError_t run(const ols_plan_s* p, const void* s, int64_t Ns, void* y, hipStream_t st) {
    return Kern<N>::forward(p, s, Ns, y, st);
  }
};
template <int N>
struct RunOccupancy {
  static hipError_t run(int nf, int flags, int* b) { return Kern<N>::occupancy(nf, flags, b); }
};
template <int N>
struct RunBwdOccupancy {
  static hipError_t run(int* b) { return Kern<N>::bwd_occupancy(b); }
};
template <int N>
struct RunBackward {
  static hipError_t run(const ols_plan_s* p, const float2* s, const float2* gy, int64_t Ns, float2* ds, float2* dh,
                        hipStream_t st) {
    return Kern<N>::backward(p, s, gy, Ns, ds, dh, st);
  }
};
template <int N>
struct RunTwiddles {
  static std::vector<float2> run() { return Kern<N>::twiddles(); }
};
template <int N>
struct RunShape {
  static int run(int which) { return which == 0 ? Kern<N>::block() : Kern<N>::segs(); }
};

void destroy_batch(ols_batch_s* b) {
  if (!b) return;
  if (b->items_dev) (void)hipFree(b->items_dev);
  if (b->spectra) (void)hipFree(b->spectra);
  for (auto* t : b->tw)
    if (t) (void)hipFree(t);
  delete b;
}

bool ranges_overlap(const void* a, size_t an, const void* b, size_t bn) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bn && b0 < a0 + an;
}

void destroy_plan(ols_plan_s* p) {
  if (!p) return;
  if (p->ws_ds) (void)hipFree(p->ws_ds);
  if (p->part_dh) (void)hipFree(p->part_dh);
  if (p->sum_dh) (void)hipFree(p->sum_dh);
  if (p->spectra) (void)hipFree(p->spectra);
  if (p->twiddles) (void)hipFree(p->twiddles);
  delete p;
}

}  // namespace

extern "C" {

const char* ols_status_string(ols_status_t s) {
  switch (s) {
    case OLS_SUCCESS: return "success";
    case OLS_ERROR_INVALID_VALUE: return "invalid value";
    case OLS_ERROR_UNSUPPORTED: return "unsupported";
    case OLS_ERROR_OUT_OF_MEMORY: return "out of memory";
    case OLS_ERROR_HIP: return "HIP runtime error";
    case OLS_ERROR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* ols_last_error(void) { return g_last_error.c_str(); }

ols_status_t ols_plan(ols_plan_t* plan, const void* h, int32_t K, int32_t M, int32_t N, ols_stream_t stream) {
  return ols_plan_ex(plan, h, K, M, N, OLS_POST_NONE, stream);
}

ols_status_t ols_plan_ex(ols_plan_t* plan, const void* h, int32_t K, int32_t M, int32_t N, int32_t flags,
                         ols_stream_t stream) {
  try {
    if (!plan) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
    *plan = nullptr;
    if (!h) return fail(OLS_ERROR_INVALID_VALUE, "h is NULL");
    if (K < 1) return fail(OLS_ERROR_INVALID_VALUE, "K must be >= 1");
    if (M < 1) return fail(OLS_ERROR_INVALID_VALUE, "M must be >= 1");
    if (flags & ~(OLS_POST_DERIVATIVE | OLS_POST_POWER | OLS_REAL)) return fail(OLS_ERROR_INVALID_VALUE, "unknown flag");
    const int align = (flags & OLS_REAL) ? 4 : 8;
    if (((uintptr_t)h) % align) return fail(OLS_ERROR_INVALID_VALUE, "h is not aligned to its element type");
    // the derivative is a convolution with [1, -1]: one more tap of aliasing
    const int Meff = (flags & OLS_POST_DERIVATIVE) ? M + 1 : M;
    if (N == 0) {
      double best = 1e301;
      for (int n = OLS_MIN_FFT_LENGTH; n <= OLS_MAX_FFT_LENGTH; n *= 2) {
        if (n < Meff) continue;
        const double c = cost_per_output(n, Meff, K);
        if (c < best) { best = c; N = n; }
      }
      if (N == 0) return fail(OLS_ERROR_INVALID_VALUE, "filter longer than the largest FFT length");
    }
    if (!is_pow2(N) || N < OLS_MIN_FFT_LENGTH || N > OLS_MAX_FFT_LENGTH)
      return fail(OLS_ERROR_UNSUPPORTED, "N must be a power of two in [256, 8192]");
    if (Meff > N) return fail(OLS_ERROR_INVALID_VALUE, "M must be <= N (M + 1 <= N with the derivative)");
    if ((int64_t)K * N > ((int64_t)1 << 40)) return fail(OLS_ERROR_INVALID_VALUE, "K*N too large");

    ols_plan_s* p = new (std::nothrow) ols_plan_s();
    if (!p) return fail(OLS_ERROR_OUT_OF_MEMORY, "host allocation failed");
    p->K = K;
    p->M = M;
    p->N = N;
    p->flags = flags;
    p->D = default_delay(N, Meff);
    p->H = N - p->D;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "hipGetDevice"); }
    e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "hipDeviceGetAttribute"); }
    p->nf = (flags & OLS_REAL) ? choose_nf_real(N, K) : choose_nf(N, K);
    int per_cu = 0;
    e = dispatch<RunOccupancy>(N, p->nf, flags, &per_cu);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "occupancy query"); }
    if (per_cu < 1) per_cu = 1;
    p->grid = per_cu * p->cus;
    p->block = dispatch<RunShape>(N, 0);
    p->segs = dispatch<RunShape>(N, 1);

    std::vector<float2> tw = dispatch<RunTwiddles>(N);
    e = hipMalloc(&p->twiddles, tw.size() * sizeof(float2));
    if (e != hipSuccess) { destroy_plan(p); (void)hipGetLastError(); return fail(OLS_ERROR_OUT_OF_MEMORY, "twiddle allocation"); }
    e = hipMalloc(&p->spectra, (size_t)K * N * sizeof(float2));
    if (e != hipSuccess) { destroy_plan(p); (void)hipGetLastError(); return fail(OLS_ERROR_OUT_OF_MEMORY, "spectra allocation"); }
    hipStream_t st = (hipStream_t)stream;
    e = hipMemcpyAsync(p->twiddles, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "twiddle upload"); }
    e = dispatch<RunSpectra>(N, h, K, M, p->spectra, (const float2*)p->twiddles, st,
                             (flags & OLS_POST_DERIVATIVE) ? 1 : 0, (flags & OLS_REAL) ? 1 : 0);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "filter spectra launch"); }
    e = hipStreamSynchronize(st);  // the host twiddle buffer and h are released after this
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "plan synchronisation"); }
    *plan = p;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan");
  }
}

ols_status_t ols_plan_update_filters(ols_plan_t p, const void* h, ols_stream_t stream) {
  try {
    if (!p || !h) return fail(OLS_ERROR_INVALID_VALUE, "NULL argument");
    if (((uintptr_t)h) % ((p->flags & OLS_REAL) ? 4 : 8))
      return fail(OLS_ERROR_INVALID_VALUE, "h is not aligned to its element type");
    hipError_t e = dispatch<RunSpectra>(p->N, h, p->K, p->M, p->spectra, (const float2*)p->twiddles,
                                        (hipStream_t)stream, (p->flags & OLS_POST_DERIVATIVE) ? 1 : 0,
                                        (p->flags & OLS_REAL) ? 1 : 0);
    if (e != hipSuccess) return hip_fail(e, "filter spectra launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_update_filters");
  }
}

ols_status_t ols_plan_set_hop(ols_plan_t p, int32_t H) {
  if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
  const int Meff = (p->flags & OLS_POST_DERIVATIVE) ? p->M + 1 : p->M;
  const int L = p->N - Meff + 1;
  if (H == 0) {
    p->D = default_delay(p->N, Meff);
    p->H = p->N - p->D;
    return OLS_SUCCESS;
  }
  if (H < 1 || H > L) return fail(OLS_ERROR_INVALID_VALUE, "hop must satisfy 1 <= H <= N-M+1");
  int D = default_delay(p->N, Meff);
  if (D + H > p->N) D = p->N - H;
  p->D = D;
  p->H = H;
  return OLS_SUCCESS;
}

ols_status_t ols_plan_get_info(ols_plan_t p, int32_t* N, int32_t* H, int32_t* D, int32_t* K, int32_t* M) {
  if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
  if (N) *N = p->N;
  if (H) *H = p->H;
  if (D) *D = p->D;
  if (K) *K = p->K;
  if (M) *M = p->M;
  return OLS_SUCCESS;
}

ols_status_t ols_plan_get_fft_length(ols_plan_t p, int32_t* N) {
  if (!p || !N) return fail(OLS_ERROR_INVALID_VALUE, "NULL argument");
  *N = p->N;
  return OLS_SUCCESS;
}

ols_status_t ols_plan_get_launch(ols_plan_t p, int32_t* grid, int32_t* block, int32_t* cus) {
  if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
  if (grid) *grid = p->grid;
  if (block) *block = p->block;
  if (cus) *cus = p->cus;
  return OLS_SUCCESS;
}

static bool nf_allowed(const ols_plan_s* p, int nf) {
  if (nf == 1) return true;
  if (nf != 2) return false;
  return (p->flags & OLS_REAL) ? p->N <= BATCH_NF2_MAX_N : p->N <= 4096;
}

ols_status_t ols_plan_set_tiling(ols_plan_t p, int32_t nf, int32_t wpc) {
  try {
    if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
    if (nf == 0) nf = (p->flags & OLS_REAL) ? choose_nf_real(p->N, p->K) : choose_nf(p->N, p->K);
    if (!nf_allowed(p, nf)) return fail(OLS_ERROR_INVALID_VALUE, "filters_per_unit must be 1 or 2 (2 only for N <= 4096, R2R N <= 2048)");
    int per_cu = 0;
    hipError_t e = dispatch<RunOccupancy>(p->N, nf, p->flags, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) per_cu = 1;
    if (wpc == 0) wpc = per_cu;
    if (wpc < 1 || wpc > per_cu) return fail(OLS_ERROR_INVALID_VALUE, "workgroups_per_cu must be in [1, occupancy]");
    p->nf = nf;
    p->grid = wpc * p->cus;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_set_tiling");
  }
}

ols_status_t ols_plan_get_tiling(ols_plan_t p, int32_t* nf, int32_t* wpc, int32_t* max_wpc) {
  if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
  if (nf) *nf = p->nf;
  if (wpc) *wpc = p->grid / p->cus;
  if (max_wpc) {
    int per_cu = 0;
    hipError_t e = dispatch<RunOccupancy>(p->N, p->nf, p->flags, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    *max_wpc = per_cu < 1 ? 1 : per_cu;
  }
  return OLS_SUCCESS;
}

ols_status_t ols_plan_get_spectra(ols_plan_t p, void* out, ols_stream_t stream) {
  try {
    if (!p || !out) return fail(OLS_ERROR_INVALID_VALUE, "NULL argument");
    if (((uintptr_t)out) % 8) return fail(OLS_ERROR_INVALID_VALUE, "out must be 8-byte aligned");
    if (ranges_overlap(out, (size_t)p->K * p->N * 8, p->spectra, (size_t)p->K * p->N * 8))
      return fail(OLS_ERROR_INVALID_VALUE, "out overlaps the plan");
    hipError_t e = dispatch<RunNatural>(p->N, (const float2*)p->spectra, p->K, (float2*)out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "spectra copy launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_get_spectra");
  }
}

ols_status_t ols_forward(ols_plan_t p, const void* s, int64_t Ns, void* y, ols_stream_t stream) {
  try {
    if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
    if (Ns < 0) return fail(OLS_ERROR_INVALID_VALUE, "N_s must be >= 0");
    if (Ns == 0) return OLS_SUCCESS;
    if (!s || !y) return fail(OLS_ERROR_INVALID_VALUE, "s or y is NULL");
    const bool real = (p->flags & OLS_REAL) != 0;
    const size_t s_el = real ? 4 : 8;                                       // sample size of s
    const size_t y_el = (real || (p->flags & OLS_POST_POWER)) ? 4 : 8;     // sample size of y
    if (((uintptr_t)s) % s_el || ((uintptr_t)y) % y_el)
      return fail(OLS_ERROR_INVALID_VALUE, "s or y is not aligned to its element type");
    if (Ns > ((int64_t)1 << 56) / 8 / p->K) return fail(OLS_ERROR_INVALID_VALUE, "K*N_s*8 overflows");
    if (ranges_overlap(s, (size_t)Ns * s_el, y, (size_t)Ns * (size_t)p->K * y_el))
      return fail(OLS_ERROR_INVALID_VALUE, "y overlaps s (out of place only)");
    hipError_t e = dispatch<RunForward>(p->N, (const ols_plan_s*)p, s, Ns, y, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_forward");
  }
}

ols_status_t ols_plan_reserve_backward(ols_plan_t p) {
  try {
    if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
    if (p->ws_ds && p->part_dh && p->sum_dh) return OLS_SUCCESS;
    int per_cu = 0;
    hipError_t e = dispatch<RunBwdOccupancy>(p->N, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) per_cu = 1;
    const int grid = per_cu * p->cus;
    const size_t ws = (size_t)grid * 2 * p->segs * p->N * sizeof(float2);
    const size_t part = (size_t)grid * p->segs * p->K * p->M * sizeof(float2);
    const size_t sums = (size_t)dh_chunks((int64_t)grid * p->segs) * p->K * p->M * sizeof(float2);
    float2 *a = nullptr, *b = nullptr, *c = nullptr;
    if (hipMalloc(&a, ws) != hipSuccess || hipMalloc(&b, part) != hipSuccess || hipMalloc(&c, sums) != hipSuccess) {
      if (a) (void)hipFree(a);
      if (b) (void)hipFree(b);
      (void)hipGetLastError();
      return fail(OLS_ERROR_OUT_OF_MEMORY, "backward workspace");
    }
    p->bwd_grid = grid;
    p->ws_ds = a;
    p->part_dh = b;
    p->sum_dh = c;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_reserve_backward");
  }
}

ols_status_t ols_backward(ols_plan_t p, const void* s, int64_t Ns, const void* gy, void* ds, void* dh,
                          ols_stream_t stream) {
  try {
    if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
    if (p->flags != OLS_POST_NONE) return fail(OLS_ERROR_UNSUPPORTED, "backward of a post-processed or R2R plan");
    if (Ns < 0) return fail(OLS_ERROR_INVALID_VALUE, "N_s must be >= 0");
    if (!ds && !dh) return OLS_SUCCESS;
    if (dh && !s && Ns > 0) return fail(OLS_ERROR_INVALID_VALUE, "s is needed for dh");
    if (Ns > 0 && !gy) return fail(OLS_ERROR_INVALID_VALUE, "gradient is NULL");
    const uintptr_t al = (uintptr_t)s | (uintptr_t)gy | (uintptr_t)ds | (uintptr_t)dh;
    if (al % 8) return fail(OLS_ERROR_INVALID_VALUE, "pointers must be 8-byte aligned");
    if (Ns > ((int64_t)1 << 56) / 8 / p->K) return fail(OLS_ERROR_INVALID_VALUE, "K*N_s*8 overflows");
    const size_t sb = (size_t)Ns * 8, gb = (size_t)Ns * 8 * p->K, hb = (size_t)p->K * p->M * 8;
    if (ds && (ranges_overlap(ds, sb, gy, gb) || (s && ranges_overlap(ds, sb, s, sb)) || (dh && ranges_overlap(ds, sb, dh, hb))))
      return fail(OLS_ERROR_INVALID_VALUE, "ds overlaps an input or dh");
    if (dh && (ranges_overlap(dh, hb, gy, gb) || ranges_overlap(dh, hb, s, sb)))
      return fail(OLS_ERROR_INVALID_VALUE, "dh overlaps an input");
    hipStream_t st = (hipStream_t)stream;
    if (Ns == 0) {  // empty signal: dh is zero, ds is empty
      if (dh) {
        hipLaunchKernelGGL(ols_zero_kernel, dim3(64), dim3(256), 0, st, (float2*)dh, (int64_t)p->K * p->M);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "zero launch");
      }
      return OLS_SUCCESS;
    }
    if (!p->ws_ds || !p->part_dh || !p->sum_dh) {
      const ols_status_t r = ols_plan_reserve_backward(p);
      if (r != OLS_SUCCESS) return r;
    }
    hipError_t e = dispatch<RunBackward>(p->N, (const ols_plan_s*)p, (const float2*)s, (const float2*)gy, Ns,
                                         (float2*)ds, (float2*)dh, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_backward");
  }
}

ols_status_t ols_plan_destroy(ols_plan_t p) {
  destroy_plan(p);
  return OLS_SUCCESS;
}

// Validates batch item i and resolves its FFT length (the caller's, or the
// cost model's when it is 0).
static ols_status_t batch_item_fft_length(const ols_batch_item_t& it, int i, int* N_out) {
  const std::string where = "item " + std::to_string(i) + ": ";
  if (it.K < 1 || it.M < 1 || it.N_s < 0) return fail(OLS_ERROR_INVALID_VALUE, where + "K, M >= 1 and N_s >= 0 required");
  if (!it.h || (it.N_s > 0 && (!it.s || !it.y))) return fail(OLS_ERROR_INVALID_VALUE, where + "NULL pointer");
  if (((uintptr_t)it.s | (uintptr_t)it.y | (uintptr_t)it.h) % 8) return fail(OLS_ERROR_INVALID_VALUE, where + "pointers must be 8-byte aligned");
  if (it.N_s > ((int64_t)1 << 56) / 8 / it.K) return fail(OLS_ERROR_INVALID_VALUE, where + "K*N_s*8 overflows");
  if (it.N_s > 0 && ranges_overlap(it.s, (size_t)it.N_s * 8, it.y, (size_t)it.N_s * 8 * it.K))
    return fail(OLS_ERROR_INVALID_VALUE, where + "y overlaps s");
  int N = it.N;
  if (N == 0) {
    double best = 1e301;
    for (int c = OLS_MIN_FFT_LENGTH; c <= OLS_MAX_BATCH_FFT_LENGTH; c *= 2) {
      if (c < it.M) continue;
      const double cost = cost_per_output(c, it.M, it.K);
      if (cost < best) { best = cost; N = c; }
    }
    if (N == 0) return fail(OLS_ERROR_UNSUPPORTED, where + "filter longer than the largest batched FFT length");
  }
  if (!is_pow2(N) || N < OLS_MIN_FFT_LENGTH || N > OLS_MAX_BATCH_FFT_LENGTH)
    return fail(OLS_ERROR_UNSUPPORTED, where + "batched N must be a power of two in [256, 4096]");
  if (it.M > N) return fail(OLS_ERROR_INVALID_VALUE, where + "M must be <= N");
  *N_out = N;
  return OLS_SUCCESS;
}

static size_t batch_twiddle_elems() {
  return RunTwiddles<256>::run().size() + RunTwiddles<512>::run().size() + RunTwiddles<1024>::run().size() +
         RunTwiddles<2048>::run().size() + RunTwiddles<4096>::run().size();
}

ols_status_t ols_batched_workspace_size(const ols_batch_item_t* items, int32_t n, size_t* bytes) {
  try {
    if (!bytes) return fail(OLS_ERROR_INVALID_VALUE, "bytes is NULL");
    *bytes = 0;
    if (!items || n < 1) return fail(OLS_ERROR_INVALID_VALUE, "items is NULL or n < 1");
    size_t spec = 0;
    for (int i = 0; i < n; ++i) {
      int N = 0;
      const ols_status_t r = batch_item_fft_length(items[i], i, &N);
      if (r != OLS_SUCCESS) return r;
      spec += (size_t)items[i].K * N;
    }
    *bytes = (spec + batch_twiddle_elems()) * sizeof(float2) + (size_t)n * sizeof(BatchItem);
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batched_workspace_size");
  }
}

ols_status_t ols_batch_plan(ols_batch_t* out, const ols_batch_item_t* items, int32_t n, ols_stream_t stream) {
  try {
    if (!out) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL");
    *out = nullptr;
    if (!items || n < 1) return fail(OLS_ERROR_INVALID_VALUE, "items is NULL or n < 1");
    ols_batch_s* b = new (std::nothrow) ols_batch_s();
    if (!b) return fail(OLS_ERROR_OUT_OF_MEMORY, "host allocation failed");
    b->n = n;
    b->items_host.resize(n);
    size_t spec_elems = 0;
    int64_t units = 0;
    for (int i = 0; i < n; ++i) {
      const ols_batch_item_t& it = items[i];
      int N = 0;
      const ols_status_t r = batch_item_fft_length(it, i, &N);
      if (r != OLS_SUCCESS) { destroy_batch(b); return r; }
      BatchItem& d = b->items_host[i];
      d.s = (const float2*)it.s;
      d.y = (float2*)it.y;
      d.Ns = it.N_s;
      d.K = it.K;
      d.M = it.M;
      d.N = N;
      d.D = default_delay(N, it.M);
      d.H = N - d.D;
      d.nf = choose_nf_batched(N, it.K);
      const int segs = 4096 / N;  // transforms per 256-thread workgroup
      const int64_t nseg = (it.N_s + d.H - 1) / d.H;
      d.ntiles = (nseg + segs - 1) / segs;
      d.units = d.ntiles * ((it.K + d.nf - 1) / d.nf);
      spec_elems += (size_t)it.K * N;
    }
    // The kernel's tile list takes the items by class (N, filters per unit),
    // in the caller's order within a class, so that each workgroup meets
    // each class in one run of tiles.
    b->order.resize(n);
    for (int i = 0; i < n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
      const BatchItem &u = b->items_host[x], &v = b->items_host[y];
      return u.N != v.N ? u.N < v.N : u.nf < v.nf;
    });
    for (int k = 0; k < n; ++k) {
      BatchItem& d = b->items_host[b->order[k]];
      d.unit_begin = units;
      units += d.units;
      d.tile_begin = b->total_tiles;
      b->total_tiles += d.ntiles;
    }
    b->total_units = units;
    hipError_t e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "hipGetDevice"); }
    if ((e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "hipDeviceGetAttribute"); }
    int per_cu = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ols_batched_kernel, 256, 0)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "occupancy query"); }
    b->grid = (per_cu < 1 ? 1 : per_cu) * b->cus;
    hipStream_t st = (hipStream_t)stream;
    // twiddle tables for every batched N
    std::vector<float2> tws[5] = {RunTwiddles<256>::run(), RunTwiddles<512>::run(), RunTwiddles<1024>::run(),
                                  RunTwiddles<2048>::run(), RunTwiddles<4096>::run()};
    for (int k = 0; k < 5; ++k) {
      if (hipMalloc(&b->tw[k], tws[k].size() * sizeof(float2)) != hipSuccess) { destroy_batch(b); (void)hipGetLastError(); return fail(OLS_ERROR_OUT_OF_MEMORY, "twiddle allocation"); }
      if ((e = hipMemcpyAsync(b->tw[k], tws[k].data(), tws[k].size() * sizeof(float2), hipMemcpyHostToDevice, st)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "twiddle upload"); }
    }
    if (hipMalloc(&b->spectra, spec_elems * sizeof(float2)) != hipSuccess) { destroy_batch(b); (void)hipGetLastError(); return fail(OLS_ERROR_OUT_OF_MEMORY, "spectra allocation"); }
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      BatchItem& d = b->items_host[i];
      float2* F = b->spectra + off;
      d.spectra = F;
      off += (size_t)d.K * d.N;
      const int k = ilog2(d.N) - 8;
      e = dispatch<RunSpectra>(d.N, items[i].h, d.K, d.M, F, (const float2*)b->tw[k], st, 0, 0);
      if (e != hipSuccess) { destroy_batch(b); return hip_fail(e, "filter spectra launch"); }
    }
    b->items_sorted.resize(n);
    for (int k = 0; k < n; ++k) b->items_sorted[k] = b->items_host[b->order[k]];
    if (hipMalloc(&b->items_dev, (size_t)n * sizeof(BatchItem)) != hipSuccess) { destroy_batch(b); (void)hipGetLastError(); return fail(OLS_ERROR_OUT_OF_MEMORY, "item table allocation"); }
    if ((e = hipMemcpyAsync(b->items_dev, b->items_sorted.data(), (size_t)n * sizeof(BatchItem), hipMemcpyHostToDevice, st)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "item table upload"); }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "batch plan synchronisation"); }
    *out = b;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batch_plan");
  }
}

ols_status_t ols_batched(ols_batch_t b, ols_stream_t stream) {
  try {
    if (!b) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL");
    if (b->total_units == 0) return OLS_SUCCESS;
    const int64_t grid = b->total_tiles < b->grid ? b->total_tiles : b->grid;
    hipLaunchKernelGGL(ols_batched_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       (const BatchItem*)b->items_dev, b->n, b->total_tiles, (const float2*)b->tw[0],
                       (const float2*)b->tw[1], (const float2*)b->tw[2], (const float2*)b->tw[3],
                       (const float2*)b->tw[4]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batched");
  }
}

ols_status_t ols_batch_get_info(ols_batch_t b, int64_t* total_units, int32_t* grid, int32_t* n) {
  if (!b) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL");
  if (total_units) *total_units = b->total_units;
  if (grid) *grid = (int32_t)(b->total_tiles < b->grid ? b->total_tiles : b->grid);
  if (n) *n = b->n;
  return OLS_SUCCESS;
}

ols_status_t ols_batch_get_item(ols_batch_t b, int32_t i, int32_t* N, int32_t* H, int32_t* D) {
  if (!b || i < 0 || i >= b->n) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL or item out of range");
  if (N) *N = b->items_host[i].N;
  if (H) *H = b->items_host[i].H;
  if (D) *D = b->items_host[i].D;
  return OLS_SUCCESS;
}

ols_status_t ols_batch_destroy(ols_batch_t b) {
  destroy_batch(b);
  return OLS_SUCCESS;
}

ols_status_t ols_calibration_copy(void* dst, const void* src, size_t bytes, ols_stream_t stream) {
  if (!dst || !src) return fail(OLS_ERROR_INVALID_VALUE, "NULL argument");
  if (bytes % 16 || ((uintptr_t)dst) % 16 || ((uintptr_t)src) % 16)
    return fail(OLS_ERROR_INVALID_VALUE, "size and pointers must be multiples of 16");
  if (ranges_overlap(dst, bytes, src, bytes)) return fail(OLS_ERROR_INVALID_VALUE, "ranges overlap");
  if (bytes == 0) return OLS_SUCCESS;
  const int64_t n = (int64_t)(bytes / 16);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(ols_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (float4*)dst,
                     (const float4*)src, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  return OLS_SUCCESS;
}

}  // extern "C"
