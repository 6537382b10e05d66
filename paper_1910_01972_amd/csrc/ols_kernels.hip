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
#include <mutex>
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
// Filters r0 .. r0 + SEGS - 1 (those < K) of one filter bank, one transform
// per G lanes; the body of the plan step and of the batch setup.
// RowShift: with mask != 0, filter r is delayed by row_delay(y, el, Ns, D,
// r, mask) samples (output rows off the 128-byte line grid).
struct SpectraShift {
  const void* y;
  int64_t Ns;
  int el, D, mask;
};

template <int N>
__device__ __forceinline__ void filter_spectra_block(const void* __restrict__ h, int K, int M, float2* __restrict__ F,
                                                     const float2* __restrict__ twt, int diff, int real, int r0,
                                                     float2* lds, const SpectraShift sh = SpectraShift{}) {
  using GE = Geo<N>;
  const int tid = threadIdx.x;
  const int grp = tid / GE::G, g = tid - grp * GE::G;
  const int r = r0 + grp;
  int par = 0;
  float2 tw[GE::TWR];
  load_lane_twiddles<N>(tw, twt, g);
  float2 x[16];
  const bool valid = r < K;
  const int64_t row = (int64_t)(valid ? r : 0) * M;
  const int delay = sh.mask ? row_delay(sh.y, sh.el, sh.Ns, sh.D, r, sh.mask) : 0;
  if (real) load_filter_real<N>(x, (const float*)h + row, M, valid, diff != 0, g, delay);
  else if (diff) load_filter_diff<N>(x, (const float2*)h + row, M, valid, g, delay);
  else load_filter<N>(x, (const float2*)h + row, M, valid, g, delay);
  fwd_from<N, 0>(x, lds, par, tw, grp, g);
  if (valid) store_spectrum<N>(x, F, r, g, 1.0f / (float)N);
}

template <int N>
__global__ __launch_bounds__(Geo<N>::WG) void ols_filter_spectra_kernel(const void* __restrict__ h, int K, int M,
                                                                        float2* __restrict__ F,
                                                                        const float2* __restrict__ twt, int diff,
                                                                        int real, const SpectraShift sh) {
  __shared__ float2 lds[2 * Geo<N>::LDS];
  filter_spectra_block<N>(h, K, M, F, twt, diff, real, blockIdx.x * Geo<N>::SEGS, lds, sh);
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

// The filter spectra delayed by every d = 0 .. LS-1 samples, for output rows
// off the 128-byte grid: out[d][r] = F[r] * exp(-2 pi i k d / N), in the same
// storage order (the phase from the exact integer k * d mod N, in float64).
// Computed with the spectra, so that a forward call only reads the plan.
template <int N>
__global__ void ols_spectra_delays_kernel(const float2* __restrict__ F, int K, int LS, float2* __restrict__ out) {
  const int64_t KN = (int64_t)K * N;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over LS * K * N
  if (i >= KN * LS) return;
  const int d = (int)(i / KN);
  const int64_t ir = i - d * KN;  // element of F
  const int r = (int)(ir / N);
  const int rem = (int)(ir - (int64_t)r * N);  // = spectrum_offset(reg, g)
  const int pair = rem >> 1, j = pair / Geo<N>::G, g = pair - j * Geo<N>::G;
  const int reg = 2 * j + (rem & 1);
  const int k = spectrum_index<N>(g, reg);
  const int m = (int)(((int64_t)k * d) % N);
  double sn, cs;
  sincospi(2.0 * (double)m / (double)N, &sn, &cs);
  out[i] = cmul(F[ir], make_float2((float)cs, (float)(-sn)));
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
// Spectrum prefetch (PF).  Vector-memory loads and stores share one in-order
// completion counter, so a load issued after a unit's output stores can only
// be waited for once those stores have been acknowledged as well: with the
// spectra loaded at the start of each unit, every unit waits until the
// previous unit's stores have drained.  With PF the spectra of unit u+1 are
// loaded right after unit u's inverse transforms and BEFORE its stores, into a
// second register set; the two sets swap roles from one unit to the next (the
// loop is unrolled by two so that no register copy is needed).  It costs a
// second set of spectrum registers: with one filter per unit it measured
// 2-7 % faster (N = 512, 2048, 4096, 8192; 2-3 % slower at N = 1024 while
// that kernel ran three workgroups per CU), with two filters per unit the
// extra 64 registers halve the occupancy.  prefetch_spectra is the rule of
// the batched kernel's bodies; the single-signal kernel also prefetches at
// N = 1024 for complex outputs: that kernel now needs more than 168 VGPRs
// anyway (two workgroups per CU either way), and prefetch measured 3-4 %
// faster with 8 or 16 filters, level with 1 or 24, and 2 % faster on one
// filter over 2^20 samples.  The power kernel (167 VGPRs, three workgroups
// per CU without it) does not.
template <int N, int NF>
constexpr bool prefetch_spectra() { return NF == 1 && N != 1024; }
template <int N, int NF, bool POWER, bool REAL>
constexpr bool prefetch_spectra_single() { return NF == 1 && (N != 1024 || (!POWER && !REAL)); }

// Exchange buffers of a forward kernel (double-buffered only across waves),
// and its LDS: the buffers, plus, for the non-local stage with transforms no
// wider than a wave, one wave-private set of stage slots per transform (wider
// transforms stage in an exchange buffer, under the exchanges' barriers).
template <int N, int NF>
constexpr int forward_bufs() { return (NF == 1 && Geo<N>::G > 64) ? 2 : NF; }
template <int N, int NF, bool STAGE>
constexpr int forward_lds() {
  return forward_bufs<N, NF>() * Geo<N>::LDS + ((STAGE && Geo<N>::G <= 64) ? Geo<N>::SEGS * stage_stride<N>() : 0);
}

// STAGE: the outputs go through the non-local stencil stage (st) instead of
// the plain store; the output rows then hold st->J * N_s elements.
// shift_mask != 0 (output rows off the 128-byte grid): row r's filter is
// delayed by d_r = row_delay(yv, el, Ns, D, r, shift_mask) samples, and row
// r's kept positions start d_r later.  Its spectrum is row
// r + delay_rows * d_r of F: the plan keeps the spectra for every delay
// (delay_rows = K), a batched item has its rows' delayed spectra computed in
// place (delay_rows = 0).
template <int N, int NF, bool POWER = false, bool REAL = false, int SMODE = STORE_NT_WHOLE,
          bool PF = prefetch_spectra<N, NF>(), bool STAGE = false>
__device__ __forceinline__ void forward_units(const void* __restrict__ sv, int64_t Ns, const float2* __restrict__ F,
                                              void* __restrict__ yv, int K, int D, int H,
                                              const float2 (&tw)[Geo<N>::TWR], int64_t u0, int64_t u1, float2* lds,
                                              int& par, const Stencil* st = nullptr, int shift_mask = 0,
                                              int delay_rows = 0) {
  using GE = Geo<N>;
  const int tid = threadIdx.x;
  const int grp = tid / GE::G, g = tid - grp * GE::G;
  const int KG = (K + NF - 1) / NF;  // filter groups
  const int64_t step = REAL ? 2 * (int64_t)H : H;  // signal advance per transform

  UnitWalk w(u0, KG);
  float2 A[16], xa[NF][16], xb[NF][16];
  // all data lives in global memory: the batched kernel reads these pointers
  // from its item table, where the compiler cannot infer that by itself
  const auto s_c = to_global((const float2*)sv);
  const auto s_r = to_global((const float*)sv);
  const auto Fg = to_global(F);
  const auto y_c = to_global((float2*)yv);
  const auto y_r = to_global((float*)yv);

  // Transform index of this lane (a segment, or a segment pair for REAL);
  // uniform over a wave when a transform spans whole waves (G >= 64).
  auto segment_of = [&](int64_t t) -> int64_t {
    const int64_t sg = t * GE::SEGS + grp;
    return GE::G >= 64 ? wave_uniform64(sg) : sg;
  };
  // segment (pair) sg, forward transformed, into A (x is scratch)
  auto transform_segment = [&](float2 (&x)[16], int64_t sg) {
    if constexpr (REAL) load_segment_pair<N>(x, s_r, Ns, sg * step - D, H, g);
    else load_segment<N>(x, s_c, Ns, sg * step - D, g);
    fwd_from<N, 0>(x, lds, par, tw, grp, g);
#pragma unroll
    for (int i = 0; i < 16; ++i) A[i] = x[i];
  };
  // spectra of filter group q; filters past K (a ragged last group) reuse the
  // last filter's spectrum and are not stored
  constexpr int EL = (REAL || POWER) ? 4 : 8;  // bytes per output sample
  auto load_group = [&](float2 (&x)[NF][16], int q) {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int r = q * NF + f;
      const int rr = r < K ? r : K - 1;
      load_spectrum<N>(x[f], Fg, rr + delay_rows * row_delay(yv, EL, Ns, D, rr, shift_mask), g);
    }
  };
  // stencil phases of filter r's segment (pair) sg, staged at region
  auto stage_out = [&](const float2* region, int r, int64_t sg) {
    const int64_t row = (int64_t)r * st->J * Ns;
    if constexpr (REAL) stage_store<N, POWER, true, SMODE>(region, *st, y_r + row, Ns, sg * step, D, H, g);
    else if constexpr (POWER) stage_store<N, true, false, SMODE>(region, *st, y_r + row, Ns, sg * H, D, H, g);
    else stage_store<N, false, false, SMODE>(region, *st, y_c + row, Ns, sg * H, D, H, g);
  };
  auto stage_group = [&](const float2 (&x)[NF][16], int q, int64_t sg) {
    if constexpr (GE::G <= 64) {
      // a transform lies in one wave, whose LDS operations complete in order:
      // its own stage slots need fences against compiler reordering only
      float2* region = lds + forward_bufs<N, NF>() * GE::LDS + grp * stage_stride<N>();
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        stage_write<N>(region, x[f], g);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int r = q * NF + f;
        if (NF == 1 || r < K) stage_out(region, r, sg);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    } else {
      static_assert(GE::SEGS * stage_stride<N>() <= GE::LDS, "stage slots fit in an exchange buffer");
      if constexpr (NF == 1) {
        // one more exchange of the two-buffer sequence (see exchange)
        float2* region = lds + (par ? GE::LDS : 0) + grp * stage_stride<N>();
        par ^= 1;
        stage_write<N>(region, x[0], g);
        __syncthreads();
        stage_out(region, q, sg);
      } else {
        // as exchange_nf: one buffer per filter, a barrier after the writes
        // and one after the reads
#pragma unroll
        for (int f = 0; f < NF; ++f) stage_write<N>(lds + f * GE::LDS + grp * stage_stride<N>(), x[f], g);
        __syncthreads();
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const int r = q * NF + f;
          if (r < K) stage_out(lds + f * GE::LDS + grp * stage_stride<N>(), r, sg);
        }
        __syncthreads();
      }
    }
  };
  auto store_group = [&](const float2 (&x)[NF][16], int q, int64_t sg) {
    if constexpr (STAGE) {
      stage_group(x, q, sg);
      return;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int r = q * NF + f;
      if (NF == 1 || r < K) {
        const int Dr = D + row_delay(yv, EL, Ns, D, r, shift_mask);  // first kept position of row r
        if constexpr (REAL)
          store_valid_pair<N, POWER, SMODE>(x[f], y_r + (int64_t)r * Ns, Ns, sg * step, Dr, H, g);
        else if constexpr (POWER)
          store_valid_power<N, SMODE>(x[f], y_r + (int64_t)r * Ns, Ns, sg * step, Dr, H, g);
        else
          store_valid<N, SMODE>(x[f], y_c + (int64_t)r * Ns, Ns, sg * step, Dr, H, g);
      }
    }
  };

  int64_t seg = segment_of(w.tile);
  if constexpr (PF) {
    load_group(xa, w.rg);
    transform_segment(xb[0], seg);
    // cur holds unit u's spectra on entry; nxt is free and receives unit u+1's
    auto unit = [&](float2 (&cur)[NF][16], float2 (&nxt)[NF][16], int64_t u) {
      if (w.tile_done(KG)) {  // next tile: new segments, one forward transform each
        w.next_tile();
        seg = segment_of(w.tile);
        transform_segment(nxt[0], seg);
      }
      inverse_of_products<N, NF>(cur, A, lds, par, tw, grp, g);
      if (u + 1 < u1) load_group(nxt, w.next_group(KG));
      __builtin_amdgcn_sched_barrier(0);  // keep those loads ahead of the stores
      store_group(cur, w.rg, seg);
      w.leave();
    };
    int64_t u = u0;
    for (; u + 1 < u1; u += 2) {
      unit(xa, xb, u);
      unit(xb, xa, u + 1);
    }
    if (u < u1) unit(xa, xb, u);
  } else {
    transform_segment(xa[0], seg);
    for (int64_t u = u0; u < u1; ++u) {
      if (w.tile_done(KG)) {
        w.next_tile();
        seg = segment_of(w.tile);
        transform_segment(xa[0], seg);
      }
      load_group(xa, w.rg);
      inverse_of_products<N, NF>(xa, A, lds, par, tw, grp, g);
      store_group(xa, w.rg, seg);
      w.leave();
    }
  }
}

template <int N, int NF, bool POWER = false, bool REAL = false, int SMODE = STORE_NT_WHOLE, bool STAGE = false>
__device__ __forceinline__ void forward_range(const void* __restrict__ sv, int64_t Ns, const float2* __restrict__ F,
                                              void* __restrict__ yv, int K, int D, int H,
                                              const float2* __restrict__ twt, int64_t u0, int64_t u1, float2* lds,
                                              int& par, const Stencil* st = nullptr, int shift_mask = 0) {
  float2 tw[Geo<N>::TWR];
  load_lane_twiddles<N>(tw, twt, threadIdx.x % Geo<N>::G);
  // the stage's accumulators take the registers of the spectrum prefetch
  forward_units<N, NF, POWER, REAL, SMODE, prefetch_spectra_single<N, NF, POWER, REAL>() && !STAGE, STAGE>(
      sv, Ns, F, yv, K, D, H, tw, u0, u1, lds, par, st, shift_mask, K);
}

// shift_mask: 0, or the row shift of output rows off the 128-byte line grid
// (row_shift_geometry; F then holds the delayed filters).
template <int N, int NF, bool POWER, bool REAL>
__global__ __launch_bounds__(Geo<N>::WG) void ols_forward_kernel(const void* __restrict__ s, int64_t Ns,
                                                                 const float2* __restrict__ F, void* __restrict__ y,
                                                                 int K, int D, int H, int64_t ntiles,
                                                                 const float2* __restrict__ twt, int shift_mask) {
  __shared__ float2 lds[forward_lds<N, NF, false>()];
  const int64_t U = ntiles * ((K + NF - 1) / NF);
  const int64_t u0 = first_unit(U, gridDim.x, blockIdx.x);
  const int64_t u1 = first_unit(U, gridDim.x, blockIdx.x + 1);
  if (u0 >= u1) return;  // uniform over the workgroup
  int par = 0;
  forward_range<N, NF, POWER, REAL>(s, Ns, F, y, K, D, H, twt, u0, u1, lds, par, nullptr, shift_mask);
}

// The forward kernel with the non-local post-processing stage (sec. 4): the
// same units, each filter's output staged in LDS and stored as st's phases.
template <int N, int NF, bool POWER, bool REAL>
__global__ __launch_bounds__(Geo<N>::WG) __attribute__((amdgpu_waves_per_eu(2))) void ols_forward_stencil_kernel(const void* __restrict__ s, int64_t Ns,
                                                                         const float2* __restrict__ F,
                                                                         void* __restrict__ y, int K, int D, int H,
                                                                         int64_t ntiles,
                                                                         const float2* __restrict__ twt,
                                                                         const Stencil st) {
  __shared__ float2 lds[forward_lds<N, NF, true>()];
  const int64_t U = ntiles * ((K + NF - 1) / NF);
  const int64_t u0 = first_unit(U, gridDim.x, blockIdx.x);
  const int64_t u1 = first_unit(U, gridDim.x, blockIdx.x + 1);
  if (u0 >= u1) return;  // uniform over the workgroup
  int par = 0;
  forward_range<N, NF, POWER, REAL, STORE_NT_WHOLE, true>(s, Ns, F, y, K, D, H, twt, u0, u1, lds, par, &st);
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
  const void* h;          // the caller's filters [K][M] (read by the spectra step)
  int64_t Ns;
  int64_t unit_begin;
  int64_t units;
  int32_t K, M, N, D, H, nf;
  int64_t tile_begin;  // first tile of this item in the batch's tile list
  int64_t ntiles;      // tiles of this item (units = ntiles * units per tile)
  int32_t shift_mask;  // rows off the 128-byte grid: filters delayed by row_delay with this mask
  int32_t pad;
};

// Values the batch setup computes on the device: totals over all items and
// the outcome of its checks.  Every later kernel of a batched call reads
// status first and does nothing unless it is OLS_SUCCESS.
struct BatchHeader {
  int32_t status;       // ols_status_t of the device-side checks
  int32_t bad_item;     // first failing item (caller's numbering), -1 if none
  int32_t n;
  int32_t pad;
  int64_t total_tiles;  // segment tiles of all items
  int64_t total_tasks;  // spectrum tasks (one workgroup's filters of one item)
  int64_t spec_elems;   // complex64 elements of filter spectra the items need
};

// Where each part of a batch's device state lives: in the caller's
// workspace (ols_batched) or in a batch plan's own allocation.  Passed to
// every batch kernel by value.
constexpr int BATCH_LENGTHS = 5;  // N = 256, 512, 1024, 2048, 4096
struct BatchLayout {
  BatchHeader* hdr;
  BatchItem* items;     // [n], in kernel order (by class, stable)
  int64_t* task_begin;  // [n + 1], first spectrum task of each item (kernel order)
  int32_t* order;       // [n], caller's index of each kernel-order item
  float2* tw[BATCH_LENGTHS];
  float2* spectra;
  int64_t spec_capacity;  // complex64 elements available at `spectra`
  int32_t n;
};

// ---------------------------------------------------------------------------
// Batch setup: one workgroup reads the caller's items (a device array),
// checks them, chooses each item's FFT length, orders the items by class
// (N, filters per unit) -- a stable counting sort -- and lays out the tile
// list, the spectrum tasks and the spectra with prefix sums.  It also writes
// the twiddle tables of the five batched lengths, evaluated in float64 from
// the exact reduced angle and rounded once to float32.
// ---------------------------------------------------------------------------
constexpr int SETUP_THREADS = 1024;

// Exclusive prefix sum over the workgroup of one value per thread; *total
// receives the sum over all threads.  sh holds SETUP_THREADS values.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SETUP_THREADS; off <<= 1) {
    const int64_t a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const int64_t incl = sh[t];
  *total = sh[SETUP_THREADS - 1];
  __syncthreads();  // sh is reused by the next scan
  return incl - v;
}

template <int N>
__device__ void device_twiddles(float2* __restrict__ out) {
  using GE = Geo<N>;
#pragma unroll
  for (int k = 0; k < GE::P - 1; ++k) {
    const int L = GE::len(k), S = GE::strd(k), cnt = GE::tw_count(k);
    for (int idx = threadIdx.x; idx < cnt; idx += SETUP_THREADS) {
      const int b = idx / S + 1, l = idx - (b - 1) * S;
      const int m = (int)(((int64_t)l * b) % L);
      double sn, cs;
      sincospi(2.0 * (double)m / (double)L, &sn, &cs);  // exp(-2 pi i m / L) = cos - i sin
      out[GE::tw_offset(k) + idx] = make_float2((float)cs, (float)(-sn));
    }
  }
}

struct ItemShape {
  int N, nf, cls, D, H, shift_mask;
  int64_t ntiles, units, spec, tasks;
};

__device__ __forceinline__ ItemShape item_shape(const ols_batch_item_t& it, int N) {
  ItemShape r;
  r.N = N;
  r.nf = choose_nf_batched(N, it.K);
  r.cls = batch_class(N, r.nf);
  r.D = default_delay(N, it.M);
  const RowShift rs = batch_row_shift(it.y, it.N_s, N, r.D);
  r.shift_mask = rs.mask;
  r.H = rs.H;
  const int H = r.H;
  const int segs = 4096 / N;  // transforms per 256-thread workgroup
  const int64_t nseg = (it.N_s + H - 1) / H;
  r.ntiles = (nseg + segs - 1) / segs;
  r.units = r.ntiles * ((it.K + r.nf - 1) / r.nf);
  r.spec = (int64_t)it.K * N;
  r.tasks = (it.K + segs - 1) / segs;
  return r;
}

__global__ __launch_bounds__(SETUP_THREADS) void ols_batch_setup_kernel(const ols_batch_item_t* __restrict__ in,
                                                                         BatchLayout L) {
  __shared__ int cnt[BATCH_CLASSES][SETUP_THREADS];
  __shared__ int64_t sh[SETUP_THREADS];
  __shared__ int64_t cls_total[BATCH_CLASSES];
  __shared__ unsigned long long s_fail;
  const int t = threadIdx.x, n = L.n;
  const int chunk = (n + SETUP_THREADS - 1) / SETUP_THREADS;
  const int i0 = t * chunk < n ? t * chunk : n;
  const int i1 = i0 + chunk < n ? i0 + chunk : n;
  if (t == 0) s_fail = ~0ull;
  __syncthreads();

  // 1. check every item, count the items of each class in this thread's chunk
  int local[BATCH_CLASSES];
#pragma unroll
  for (int c = 0; c < BATCH_CLASSES; ++c) local[c] = 0;
  for (int i = i0; i < i1; ++i) {
    const ols_batch_item_t it = in[i];
    int N = 0;
    const int st = batch_item_check(it.s, it.N_s, it.h, it.K, it.M, it.N, it.y, &N);
    if (st != 0) {
      atomicMin(&s_fail, ((unsigned long long)i << 8) | (unsigned)st);
      continue;
    }
    ++local[batch_class(N, choose_nf_batched(N, it.K))];
  }
  __syncthreads();
  if (s_fail != ~0ull) {  // uniform: no item is processed
    if (t == 0) {
      L.hdr->status = (int32_t)(s_fail & 0xff);
      L.hdr->bad_item = (int32_t)(s_fail >> 8);
      L.hdr->n = n;
      L.hdr->total_tiles = 0;
      L.hdr->total_tasks = 0;
      L.hdr->spec_elems = 0;
    }
    return;
  }

  // 2. stable counting sort by class: exclusive prefix of every class's
  // counts over the threads, then class bases
#pragma unroll
  for (int c = 0; c < BATCH_CLASSES; ++c) {
    int64_t tot;
    cnt[c][t] = (int)block_exclusive_scan(local[c], sh, &tot);
    if (t == 0) cls_total[c] = tot;
  }
  __syncthreads();
  int64_t base[BATCH_CLASSES];
  {
    int64_t acc = 0;
#pragma unroll
    for (int c = 0; c < BATCH_CLASSES; ++c) {
      base[c] = acc + cnt[c][t];
      acc += cls_total[c];
    }
  }
  for (int i = i0; i < i1; ++i) {
    const ols_batch_item_t it = in[i];
    int N = 0;
    (void)batch_item_check(it.s, it.N_s, it.h, it.K, it.M, it.N, it.y, &N);
    const ItemShape sh_ = item_shape(it, N);
    const int64_t pos = base[sh_.cls]++;
    BatchItem b;
    b.s = (const float2*)it.s;
    b.y = (float2*)it.y;
    b.spectra = nullptr;
    b.h = it.h;
    b.Ns = it.N_s;
    b.unit_begin = 0;
    b.units = sh_.units;
    b.K = it.K;
    b.M = it.M;
    b.N = N;
    b.D = sh_.D;
    b.H = sh_.H;
    b.shift_mask = sh_.shift_mask;
    b.pad = 0;
    b.nf = sh_.nf;
    b.tile_begin = 0;
    b.ntiles = sh_.ntiles;
    L.items[pos] = b;
    L.order[pos] = i;
  }
  __syncthreads();  // the sorted table is complete (workgroup-scope visibility of global writes)

  // 3. prefix sums in kernel order: tiles, units, spectra, spectrum tasks
  int64_t my_tiles = 0, my_units = 0, my_spec = 0, my_tasks = 0;
  for (int p = i0; p < i1; ++p) {
    const BatchItem& b = L.items[p];
    my_tiles += b.ntiles;
    my_units += b.units;
    my_spec += (int64_t)b.K * b.N;
    my_tasks += (b.K + 4096 / b.N - 1) / (4096 / b.N);
  }
  int64_t tot_tiles, tot_units, tot_spec, tot_tasks;
  int64_t o_tiles = block_exclusive_scan(my_tiles, sh, &tot_tiles);
  int64_t o_units = block_exclusive_scan(my_units, sh, &tot_units);
  int64_t o_spec = block_exclusive_scan(my_spec, sh, &tot_spec);
  int64_t o_tasks = block_exclusive_scan(my_tasks, sh, &tot_tasks);
  const bool fits = tot_spec <= L.spec_capacity;
  for (int p = i0; p < i1; ++p) {
    BatchItem& b = L.items[p];
    b.tile_begin = o_tiles;
    b.unit_begin = o_units;
    b.spectra = fits ? L.spectra + o_spec : nullptr;
    L.task_begin[p] = o_tasks;
    o_tiles += b.ntiles;
    o_units += b.units;
    o_spec += (int64_t)b.K * b.N;
    o_tasks += (b.K + 4096 / b.N - 1) / (4096 / b.N);
  }
  if (t == 0) {
    L.task_begin[n] = tot_tasks;
    L.hdr->status = fits ? 0 : (int32_t)OLS_ERROR_INVALID_VALUE;
    L.hdr->bad_item = -1;
    L.hdr->n = n;
    L.hdr->total_tiles = tot_tiles;
    L.hdr->total_tasks = tot_tasks;
    L.hdr->spec_elems = tot_spec;
  }

  // 4. twiddle tables
  device_twiddles<256>(L.tw[0]);
  device_twiddles<512>(L.tw[1]);
  device_twiddles<1024>(L.tw[2]);
  device_twiddles<2048>(L.tw[3]);
  device_twiddles<4096>(L.tw[4]);
}

// One length's spectrum body as its own function, so the kernel's register
// count is the largest body's rather than the sum of all five.
template <int N>
__device__ __attribute__((noinline)) void batch_spectra_task(const BatchItem& it, const float2* __restrict__ twt,
                                                              int r0, float2* lds) {
  filter_spectra_block<N>(it.h, it.K, it.M, (float2*)it.spectra, twt, 0, 0, r0, lds,
                          SpectraShift{it.y, it.Ns, 8, it.D, it.shift_mask});
}

// Filter spectra of every item: task tau is one workgroup's filters of one
// item (SEGS = 4096 / N of them); persistent workgroups take tasks b, b + P, ...
__global__ __launch_bounds__(256) void ols_batch_spectra_kernel(BatchLayout L) {
  __shared__ float2 lds[2 * Geo<4096>::LDS];
  if (L.hdr->status != 0) return;
  const int64_t tasks = L.hdr->total_tasks;
  for (int64_t tau = blockIdx.x; tau < tasks; tau += gridDim.x) {
    // the item whose task range holds tau: task_begin[i] <= tau < task_begin[i + 1]
    int lo = 0, hi = L.n;  // invariant: task_begin[lo] <= tau < task_begin[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (L.task_begin[mid] <= tau) lo = mid;
      else hi = mid;
    }
    const BatchItem& it = L.items[lo];
    const int r0 = (int)(tau - L.task_begin[lo]) * (4096 / it.N);
    __syncthreads();  // the previous task's transform may still read LDS
    switch (it.N) {
      case 256: batch_spectra_task<256>(it, L.tw[0], r0, lds); break;
      case 512: batch_spectra_task<512>(it, L.tw[1], r0, lds); break;
      case 1024: batch_spectra_task<1024>(it, L.tw[2], r0, lds); break;
      case 2048: batch_spectra_task<2048>(it, L.tw[3], r0, lds); break;
      default: batch_spectra_task<4096>(it, L.tw[4], r0, lds); break;
    }
  }
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

// Each (N, filters per unit) body is its own non-inlined function, so its
// registers are allocated on their own and the kernel needs only the
// maximum, not the sum, over the branches it may take.  A body runs the
// workgroup's tiles t, t + P, t + 2P, ... for as long as their items keep its
// (N, filters per unit): the lane twiddles are loaded once per run, and
// consecutive tiles of one class need no barrier between them (the same
// exchange protocol as consecutive tiles of the single-signal kernel).  The
// setup orders the items by class, so a workgroup meets each class in one
// run.  Returns the workgroup's first tile of another class (or past the
// end); i follows the item walk.
// The fields of one item, read through a global pointer (see gptr).  The
// whole workgroup works on one item at a time (i is uniform), so the fields
// are declared wave-uniform: address arithmetic stays scalar and the store
// descriptors need no per-lane loop.
__device__ __forceinline__ BatchItem read_item(gptr<const BatchItem> items, int i) {
  BatchItem r;
  r.s = wave_uniform_ptr(items[i].s);
  r.y = wave_uniform_ptr(items[i].y);
  r.spectra = wave_uniform_ptr(items[i].spectra);
  r.h = wave_uniform_ptr(items[i].h);
  r.Ns = wave_uniform64(items[i].Ns);
  r.unit_begin = wave_uniform64(items[i].unit_begin);
  r.units = wave_uniform64(items[i].units);
  r.K = __builtin_amdgcn_readfirstlane(items[i].K);
  r.M = __builtin_amdgcn_readfirstlane(items[i].M);
  r.N = __builtin_amdgcn_readfirstlane(items[i].N);
  r.D = __builtin_amdgcn_readfirstlane(items[i].D);
  r.H = __builtin_amdgcn_readfirstlane(items[i].H);
  r.nf = __builtin_amdgcn_readfirstlane(items[i].nf);
  r.tile_begin = wave_uniform64(items[i].tile_begin);
  r.ntiles = wave_uniform64(items[i].ntiles);
  r.shift_mask = __builtin_amdgcn_readfirstlane(items[i].shift_mask);
  return r;
}

// Where a workgroup's walk over the tiles stands between class runs: its next
// tile, the item it is in, and the parity of its next LDS exchange buffer
// (passed by value so that no state goes through the stack).
struct BatchWalk {
  int64_t t;
  int i;
  int par;
};

template <int N, int NF>
__device__ __attribute__((noinline)) BatchWalk batched_run(const BatchItem* __restrict__ items_in, int nitems,
                                                           BatchWalk w, int64_t total_tiles,
                                                           const float2* __restrict__ twt, float2* lds) {
  const gptr<const BatchItem> items = to_global(items_in);
  int64_t t = w.t;
  int i = w.i, par = w.par;
  const int64_t P = gridDim.x;
  float2 tw[Geo<N>::TWR];
  load_lane_twiddles<N>(tw, to_global(twt), threadIdx.x % Geo<N>::G);
  for (;;) {
    const BatchItem it = read_item(items, i);
    const int64_t per_tile = it.units / it.ntiles;
    const int64_t a = (t - it.tile_begin) * per_tile;
    forward_units<N, NF, false, false, STORE_NT_WHOLE>(it.s, it.Ns, it.spectra, it.y, it.K, it.D, it.H, tw, a,
                                                       a + per_tile, lds, par, nullptr, it.shift_mask);
    t = next_batch_tile(t, P);
    if (t >= total_tiles) return BatchWalk{t, i, par};
    // t grows, so the item walk only moves forward (items without tiles are skipped)
    while (i + 1 < nitems && items[i + 1].tile_begin <= t) ++i;
    if (items[i].N != N || items[i].nf != NF) return BatchWalk{t, i, par};
  }
}

// Two filters per unit only up to N = 2048 here (BATCH_NF2_MAX_N): the
// N = 4096 two-filter body needs more than 256 registers as a separate
// function, which would drop the whole kernel to one wave per SIMD.

template <int N>
__device__ __forceinline__ BatchWalk batched_class(const BatchItem* __restrict__ items, int nitems, BatchWalk w,
                                                   int64_t total_tiles, const float2* __restrict__ twt, float2* lds) {
  if constexpr (N <= BATCH_NF2_MAX_N) {
    if (to_global(items)[w.i].nf == 2) return batched_run<N, 2>(items, nitems, w, total_tiles, twt, lds);
  }
  return batched_run<N, 1>(items, nitems, w, total_tiles, twt, lds);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ols_batched_kernel(BatchLayout L) {
  __shared__ float2 lds[2 * Geo<4096>::LDS];
  static_assert(Geo<256>::LDS == Geo<4096>::LDS && Geo<2048>::LDS == Geo<4096>::LDS, "same LDS footprint");
  if (L.hdr->status != 0) return;
  const int64_t total_tiles = L.hdr->total_tiles;
  const BatchItem* __restrict__ items = L.items;
  const int nitems = L.n;
  // Tiles of all items, in the setup's item order, dealt round-robin in
  // chunks to the workgroups (first_batch_tile, next_batch_tile,
  // batch_workgroup_order), each tile with all of its filters.  At any moment
  // the whole grid works on neighbouring tiles of one or two items, so the L2s
  // keep those items' filter spectra (balanced contiguous unit ranges spread
  // the grid over all items at once and re-read the spectra from HBM: 19 %
  // slower on the uneven batch).  The imbalance is at most one chunk per
  // workgroup.
  const int64_t P = gridDim.x;
  BatchWalk w{first_batch_tile(batch_workgroup_order(blockIdx.x, P)), 0, 0};
  const gptr<const BatchItem> gitems = to_global(items);
  while (w.t < total_tiles) {
    while (w.i + 1 < nitems && gitems[w.i + 1].tile_begin <= w.t) ++w.i;
    // items of another class lay out the LDS buffers differently, and
    // single-wave transforms exchange without barriers: every wave must have
    // finished with the previous run's buffers
    __syncthreads();
    switch (gitems[w.i].N) {
      case 256: w = batched_class<256>(items, nitems, w, total_tiles, L.tw[0], lds); break;
      case 512: w = batched_class<512>(items, nitems, w, total_tiles, L.tw[1], lds); break;
      case 1024: w = batched_class<1024>(items, nitems, w, total_tiles, L.tw[2], lds); break;
      case 2048: w = batched_class<2048>(items, nitems, w, total_tiles, L.tw[3], lds); break;
      default: w = batched_class<4096>(items, nitems, w, total_tiles, L.tw[4], lds); break;
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

// ---------------------------------------------------------------------------
// Adjoint with paired segments (N <= 2048).  dh_r takes the first M lags of
// IFFT(sum_j conj(S_j)/N * G_{r,j}) over the segments j, and the inverse
// transform is linear, so the products of two segments may be added before a
// single inverse.  The workgroup holds BwdGeo<N>::SEGS transforms; groups 2p
// and 2p+1 form a pair working on two neighbouring segments of one tile.  A
// unit is (tile, filter pair r = 2q, 2q+1): every group forward transforms
// its segment's gradient window for both filters (both feed its ds
// accumulator), keeps the product for the filter it collects (the parity of
// its group index) and hands the other product to its partner through LDS;
// then each group adds the partner's product to its own and runs one inverse
// for its filter.  Per (segment, filter): one forward transform and half an
// inverse, against one of each in ols_backward_kernel, and half the dh
// read-modify-writes.  A filter index past K (odd K) is transformed like the
// last filter and then ignored, so that every group meets the same barriers.
// ---------------------------------------------------------------------------
template <int N>
struct BwdGeo {
  using GE = Geo<N>;
  // two transforms at least (a 512-thread workgroup at N = 4096, were it used)
  static constexpr int WG = GE::WG / GE::G >= 2 ? GE::WG : 2 * GE::G;
  static constexpr int SEGS = WG / GE::G;
  static constexpr int lds_e(int e) { return GE::pad(e, SEGS * N - 1) + 1; }
  static constexpr int lds_max(int e) { return e < 0 ? 1 : (lds_e(e) > lds_max(e - 1) ? lds_e(e) : lds_max(e - 1)); }
  static constexpr int XLDS = lds_max(GE::P - 2);  // exchange buffer (float2)
  static constexpr int HLDS = SEGS * N;            // hand-over buffer (float2)
  static_assert(SEGS % 2 == 0, "groups come in pairs");
};

// One exchange through a single LDS buffer: the buffer is reused by the next
// exchange, so transforms that span several waves also need the trailing
// barrier (single-wave transforms exchange in program order).
template <int N, int E, int KW, int KR>
__device__ __forceinline__ void exchange_single(float2 (&x)[16], float2* buf, int grp, int g) {
  lds_store<N, E, KW>(buf, x, grp, g);
  exchange_sync<N>();
  lds_load<N, E, KR>(buf, x, grp, g);
  if constexpr (Geo<N>::G > 64) __syncthreads();
}

template <int N, int K>
__device__ __forceinline__ void fwd_single(float2 (&x)[16], float2* buf, const float2* tw, int grp, int g) {
  run_pass<N, K, false>(x, tw + Geo<N>::lane_tw_offset(K));
  if constexpr (K + 1 < Geo<N>::P) {
    exchange_single<N, K, K, K + 1>(x, buf, grp, g);
    fwd_single<N, K + 1>(x, buf, tw, grp, g);
  }
}

template <int N, int K>
__device__ __forceinline__ void inv_single(float2 (&x)[16], float2* buf, const float2* tw, int grp, int g) {
  inverse_pass<N, K>(x, tw + Geo<N>::lane_tw_offset(K));
  if constexpr (K > 0) {
    exchange_single<N, K - 1, K, K - 1>(x, buf, grp, g);
    inv_single<N, K - 1>(x, buf, tw, grp, g);
  }
}

// Synchronisation of the hand-over between the two groups of a pair: a fence
// when the pair shares a wave, a barrier otherwise.
template <int N>
__device__ __forceinline__ void pair_sync() {
  if constexpr (2 * Geo<N>::G <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int N>
__global__ __launch_bounds__(BwdGeo<N>::WG) __attribute__((amdgpu_waves_per_eu(2))) void ols_backward_pair_kernel(
    const float2* __restrict__ s, const float2* __restrict__ gy, int64_t Ns, const float2* __restrict__ F, int K,
    int M, int H, int64_t ntiles, const float2* __restrict__ twt, float2* __restrict__ ds,
    float2* __restrict__ ws_ds, float2* __restrict__ part_dh, int want_ds, int want_dh) {
  using GE = Geo<N>;
  using BG = BwdGeo<N>;
  __shared__ float2 lds[BG::XLDS + BG::HLDS];
  float2* const xbuf = lds;
  float2* const hbuf = lds + BG::XLDS;
  const int tid = threadIdx.x;
  const int grp = tid / GE::G, g = tid - grp * GE::G;
  const int side = grp & 1;  // parity of the filters this group collects
  const int KP = (K + 1) / 2;
  const int64_t P = gridDim.x, b = blockIdx.x;
  const int64_t U = ntiles * KP;
  const int64_t u0 = first_unit(U, P, b), u1 = first_unit(U, P, b + 1);
  if (u0 >= u1) return;  // uniform over the workgroup

  float2 tw[GE::TWR];
  load_lane_twiddles<N>(tw, twt, g);
  float2* part = part_dh + (b * BG::SEGS + grp) * (int64_t)K * M;
  if (want_dh)
    for (int r = 0; r < K; ++r) zero_lags<N>(part + (int64_t)r * M, M, g);

  const int64_t t_first = u0 / KP;
  int64_t tile = t_first;
  int q = (int)(u0 - tile * KP);
  float2 S[16], E[16], mine[16], x[16], f[16];
  auto segment_of = [&](int64_t t) -> int64_t {
    const int64_t sg = t * BG::SEGS + grp;
    return GE::G >= 64 ? wave_uniform64(sg) : sg;
  };
  int64_t seg = segment_of(tile);

  auto start_tile = [&]() {
    seg = segment_of(tile);
    if (want_dh) {
      load_window<N>(x, s, Ns, seg * H, H, g);
      fwd_single<N, 0>(x, xbuf, tw, grp, g);
      conj_scaled(S, x, 1.0f / (float)N);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) E[i] = make_float2(0.f, 0.f);
  };
  auto finish_tile = [&]() {
    if (!want_ds) return;
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = E[i];
    inv_single<N, GE::P - 1>(x, xbuf, tw, grp, g);
    const bool complete = tile * KP >= u0 && (tile + 1) * KP <= u1;
    if (complete) {
      store_valid<N>(x, ds, Ns, seg * H, 0, H, g);
    } else {
      const int slot = tile == t_first ? 0 : 1;
      float2* w = ws_ds + ((b * 2 + slot) * BG::SEGS + grp) * (int64_t)N;
      store_valid<N>(x, w, (int64_t)H, 0, 0, H, g);
    }
  };
  // gradient window of filter r (r < K) of this group's segment, forward
  // transformed into x and accumulated into E when it is a real filter
  auto gradient_spectrum = [&](int r) {
    const bool real_filter = r < K;
    const int rr = real_filter ? r : K - 1;
    load_window<N>(x, gy + (int64_t)rr * Ns, Ns, seg * H, N, g);
    fwd_single<N, 0>(x, xbuf, tw, grp, g);
    if (want_ds && real_filter) {
      load_spectrum<N>(f, F, rr, g);
      acc_conj_product(E, x, f);
    }
  };

  start_tile();
  for (int64_t u = u0; u < u1; ++u) {
    if (q == KP) {
      finish_tile();
      q = 0;
      ++tile;
      start_tile();
    }
    const int r_other = 2 * q + (1 - side), r_own = 2 * q + side;
    // the partner's filter first: its product goes to the hand-over buffer
    gradient_spectrum(r_other);
    if (want_dh) {
#pragma unroll
      for (int i = 0; i < 16; ++i) hbuf[(grp * 16 + i) * GE::G + g] = cmul(S[i], x[i]);
    }
    gradient_spectrum(r_own);
    if (want_dh) {
#pragma unroll
      for (int i = 0; i < 16; ++i) mine[i] = cmul(S[i], x[i]);
      pair_sync<N>();
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = cadd(mine[i], hbuf[((grp ^ 1) * 16 + i) * GE::G + g]);
      // single-wave transforms exchange without barriers: keep the partner
      // from overwriting the hand-over buffer before it has been read
      if constexpr (GE::G == 64) __syncthreads();
      inv_single<N, GE::P - 1>(x, xbuf, tw, grp, g);
      if (r_own < K) add_lags<N>(part + (int64_t)r_own * M, x, M, g);
    }
    ++q;
  }
  finish_tile();
}

// Sums the partial ds windows of tiles split between workgroups; block b-1
// handles the boundary between workgroups b-1 and b (the first boundary
// inside a tile does the whole tile).  SEGS transforms per tile, K units per
// tile (the filters, or the filter pairs of the paired adjoint).
template <int N, int SEGS>
__global__ void ols_ds_fixup_kernel(const float2* __restrict__ ws_ds, float2* __restrict__ ds, int64_t Ns, int K,
                                    int H, int64_t ntiles, int64_t P) {
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
  for (int sg = 0; sg < SEGS; ++sg) {
    const int64_t o0 = (t * SEGS + sg) * H;
    for (int p = threadIdx.x + blockIdx.y * blockDim.x; p < H; p += stride) {
      if (o0 + p >= Ns) break;
      // the sharing workgroups' windows in workgroup order, loaded four at a
      // time so that the loads overlap
      float2 a = make_float2(0.f, 0.f);
      int64_t bb = blo;
      for (; bb + 4 <= bhi + 1; bb += 4) {
        float2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int64_t slot = bb + k == blo ? slot_lo : 0;
          v[k] = ws_ds[(((bb + k) * 2 + slot) * SEGS + sg) * (int64_t)N + p];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) a = cadd(a, v[k]);
      }
      if (bb <= bhi) {
        // the last one to three windows
        float2 v[3];
        const int rem = (int)(bhi + 1 - bb);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int64_t slot = bb + k == blo ? slot_lo : 0;
          v[k] = k < rem ? ws_ds[(((bb + k) * 2 + slot) * SEGS + sg) * (int64_t)N + p] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (k < rem) a = cadd(a, v[k]);
      }
      ds[o0 + p] = a;
    }
  }
}

// a + part[s0][i] + part[s0 + 1][i] + ... + part[s1 - 1][i], added in that
// order; the loads go out eight at a time so that their latencies overlap
// (one at a time, the sum took ~9 us for 16 or 32 slots).
__device__ __forceinline__ float2 sum_slots(const float2* __restrict__ part, int64_t s0, int64_t s1, int64_t KM,
                                            int64_t i) {
  float2 a = make_float2(0.f, 0.f);
  int64_t sl = s0;
  for (; sl + 8 <= s1; sl += 8) {
    float2 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = part[(sl + k) * KM + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) a = cadd(a, v[k]);
  }
  for (; sl < s1; ++sl) a = cadd(a, part[sl * KM + i]);
  return a;
}

// First level of the dh reduction: sums[c][i] = sum of part[slot][i] over
// the slots of chunk c = blockIdx.y, in slot order.
__global__ void ols_dh_chunk_kernel(const float2* __restrict__ part, int64_t nslots, int64_t KM,
                                    float2* __restrict__ sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KM) return;
  const int64_t c = blockIdx.y;
  const int64_t s0 = c * DH_CHUNK, s1 = s0 + DH_CHUNK < nslots ? s0 + DH_CHUNK : nslots;
  sums[c * KM + i] = sum_slots(part, s0, s1, KM, i);
}

// dh[i] = sum over slots of part[slot][i], in slot order (second level: the
// chunk sums in chunk order).
__global__ void ols_dh_reduce_kernel(const float2* __restrict__ part, int64_t nslots, int64_t KM,
                                     float2* __restrict__ dh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KM) return;
  dh[i] = sum_slots(part, 0, nslots, KM, i);
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

// A single-signal call re-aligns its output rows (row_shift_geometry) only
// from this many outputs (K * N_s) on: smaller calls are bound by launch and
// memory latency, where aligned stores measured no gain, while re-aligned
// rows run with a hop up to two lines shorter (3-8 % saved at 2^22-2^23
// outputs, 14 % at 2^28).
constexpr int64_t SHIFT_MIN_OUTPUTS = (int64_t)1 << 22;
// Device memory a plan may spend on the spectra for every row delay (16
// copies of its spectra for complex outputs, 32 for float32 ones); larger
// plans do not re-align their rows.
constexpr int64_t SHIFT_SPECTRA_MAX_BYTES = (int64_t)256 << 20;

// Scratch of the adjoint: partial ds windows of tiles split between
// workgroups, per-workgroup dh lag partials and their chunk sums.  Sized for a
// grid of persistent workgroups (bwd_ws_bytes); every part is written before
// it is read within one call, so nothing needs clearing beforehand.
struct BwdWorkspace {
  int grid = 0;
  float2* ws_ds = nullptr;    // [grid][2][SEGS][N]
  float2* part_dh = nullptr;  // [grid][SEGS][K][M]
  float2* sum_dh = nullptr;   // [dh_chunks(grid * SEGS)][K][M]
};

// Bytes of each part of a BwdWorkspace, each rounded up to 256 bytes.
struct BwdWorkspaceSizes {
  size_t ds = 0, part = 0, sums = 0;
  size_t total() const { return ds + part + sums; }
};

inline size_t round256(size_t v) { return (v + 255) / 256 * 256; }

inline BwdWorkspaceSizes bwd_ws_bytes(int grid, int segs, int N, int K, int M) {
  BwdWorkspaceSizes z;
  z.ds = round256((size_t)grid * 2 * segs * N * sizeof(float2));
  z.part = round256((size_t)grid * segs * K * M * sizeof(float2));
  z.sums = round256((size_t)dh_chunks((int64_t)grid * segs) * K * M * sizeof(float2));
  return z;
}

// Carves a workspace for `grid` workgroups out of one buffer of at least
// bwd_ws_bytes(grid, ...).total() bytes.
inline BwdWorkspace bwd_ws_carve(void* base, int grid, int segs, int N, int K, int M) {
  const BwdWorkspaceSizes z = bwd_ws_bytes(grid, segs, N, K, M);
  char* b = (char*)base;
  BwdWorkspace w;
  w.grid = grid;
  w.ws_ds = (float2*)b;
  w.part_dh = (float2*)(b + z.ds);
  w.sum_dh = (float2*)(b + z.ds + z.part);
  return w;
}

struct ols_plan_s {
  int K = 0, M = 0, N = 0, D = 0, H = 0;
  int device = 0;
  int cus = 0;
  int grid = 0;   // persistent workgroups of the forward kernel
  int block = 0;  // threads per workgroup
  int segs = 0;   // segments per tile
  int nf = 1;     // filters per work unit of the forward kernel
  int flags = 0;  // OLS_POST_* and OLS_REAL
  bool stencil_on = false;  // non-local stage (ols_plan_set_stencil)
  int stencil_R = 0;        // its reach ahead (taps after the sample)
  Stencil stencil{};
  void* bwd_mem = nullptr;  // the adjoint's scratch, allocated by ols_plan_reserve_backward
  BwdWorkspace bwd{};       // carved from bwd_mem for the adjoint's full grid
  float2* spectra = nullptr;
  float2* spectra_delays = nullptr;  // [delay_ls][K][N]: the spectra delayed by 0 .. delay_ls-1 samples
  int delay_ls = 0;                   // outputs per 128-byte line (0: no delayed spectra, rows not re-aligned)
  float2* twiddles = nullptr;
};

struct ols_batch_s {
  int n = 0;
  int grid = 0;         // persistent workgroups of the batched kernel
  void* ws = nullptr;   // the batch's own workspace (same layout as ols_batched's)
  ols_batch_item_t* dev_items = nullptr;
  BatchLayout L{};
  std::vector<BatchItem> items_sorted;  // kernel order (copied back after the setup)
  std::vector<int32_t> order;           // caller's index of each kernel-order item
  std::vector<int32_t> pos_of;          // kernel position of each caller item
  int64_t total_units = 0;
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


template <int N>
struct Kern {
  using GE = Geo<N>;
  static constexpr bool HAS_NF2 = N <= 4096;

  static hipError_t spectra(const void* h, int K, int M, float2* F, const float2* tw, hipStream_t st, int diff,
                            int real) {
    const int blocks = (K + GE::SEGS - 1) / GE::SEGS;
    hipLaunchKernelGGL(ols_filter_spectra_kernel<N>, dim3(blocks), dim3(GE::WG), 0, st, h, K, M, F, tw, diff, real,
                       SpectraShift{});
    return hipGetLastError();
  }
  static hipError_t delays(const float2* F, int K, int LS, float2* out, hipStream_t st) {
    const int64_t total = (int64_t)K * N * LS;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(ols_spectra_delays_kernel<N>, dim3((unsigned)blocks), dim3(threads), 0, st, F, K, LS, out);
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
  using ForwardFn = void (*)(const void*, int64_t, const float2*, void*, int, int, int, int64_t, const float2*, int);
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
  // The same for the kernel with the non-local stencil stage.
  using StencilFn = void (*)(const void*, int64_t, const float2*, void*, int, int, int, int64_t, const float2*,
                             const Stencil);
  template <int NF>
  static StencilFn stencil_fn_nf(bool power, bool real) {
    if (real) {
      constexpr int NFR = N <= BATCH_NF2_MAX_N ? NF : 1;
      return power ? ols_forward_stencil_kernel<N, NFR, true, true> : ols_forward_stencil_kernel<N, NFR, false, true>;
    }
    return power ? ols_forward_stencil_kernel<N, NF, true, false> : ols_forward_stencil_kernel<N, NF, false, false>;
  }
  static StencilFn stencil_fn(int nf, int flags) {
    const bool power = (flags & OLS_POST_POWER) != 0, real = (flags & OLS_REAL) != 0;
    if constexpr (HAS_NF2) {
      if (nf == 2) return stencil_fn_nf<2>(power, real);
    }
    return stencil_fn_nf<1>(power, real);
  }
  static hipError_t forward(const ols_plan_s* p, const void* s, int64_t Ns, void* y, hipStream_t st) {
    // output rows off the 128-byte grid read the plan's spectra for each
    // row's delay (the call only reads the plan)
    const bool float_out = (p->flags & (OLS_REAL | OLS_POST_POWER)) != 0;
    const RowShift rs = row_shift_geometry(
        y, Ns, N, p->D, p->H, float_out ? 4 : 8,
        p->spectra_delays && !p->stencil_on && (int64_t)p->K * Ns >= SHIFT_MIN_OUTPUTS);
    const float2* F = rs.mask ? p->spectra_delays : p->spectra;
    const int H = rs.H;
    const int64_t nseg = (Ns + H - 1) / H;
    const int64_t ntrans = (p->flags & OLS_REAL) ? (nseg + 1) / 2 : nseg;  // R2R: segment pairs
    const int64_t ntiles = (ntrans + GE::SEGS - 1) / GE::SEGS;
    const int64_t units = ntiles * ((p->K + p->nf - 1) / p->nf);
    const int64_t grid = units < p->grid ? units : p->grid;
    if (p->stencil_on) {
      // J <= 2 phases go out as one element per sample when y is aligned to it
      Stencil sten = p->stencil;
      const uintptr_t el = (uintptr_t)sten.J * (float_out ? 4 : 8);
      sten.packed = sten.J <= 2 && (uintptr_t)y % el == 0;
      hipLaunchKernelGGL(stencil_fn(p->nf, p->flags), dim3((unsigned)grid), dim3(GE::WG), 0, st, s, Ns, p->spectra, y,
                         p->K, p->D, p->H, ntiles, p->twiddles, sten);
    } else
      hipLaunchKernelGGL(forward_fn(p->nf, p->flags), dim3((unsigned)grid), dim3(GE::WG), 0, st, s, Ns, F, y, p->K,
                         p->D, H, ntiles, p->twiddles, rs.mask);
    return hipGetLastError();
  }
  static hipError_t occupancy(int nf, int flags, bool stage, int* blocks_per_cu) {
    if (stage) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, stencil_fn(nf, flags), GE::WG, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, forward_fn(nf, flags), GE::WG, 0);
  }
  // The adjoint: paired segments up to N = 2048 (ols_backward_pair_kernel),
  // one segment per group above.
  // At N = 4096 a pair needs a 512-thread workgroup and 135 KB of LDS, one
  // workgroup per CU: measured 7 % slower than the one-segment kernel there,
  // 2-5 % faster at N = 512 .. 2048 (16 filters, 2^22 samples).
  static constexpr bool PAIRED = N <= 2048;
  static constexpr int BWD_SEGS = PAIRED ? BwdGeo<N>::SEGS : GE::SEGS;
  static constexpr int BWD_WG = PAIRED ? BwdGeo<N>::WG : GE::WG;
  using BwdFn = void (*)(const float2*, const float2*, int64_t, const float2*, int, int, int, int64_t, const float2*,
                         float2*, float2*, float2*, int, int);
  static BwdFn bwd_fn() {
    if constexpr (PAIRED) return ols_backward_pair_kernel<N>;
    else return ols_backward_kernel<N>;
  }
  static hipError_t bwd_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, bwd_fn(), BWD_WG, 0);
  }
  static hipError_t backward(const ols_plan_s* p, const BwdWorkspace& w, const float2* s, const float2* gy,
                             int64_t Ns, float2* ds, float2* dh, hipStream_t st) {
    const int64_t nseg = (Ns + p->H - 1) / p->H;
    const int64_t ntiles = (nseg + BWD_SEGS - 1) / BWD_SEGS;
    const int upt = PAIRED ? (p->K + 1) / 2 : p->K;  // units per tile
    const int64_t units = ntiles * upt;
    const int64_t grid = units < w.grid ? units : w.grid;
    hipLaunchKernelGGL(bwd_fn(), dim3((unsigned)grid), dim3(BWD_WG), 0, st, s, gy, Ns, p->spectra, p->K, p->M, p->H,
                       ntiles, p->twiddles, ds, w.ws_ds, w.part_dh, ds ? 1 : 0, dh ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ds && grid > 1) {
      // one workgroup per (tile boundary, eighth of the window): H <= 8192 outputs, at most 4 per lane
      hipLaunchKernelGGL((ols_ds_fixup_kernel<N, BWD_SEGS>), dim3((unsigned)(grid - 1), 8), dim3(256), 0, st, w.ws_ds,
                         ds, Ns, upt, p->H, ntiles, grid);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (dh) {
      const int64_t KM = (int64_t)p->K * p->M;
      const int64_t nslots = grid * BWD_SEGS, nch = dh_chunks(nslots);
      const unsigned bx = (unsigned)((KM + 255) / 256);
      hipLaunchKernelGGL(ols_dh_chunk_kernel, dim3(bx, (unsigned)nch), dim3(256), 0, st, w.part_dh, nslots, KM,
                         w.sum_dh);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(ols_dh_reduce_kernel, dim3(bx), dim3(256), 0, st, w.sum_dh, nch, KM, dh);
      e = hipGetLastError();
    }
    return e;
  }
  static std::vector<float2> twiddles() { return build_twiddles<N>(); }
  static int bwd_segs() { return BWD_SEGS; }
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
struct RunDelays {
  static hipError_t run(const float2* F, int K, int LS, float2* out, hipStream_t st) {
    return Kern<N>::delays(F, K, LS, out, st);
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
  static hipError_t run(int nf, int flags, bool stage, int* b) { return Kern<N>::occupancy(nf, flags, stage, b); }
};
template <int N>
struct RunBwdOccupancy {
  static hipError_t run(int* b) { return Kern<N>::bwd_occupancy(b); }
};
template <int N>
struct RunBackward {
  static hipError_t run(const ols_plan_s* p, const BwdWorkspace& w, const float2* s, const float2* gy, int64_t Ns,
                        float2* ds, float2* dh, hipStream_t st) {
    return Kern<N>::backward(p, w, s, gy, Ns, ds, dh, st);
  }
};
template <int N>
struct RunTwiddles {
  static std::vector<float2> run() { return Kern<N>::twiddles(); }
};
template <int N>
struct RunBwdSegs {
  static int run() { return Kern<N>::bwd_segs(); }
};
template <int N>
struct RunShape {
  static int run(int which) { return which == 0 ? Kern<N>::block() : Kern<N>::segs(); }
};

void destroy_batch(ols_batch_s* b) {
  if (!b) return;
  if (b->ws) (void)hipFree(b->ws);
  if (b->dev_items) (void)hipFree(b->dev_items);
  delete b;
}

// Layout of a batch workspace for n items: header, the five twiddle tables,
// the kernel-order item table, spectrum-task offsets, the caller order, then
// the filter spectra; every part starts on a 256-byte boundary.
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
constexpr int BATCH_TW_ELEMS[BATCH_LENGTHS] = {Geo<256>::TW_TOTAL, Geo<512>::TW_TOTAL, Geo<1024>::TW_TOTAL,
                                               Geo<2048>::TW_TOTAL, Geo<4096>::TW_TOTAL};
struct BatchOffsets {
  size_t hdr, tw[BATCH_LENGTHS], items, task, order, spec;
};
BatchOffsets batch_offsets(int n) {
  BatchOffsets o{};
  size_t off = 0;
  o.hdr = off;
  off = align256(off + sizeof(BatchHeader));
  for (int k = 0; k < BATCH_LENGTHS; ++k) {
    o.tw[k] = off;
    off = align256(off + (size_t)BATCH_TW_ELEMS[k] * sizeof(float2));
  }
  o.items = off;
  off = align256(off + (size_t)n * sizeof(BatchItem));
  o.task = off;
  off = align256(off + (size_t)(n + 1) * sizeof(int64_t));
  o.order = off;
  off = align256(off + (size_t)n * sizeof(int32_t));
  o.spec = off;
  return o;
}
BatchLayout batch_layout(void* ws, size_t bytes, int n) {
  const BatchOffsets o = batch_offsets(n);
  char* base = (char*)ws;
  BatchLayout L{};
  L.hdr = (BatchHeader*)(base + o.hdr);
  for (int k = 0; k < BATCH_LENGTHS; ++k) L.tw[k] = (float2*)(base + o.tw[k]);
  L.items = (BatchItem*)(base + o.items);
  L.task_begin = (int64_t*)(base + o.task);
  L.order = (int32_t*)(base + o.order);
  L.spectra = (float2*)(base + o.spec);
  L.spec_capacity = bytes > o.spec ? (int64_t)((bytes - o.spec) / sizeof(float2)) : 0;
  L.n = n;
  return L;
}

// Persistent grids of the batch kernels on the current device.
hipError_t batch_grids(int* batched, int* spectra) {
  int dev = 0, cus = 0, a = 0, b = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, ols_batched_kernel, 256, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, ols_batch_spectra_kernel, 256, 0);
  *batched = (a < 1 ? 1 : a) * cus;
  *spectra = (b < 1 ? 1 : b) * cus;
  return e;
}

// The three launches of a batched call: setup, filter spectra, the persistent
// forward.  Allocate nothing; capturable.
hipError_t launch_batch(const ols_batch_item_t* dev_items, const BatchLayout& L, bool forward, hipStream_t st) {
  int grid = 0, sgrid = 0;
  hipError_t e = batch_grids(&grid, &sgrid);
  if (e != hipSuccess) return e;
  if (dev_items) {
    hipLaunchKernelGGL(ols_batch_setup_kernel, dim3(1), dim3(SETUP_THREADS), 0, st, dev_items, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(ols_batch_spectra_kernel, dim3(sgrid), dim3(256), 0, st, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (forward) {
    hipLaunchKernelGGL(ols_batched_kernel, dim3(grid), dim3(256), 0, st, L);
    e = hipGetLastError();
  }
  return e;
}

bool ranges_overlap(const void* a, size_t an, const void* b, size_t bn) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bn && b0 < a0 + an;
}

void destroy_plan(ols_plan_s* p) {
  if (!p) return;
  if (p->bwd_mem) (void)hipFree(p->bwd_mem);
  if (p->spectra) (void)hipFree(p->spectra);
  if (p->spectra_delays) (void)hipFree(p->spectra_delays);
  if (p->twiddles) (void)hipFree(p->twiddles);
  delete p;
}

}  // namespace

namespace {

// Persistent workgroups of the adjoint kernel: as many as fit on the device.
ols_status_t bwd_full_grid(const ols_plan_s* p, int* grid) {
  int per_cu = 0;
  hipError_t e = dispatch<RunBwdOccupancy>(p->N, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "occupancy query");
  if (per_cu < 1) per_cu = 1;
  *grid = per_cu * p->cus;
  return OLS_SUCCESS;
}

// Host-side checks shared by the adjoint entry points.  *done is set when the
// call is complete without the adjoint kernels (nothing asked, or N_s = 0).
ols_status_t bwd_validate(ols_plan_t p, const void* s, int64_t Ns, const void* gy, void* ds, void* dh, hipStream_t st,
                          bool* done) {
  *done = false;
  if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
  if (p->flags != OLS_POST_NONE || p->stencil_on)
    return fail(OLS_ERROR_UNSUPPORTED, "backward of a post-processed or R2R plan");
  if (Ns < 0) return fail(OLS_ERROR_INVALID_VALUE, "N_s must be >= 0");
  if (!ds && !dh) {
    *done = true;
    return OLS_SUCCESS;
  }
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
  if (Ns == 0) {  // empty signal: dh is zero, ds is empty
    if (dh) {
      hipLaunchKernelGGL(ols_zero_kernel, dim3(64), dim3(256), 0, st, (float2*)dh, (int64_t)p->K * p->M);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "zero launch");
    }
    *done = true;
  }
  return OLS_SUCCESS;
}

}  // namespace

// ---------------------------------------------------------------------------
// ols_backward_static: the adjoint with its scratch in a file-scope device
// array instead of plan memory, for callers that cannot allocate.  In host
// code `scratch` names a host-side shadow, not device memory: kernels only
// ever receive the device address obtained with hipGetSymbolAddress, looked
// up once per device (each device holds its own copy of the array).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[OLS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

ols_status_t static_scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(OLS_ERROR_INVALID_VALUE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return OLS_SUCCESS;
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
      N = cost_model_fft_length(K, Meff, OLS_MAX_FFT_LENGTH);
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
    e = dispatch<RunOccupancy>(N, p->nf, flags, false, &per_cu);
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
    // the spectra for every row delay, when they fit the budget
    const int ls = (flags & (OLS_REAL | OLS_POST_POWER)) ? 32 : 16;
    if ((int64_t)K * N * ls * (int64_t)sizeof(float2) <= SHIFT_SPECTRA_MAX_BYTES) {
      e = hipMalloc(&p->spectra_delays, (size_t)K * N * ls * sizeof(float2));
      if (e != hipSuccess) { destroy_plan(p); (void)hipGetLastError(); return fail(OLS_ERROR_OUT_OF_MEMORY, "spectra allocation"); }
      p->delay_ls = ls;
    }
    hipStream_t st = (hipStream_t)stream;
    e = hipMemcpyAsync(p->twiddles, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "twiddle upload"); }
    e = dispatch<RunSpectra>(N, h, K, M, p->spectra, (const float2*)p->twiddles, st,
                             (flags & OLS_POST_DERIVATIVE) ? 1 : 0, (flags & OLS_REAL) ? 1 : 0);
    if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "filter spectra launch"); }
    if (p->spectra_delays) {
      e = dispatch<RunDelays>(N, (const float2*)p->spectra, K, p->delay_ls, p->spectra_delays, st);
      if (e != hipSuccess) { destroy_plan(p); return hip_fail(e, "delayed spectra launch"); }
    }
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
    if (p->spectra_delays) {
      e = dispatch<RunDelays>(p->N, (const float2*)p->spectra, p->K, p->delay_ls, p->spectra_delays,
                              (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "delayed spectra launch");
    }
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_update_filters");
  }
}

ols_status_t ols_plan_set_hop(ols_plan_t p, int32_t H) {
  if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
  const int Meff = (p->flags & OLS_POST_DERIVATIVE) ? p->M + 1 : p->M;
  // a stencil needs sL unaliased outputs before each kept one and sR after it
  const int sL = p->stencil_on ? p->stencil.L : 0, sR = p->stencil_on ? p->stencil_R : 0;
  const int Hmax = p->N - (Meff - 1 + sL) - sR;
  if (H == 0) {
    p->D = stencil_delay(p->N, Meff, sL, sR);
    p->H = stencil_hop(p->N, p->D, sR);
    return OLS_SUCCESS;
  }
  if (H < 1 || H > Hmax) return fail(OLS_ERROR_INVALID_VALUE, "hop must satisfy 1 <= H <= N-M+1 (less the stencil's reach)");
  int D = stencil_delay(p->N, Meff, sL, sR);
  if (D + H + sR > p->N) D = p->N - H - sR;
  p->D = D;
  p->H = H;
  return OLS_SUCCESS;
}

ols_status_t ols_plan_set_stencil(ols_plan_t p, int32_t J, int32_t L, int32_t R, const float* w) {
  try {
    if (!p) return fail(OLS_ERROR_INVALID_VALUE, "plan is NULL");
    const int Meff = (p->flags & OLS_POST_DERIVATIVE) ? p->M + 1 : p->M;
    Stencil st{};
    if (J != 0) {
      if (J < 1 || J > STENCIL_MAX_PHASES) return fail(OLS_ERROR_INVALID_VALUE, "phases must be in [1, 4] (0 removes the stencil)");
      if (L < 0 || R < 0 || L + 1 + R > STENCIL_MAX_TAPS)
        return fail(OLS_ERROR_INVALID_VALUE, "the stencil needs left, right >= 0 and left + 1 + right <= 8 taps");
      if (!w) return fail(OLS_ERROR_INVALID_VALUE, "weights are NULL");
      if (Meff - 1 + L + R > p->N - 1)
        return fail(OLS_ERROR_INVALID_VALUE, "M - 1 + left + right must be < N (no kept output would remain)");
      st.J = J;
      st.L = L;
      st.T = L + 1 + R;
      for (int j = 0; j < J; ++j)
        for (int d = 0; d < st.T; ++d) st.w[j][d] = w[j * st.T + d];
    }
    // one filter per unit with the stage: with two, the stage kernels at
    // N = 2048 spill registers and measured 5-15 % slower
    const int nf = J != 0 ? 1 : ((p->flags & OLS_REAL) ? choose_nf_real(p->N, p->K) : choose_nf(p->N, p->K));
    int per_cu = 0;
    hipError_t e = dispatch<RunOccupancy>(p->N, nf, p->flags, J != 0, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) per_cu = 1;
    p->nf = nf;
    p->stencil_on = J != 0;
    p->stencil = st;
    p->stencil_R = J != 0 ? R : 0;
    p->D = stencil_delay(p->N, Meff, p->stencil_on ? L : 0, p->stencil_R);
    p->H = stencil_hop(p->N, p->D, p->stencil_R);
    p->grid = per_cu * p->cus;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_set_stencil");
  }
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
    hipError_t e = dispatch<RunOccupancy>(p->N, nf, p->flags, p->stencil_on, &per_cu);
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
    hipError_t e = dispatch<RunOccupancy>(p->N, p->nf, p->flags, p->stencil_on, &per_cu);
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
    const int J = p->stencil_on ? p->stencil.J : 1;  // outputs per sample
    if (Ns > ((int64_t)1 << 56) / 8 / p->K / J) return fail(OLS_ERROR_INVALID_VALUE, "K*J*N_s*8 overflows");
    if (ranges_overlap(s, (size_t)Ns * s_el, y, (size_t)Ns * (size_t)p->K * (size_t)J * y_el))
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
    if (p->bwd_mem) return OLS_SUCCESS;
    int grid = 0;
    const ols_status_t r = bwd_full_grid(p, &grid);
    if (r != OLS_SUCCESS) return r;
    const size_t bytes = bwd_ws_bytes(grid, dispatch<RunBwdSegs>(p->N), p->N, p->K, p->M).total();
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(OLS_ERROR_OUT_OF_MEMORY, "backward workspace");
    }
    p->bwd_mem = mem;
    p->bwd = bwd_ws_carve(mem, grid, dispatch<RunBwdSegs>(p->N), p->N, p->K, p->M);
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_plan_reserve_backward");
  }
}

ols_status_t ols_backward(ols_plan_t p, const void* s, int64_t Ns, const void* gy, void* ds, void* dh,
                          ols_stream_t stream) {
  try {
    hipStream_t st = (hipStream_t)stream;
    bool done = false;
    ols_status_t r = bwd_validate(p, s, Ns, gy, ds, dh, st, &done);
    if (r != OLS_SUCCESS || done) return r;
    if (!p->bwd_mem) {
      r = ols_plan_reserve_backward(p);
      if (r != OLS_SUCCESS) return r;
    }
    hipError_t e = dispatch<RunBackward>(p->N, (const ols_plan_s*)p, (const BwdWorkspace&)p->bwd, (const float2*)s,
                                         (const float2*)gy, Ns, (float2*)ds, (float2*)dh, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_backward");
  }
}


ols_status_t ols_backward_static(ols_plan_t p, const void* s, int64_t Ns, const void* gy, void* ds, void* dh,
                                 ols_stream_t stream) {
  try {
    hipStream_t st = (hipStream_t)stream;
    bool done = false;
    ols_status_t r = bwd_validate(p, s, Ns, gy, ds, dh, st, &done);
    if (r != OLS_SUCCESS || done) return r;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != p->device) return fail(OLS_ERROR_INVALID_VALUE, "the plan belongs to another device");
    int grid = 0;
    r = bwd_full_grid(p, &grid);
    if (r != OLS_SUCCESS) return r;
    // as many workgroups as the scratch holds, at most the full grid
    const size_t one = bwd_ws_bytes(1, dispatch<RunBwdSegs>(p->N), p->N, p->K, p->M).total();
    if (one > OLS_STATIC_SCRATCH_BYTES)
      return fail(OLS_ERROR_INVALID_VALUE,
                  "the adjoint of this plan needs " + std::to_string(one) + " bytes of scratch per workgroup, more than "
                  "the " + std::to_string((size_t)OLS_STATIC_SCRATCH_BYTES) + " bytes of ols_backward_static");
    while (grid > 1 && bwd_ws_bytes(grid, dispatch<RunBwdSegs>(p->N), p->N, p->K, p->M).total() > OLS_STATIC_SCRATCH_BYTES) --grid;
    void* base = nullptr;
    r = static_scratch_address(&base);
    if (r != OLS_SUCCESS) return r;
    const BwdWorkspace w = bwd_ws_carve(base, grid, dispatch<RunBwdSegs>(p->N), p->N, p->K, p->M);
    e = dispatch<RunBackward>(p->N, (const ols_plan_s*)p, w, (const float2*)s, (const float2*)gy, Ns, (float2*)ds,
                              (float2*)dh, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_backward_static");
  }
}

ols_status_t ols_plan_destroy(ols_plan_t p) {
  destroy_plan(p);
  return OLS_SUCCESS;
}

// Host-side check of batch item i (the same checks the device-side setup
// repeats), with a message naming the item.
static ols_status_t batch_item_host_check(const ols_batch_item_t& it, int i, int* N_out) {
  const int st = batch_item_check(it.s, it.N_s, it.h, it.K, it.M, it.N, it.y, N_out);
  if (st == 0) return OLS_SUCCESS;
  const std::string where = "item " + std::to_string(i) + ": ";
  if (st == OLS_ERROR_UNSUPPORTED)
    return fail(OLS_ERROR_UNSUPPORTED, where + "batched N must be a power of two in [256, 4096] (or 0 with M <= 4096)");
  return fail(OLS_ERROR_INVALID_VALUE, where + "K, M >= 1, N_s >= 0, non-NULL 8-byte aligned pointers, M <= N, "
                                               "K*N_s*8 in range and y not overlapping s are required");
}

// Workspace bytes of a batched call over these items; host checks only.
static ols_status_t batch_bytes(const ols_batch_item_t* items, int32_t n, size_t* bytes) {
  if (!items || n < 1) return fail(OLS_ERROR_INVALID_VALUE, "items is NULL or n < 1");
  size_t spec = 0;
  for (int i = 0; i < n; ++i) {
    int N = 0;
    const ols_status_t r = batch_item_host_check(items[i], i, &N);
    if (r != OLS_SUCCESS) return r;
    spec += (size_t)items[i].K * N;
  }
  *bytes = batch_offsets(n).spec + spec * sizeof(float2);
  return OLS_SUCCESS;
}

ols_status_t ols_batched_workspace_size(const ols_batch_item_t* items, int32_t n, size_t* bytes) {
  try {
    if (!bytes) return fail(OLS_ERROR_INVALID_VALUE, "bytes is NULL");
    *bytes = 0;
    return batch_bytes(items, n, bytes);
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batched_workspace_size");
  }
}

ols_status_t ols_batched(const ols_batch_item_t* dev_items, int32_t n, void* workspace, size_t ws_bytes,
                         ols_stream_t stream) {
  try {
    if (!dev_items || n < 1) return fail(OLS_ERROR_INVALID_VALUE, "dev_items is NULL or n < 1");
    if ((uintptr_t)dev_items % 8) return fail(OLS_ERROR_INVALID_VALUE, "dev_items must be 8-byte aligned");
    if (!workspace || (uintptr_t)workspace % 256) return fail(OLS_ERROR_INVALID_VALUE, "workspace is NULL or not 256-byte aligned");
    // every item needs at least K * N >= 256 spectrum elements
    if (ws_bytes < batch_offsets(n).spec + (size_t)n * OLS_MIN_FFT_LENGTH * sizeof(float2))
      return fail(OLS_ERROR_INVALID_VALUE, "workspace too small for n items");
    const BatchLayout L = batch_layout(workspace, ws_bytes, n);
    const hipError_t e = launch_batch(dev_items, L, true, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batched");
  }
}

ols_status_t ols_batched_status(const void* workspace, ols_stream_t stream, int32_t* status, int32_t* bad_item) {
  try {
    if (!workspace || (uintptr_t)workspace % 256) return fail(OLS_ERROR_INVALID_VALUE, "workspace is NULL or not 256-byte aligned");
    BatchHeader hd{};
    hipError_t e = hipMemcpyAsync(&hd, workspace, sizeof(hd), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "status read-back");
    if (status) *status = hd.status;
    if (bad_item) *bad_item = hd.bad_item;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batched_status");
  }
}

ols_status_t ols_batch_plan(ols_batch_t* out, const ols_batch_item_t* items, int32_t n, ols_stream_t stream) {
  try {
    if (!out) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL");
    *out = nullptr;
    size_t bytes = 0;
    const ols_status_t r = batch_bytes(items, n, &bytes);
    if (r != OLS_SUCCESS) return r;
    ols_batch_s* b = new (std::nothrow) ols_batch_s();
    if (!b) return fail(OLS_ERROR_OUT_OF_MEMORY, "host allocation failed");
    b->n = n;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    int sgrid = 0;
    if ((e = batch_grids(&b->grid, &sgrid)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "occupancy query"); }
    if (hipMalloc(&b->ws, bytes) != hipSuccess || hipMalloc(&b->dev_items, (size_t)n * sizeof(ols_batch_item_t)) != hipSuccess) {
      destroy_batch(b);
      (void)hipGetLastError();
      return fail(OLS_ERROR_OUT_OF_MEMORY, "batch allocation");
    }
    b->L = batch_layout(b->ws, bytes, n);
    if ((e = hipMemcpyAsync(b->dev_items, items, (size_t)n * sizeof(ols_batch_item_t), hipMemcpyHostToDevice, st)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "item upload"); }
    // the same setup and spectra kernels as ols_batched, once
    if ((e = launch_batch(b->dev_items, b->L, false, st)) != hipSuccess) { destroy_batch(b); return hip_fail(e, "batch setup launch"); }
    BatchHeader hd{};
    b->items_sorted.resize(n);
    b->order.resize(n);
    if ((e = hipMemcpyAsync(&hd, b->L.hdr, sizeof(hd), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(b->items_sorted.data(), b->L.items, (size_t)n * sizeof(BatchItem), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(b->order.data(), b->L.order, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      destroy_batch(b);
      return hip_fail(e, "batch setup read-back");
    }
    if (hd.status != OLS_SUCCESS) {
      destroy_batch(b);
      return fail(OLS_ERROR_INTERNAL, "device-side batch setup disagreed with the host checks");
    }
    b->total_tiles = hd.total_tiles;
    b->pos_of.assign(n, -1);
    for (int k = 0; k < n; ++k) {
      b->pos_of[b->order[k]] = k;
      b->total_units += b->items_sorted[k].units;
    }
    *out = b;
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batch_plan");
  }
}

ols_status_t ols_batch_run(ols_batch_t b, ols_stream_t stream) {
  try {
    if (!b) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL");
    const hipError_t e = launch_batch(nullptr, b->L, true, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return OLS_SUCCESS;
  } catch (...) {
    return fail(OLS_ERROR_INTERNAL, "exception in ols_batch_run");
  }
}

ols_status_t ols_batch_get_info(ols_batch_t b, int64_t* total_units, int32_t* grid, int32_t* n) {
  if (!b) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL");
  if (total_units) *total_units = b->total_units;
  if (grid) *grid = b->grid;
  if (n) *n = b->n;
  return OLS_SUCCESS;
}

ols_status_t ols_batch_get_item(ols_batch_t b, int32_t i, int32_t* N, int32_t* H, int32_t* D) {
  if (!b || i < 0 || i >= b->n) return fail(OLS_ERROR_INVALID_VALUE, "batch is NULL or item out of range");
  const BatchItem& it = b->items_sorted[b->pos_of[i]];
  if (N) *N = it.N;
  if (H) *H = it.H;
  if (D) *D = it.D;
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
