// Host emulation of the fused overlap-and-save kernels.
//
// Runs the very same per-lane code as the device kernels (ols_fft.hpp,
// ols_ops.hpp) on the CPU, lane by lane, with every workgroup barrier replaced
// by "all lanes finish this phase before any lane starts the next".  Used by
// CPU tests to check, before anything runs on a GPU:
//   * the transform and the overlap-and-save dataflow against the oracle;
//   * that every LDS exchange is a bijection inside the LDS allocation and
//     free of bank conflicts (for 32 and for 64 four-byte banks);
//   * that no global access leaves its buffer (NaN guard bands) and every
//     output is written (NaN pre-fill).
// Built as a host library (libols_emu.so); it makes no HIP runtime calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <vector>

#include "ols_fft.hpp"
#include "ols_ops.hpp"
#include "ols_twiddle.hpp"

namespace ols {
namespace emu {

using Regs = float2[16];

template <int N>
struct Group {
  using GE = Geo<N>;
  std::vector<float2> lds;  // with guard bands
  float2* L;
  static constexpr int GUARD = 4096;
  Group() : lds(GE::LDS + 2 * GUARD) { L = lds.data() + GUARD; }
  void poison() {
    const float nan = std::numeric_limits<float>::quiet_NaN();
    for (auto& v : lds) v = make_float2(nan, nan);
  }
  bool guards_ok() const {
    for (int i = 0; i < GUARD; ++i) {
      if (!std::isnan(lds[i].x) || !std::isnan(lds[lds.size() - 1 - i].x)) return false;
    }
    return true;
  }
};

template <int N, int E, int KW, int KR>
void exchange_phase(std::vector<std::array<float2, 16>>& xs, Group<N>& G) {
  using GE = Geo<N>;
  G.poison();
  for (int t = 0; t < GE::WG; ++t)
    lds_store<N, E, KW>(G.L, *reinterpret_cast<float2(*)[16]>(xs[t].data()), t / GE::G, t % GE::G);
  for (int t = 0; t < GE::WG; ++t)
    lds_load<N, E, KR>(G.L, *reinterpret_cast<float2(*)[16]>(xs[t].data()), t / GE::G, t % GE::G);
}

template <int N, int K>
void fwd_from(std::vector<std::array<float2, 16>>& xs, Group<N>& G, const std::vector<std::array<float2, Geo<N>::TWR>>& tw) {
  using GE = Geo<N>;
  const int T = GE::WG;
  for (int t = 0; t < T; ++t) {
    float2(&x)[16] = *reinterpret_cast<float2(*)[16]>(xs[t].data());
    run_pass<N, K, false>(x, tw[t].data() + GE::lane_tw_offset(K));
  }
  if constexpr (K + 1 < GE::P) {
    G.poison();
    for (int t = 0; t < T; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      lds_store<N, K, K>(G.L, *reinterpret_cast<float2(*)[16]>(xs[t].data()), grp, g);
    }
    for (int t = 0; t < T; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      lds_load<N, K, K + 1>(G.L, *reinterpret_cast<float2(*)[16]>(xs[t].data()), grp, g);
    }
    fwd_from<N, K + 1>(xs, G, tw);
  }
}

template <int N, int K>
void inv_from(std::vector<std::array<float2, 16>>& xs, Group<N>& G, const std::vector<std::array<float2, Geo<N>::TWR>>& tw) {
  using GE = Geo<N>;
  const int T = GE::WG;
  for (int t = 0; t < T; ++t) {
    float2(&x)[16] = *reinterpret_cast<float2(*)[16]>(xs[t].data());
    inverse_pass<N, K>(x, tw[t].data() + GE::lane_tw_offset(K));
  }
  if constexpr (K > 0) {
    G.poison();
    for (int t = 0; t < T; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      lds_store<N, K - 1, K>(G.L, *reinterpret_cast<float2(*)[16]>(xs[t].data()), grp, g);
    }
    for (int t = 0; t < T; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      lds_load<N, K - 1, K - 1>(G.L, *reinterpret_cast<float2(*)[16]>(xs[t].data()), grp, g);
    }
    inv_from<N, K - 1>(xs, G, tw);
  }
}

template <int N>
std::vector<std::array<float2, Geo<N>::TWR>> lane_twiddles(const std::vector<float2>& table) {
  using GE = Geo<N>;
  std::vector<std::array<float2, GE::TWR>> tw(GE::WG);
  for (int t = 0; t < GE::WG; ++t) {
    float2 tmp[GE::TWR];
    load_lane_twiddles<N>(tmp, table.data(), t % GE::G);
    for (int i = 0; i < GE::TWR; ++i) tw[t][i] = tmp[i];
  }
  return tw;
}

// Filter spectra in kernel order F[K][8][G][2] (as the device plan stores them).
// shift_mask != 0: filter r delayed by row_delay(shift_y, shift_el, shift_ns,
// shift_d, r, shift_mask) samples (output rows off the 128-byte line grid), here by
// placing its taps later (the device plan multiplies its spectra by the
// phase of the delay instead).
template <int N>
std::vector<float2> spectra(const float2* h, int K, int M, const std::vector<float2>& table, bool* guards,
                            bool diff = false, bool real = false, const void* shift_y = nullptr, int shift_el = 8,
                            int64_t shift_ns = 0, int shift_d = 0, int shift_mask = 0) {
  using GE = Geo<N>;
  auto tw = lane_twiddles<N>(table);
  std::vector<float2> F((size_t)K * N);
  Group<N> G;
  G.poison();
  std::vector<std::array<float2, 16>> xs(GE::WG);
  const int blocks = (K + GE::SEGS - 1) / GE::SEGS;
  for (int b = 0; b < blocks; ++b) {
    for (int t = 0; t < GE::WG; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      const int r = b * GE::SEGS + grp;
      const bool valid = r < K;
      float2(&x)[16] = *reinterpret_cast<float2(*)[16]>(xs[t].data());
      const int64_t row = (int64_t)(valid ? r : 0) * M;
      const int delay = shift_mask ? row_delay(shift_y, shift_el, shift_ns, shift_d, r, shift_mask) : 0;
      if (real) load_filter_real<N>(x, reinterpret_cast<const float*>(h) + row, M, valid, diff, g, delay);
      else if (diff) load_filter_diff<N>(x, h + row, M, valid, g, delay);
      else load_filter<N>(x, h + row, M, valid, g, delay);
    }
    fwd_from<N, 0>(xs, G, tw);
    for (int t = 0; t < GE::WG; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      const int r = b * GE::SEGS + grp;
      if (r < K) store_spectrum<N>(*reinterpret_cast<float2(*)[16]>(xs[t].data()), F.data(), r, g, 1.0f / (float)N);
    }
  }
  if (guards) *guards = G.guards_ok();
  return F;
}

// Units [u0, u1) of one signal through the kernel's per-lane code (the body
// of the device range function); a unit is one tile and NF filters.
template <int N>
void forward_range(const float2* s, int64_t Ns, const float2* F, float2* y, int K, int D, int H, int64_t u0,
                   int64_t u1, Group<N>& G, const std::vector<std::array<float2, Geo<N>::TWR>>& tw, int NF = 1,
                   bool power = false, bool real = false, const Stencil* st = nullptr, int shift_mask = 0) {
  using GE = Geo<N>;
  const int KG = (K + NF - 1) / NF;
  std::vector<std::array<float2, 16>> xs(GE::WG), A(GE::WG);
  UnitWalk w(u0, KG);  // the device kernels' walk
  auto forward_tile = [&]() {
    for (int t = 0; t < GE::WG; ++t) {
      const int grp = t / GE::G, g = t % GE::G;
      const int64_t seg = w.tile * GE::SEGS + grp;
      float2(&x)[16] = *reinterpret_cast<float2(*)[16]>(xs[t].data());
      if (real) load_segment_pair<N>(x, reinterpret_cast<const float*>(s), Ns, seg * 2 * H - D, H, g);
      else load_segment<N>(x, s, Ns, seg * H - D, g);
    }
    fwd_from<N, 0>(xs, G, tw);
    A = xs;
  };
  forward_tile();
  for (int64_t u = u0; u < u1; ++u) {
    if (w.tile_done(KG)) {
      w.next_tile();
      forward_tile();
    }
    for (int f = 0; f < NF; ++f) {
      const int r = w.rg * NF + f;
      if (r >= K) continue;  // padded last group: computed on the device, never stored
      for (int t = 0; t < GE::WG; ++t) {
        const int g = t % GE::G;
        float2 a[16];
        for (int i = 0; i < 16; ++i) a[i] = A[t][i];
        load_spectrum<N>(*reinterpret_cast<float2(*)[16]>(xs[t].data()), F, r, g);
        product_pass<N>(*reinterpret_cast<float2(*)[16]>(xs[t].data()), a);
      }
      exchange_phase<N, GE::P - 2, GE::P - 1, GE::P - 2>(xs, G);
      inv_from<N, GE::P - 2>(xs, G, tw);
      if (st) {
        // the non-local stage: each segment's outputs staged in slots that
        // start as NaN, so a kept output that read an unstaged slot shows up
        const int64_t row = (int64_t)r * st->J * Ns;
        for (int grp = 0; grp < GE::SEGS; ++grp) {
          std::vector<float2> region(stage_stride<N>(), make_float2(NAN, NAN));
          for (int g = 0; g < GE::G; ++g)
            stage_write<N>(region.data(), *reinterpret_cast<const float2(*)[16]>(xs[grp * GE::G + g].data()), g);
          const int64_t seg = w.tile * GE::SEGS + grp;
          float* yr = reinterpret_cast<float*>(y) + row;
          for (int g = 0; g < GE::G; ++g) {
            if (real && power) stage_store<N, true, true>(region.data(), *st, yr, Ns, seg * 2 * H, D, H, g);
            else if (real) stage_store<N, false, true>(region.data(), *st, yr, Ns, seg * 2 * H, D, H, g);
            else if (power) stage_store<N, true, false>(region.data(), *st, yr, Ns, seg * H, D, H, g);
            else stage_store<N, false, false>(region.data(), *st, y + row, Ns, seg * H, D, H, g);
          }
        }
        continue;
      }
      for (int t = 0; t < GE::WG; ++t) {
        const int grp = t / GE::G, g = t % GE::G;
        const int64_t seg = w.tile * GE::SEGS + grp;
        const float2(&x)[16] = *reinterpret_cast<float2(*)[16]>(xs[t].data());
        float* yr = reinterpret_cast<float*>(y) + (int64_t)r * Ns;
        const int Dr = D + row_delay(y, (real || power) ? 4 : 8, Ns, D, r, shift_mask);
        if (real && power) store_valid_pair<N, true>(x, yr, Ns, seg * 2 * H, Dr, H, g);
        else if (real) store_valid_pair<N, false>(x, yr, Ns, seg * 2 * H, Dr, H, g);
        else if (power) store_valid_power<N>(x, yr, Ns, seg * H, Dr, H, g);
        else store_valid<N>(x, y + (int64_t)r * Ns, Ns, seg * H, Dr, H, g);
      }
    }
    w.leave();
  }
}

// post & 8: the library's treatment of output rows off the 128-byte grid
// (row_shift_geometry on the given D and H; delayed filters), whatever the
// size (the library applies it from 2^22 outputs per call on).
template <int N>
int forward(const float2* s, int64_t Ns, const float2* h, int K, int M, int D, int H, int grid, float2* y,
            int post = 0, const Stencil* st = nullptr) {
  using GE = Geo<N>;
  const std::vector<float2> table = build_twiddles<N>();
  bool guards = true;
  const bool real = (post & 4) != 0;
  const int el = (post & 6) ? 4 : 8;
  RowShift rs{H, 0};
  if ((post & 8) && !st) rs = row_shift_geometry(y, Ns, N, D, H, el, true);
  H = rs.H;
  const std::vector<float2> F = spectra<N>(h, K, M, table, &guards, (post & 1) != 0, real, y, el, Ns, D, rs.mask);
  if (!guards) return 2;
  auto tw = lane_twiddles<N>(table);
  const int nf = real ? choose_nf_real(N, K) : choose_nf(N, K);
  const int64_t nseg = (Ns + H - 1) / H;
  const int64_t ntrans = real ? (nseg + 1) / 2 : nseg;
  const int64_t ntiles = (ntrans + GE::SEGS - 1) / GE::SEGS;
  const int64_t U = ntiles * ((K + nf - 1) / nf);
  if (grid > U) grid = (int)U;
  Group<N> G;
  G.poison();
  for (int b = 0; b < grid; ++b) {
    const int64_t u0 = first_unit(U, grid, b), u1 = first_unit(U, grid, b + 1);
    if (u0 < u1) forward_range<N>(s, Ns, F.data(), y, K, D, H, u0, u1, G, tw, nf, (post & 2) != 0, real, st, rs.mask);
  }
  return G.guards_ok() ? 0 : 3;
}

// Adjoint: the same unit partition, tile start/finish, split-tile fixup and
// fixed-order dh reduction as the device kernels.
template <int N>
int backward(const float2* s, int64_t Ns, const float2* gy, const float2* h, int K, int M, int D, int H, int grid,
             float2* ds, float2* dh) {
  using GE = Geo<N>;
  (void)D;
  const std::vector<float2> table = build_twiddles<N>();
  bool guards = true;
  const std::vector<float2> F = spectra<N>(h, K, M, table, &guards);
  if (!guards) return 2;
  auto tw = lane_twiddles<N>(table);
  const int64_t nseg = (Ns + H - 1) / H;
  const int64_t ntiles = (nseg + GE::SEGS - 1) / GE::SEGS;
  const int64_t U = ntiles * K;
  if (grid > U) grid = (int)U;
  const int64_t P = grid;
  std::vector<float2> ws((size_t)P * 2 * GE::SEGS * N, make_float2(0.f, 0.f));
  std::vector<float2> part((size_t)P * GE::SEGS * K * M, make_float2(0.f, 0.f));
  Group<N> G;
  G.poison();
  std::vector<std::array<float2, 16>> xs(GE::WG), A(GE::WG), acc(GE::WG);
  for (int64_t b = 0; b < P; ++b) {
    const int64_t u0 = first_unit(U, P, b), u1 = first_unit(U, P, b + 1);
    if (u0 >= u1) continue;
    const int64_t t_first = u0 / K;
    int64_t tile = t_first;
    int r = (int)(u0 - tile * K);
    for (int t = 0; t < GE::WG; ++t)
      for (int rr = 0; rr < K; ++rr)
        zero_lags<N>(part.data() + ((b * GE::SEGS + t / GE::G) * (int64_t)K + rr) * M, M, t % GE::G);
    auto segof = [&](int t) { return tile * GE::SEGS + t / GE::G; };
    auto start_tile = [&]() {
      for (int t = 0; t < GE::WG; ++t)
        load_window<N>(*reinterpret_cast<float2(*)[16]>(xs[t].data()), s, Ns, segof(t) * H, H, t % GE::G);
      fwd_from<N, 0>(xs, G, tw);
      for (int t = 0; t < GE::WG; ++t) {
        conj_scaled(*reinterpret_cast<float2(*)[16]>(A[t].data()), *reinterpret_cast<float2(*)[16]>(xs[t].data()),
                    1.0f / (float)N);
        for (int i = 0; i < 16; ++i) acc[t][i] = make_float2(0.f, 0.f);
      }
    };
    auto finish_tile = [&]() {
      xs = acc;
      inv_from<N, GE::P - 1>(xs, G, tw);
      const bool complete = tile * K >= u0 && (tile + 1) * K <= u1;
      for (int t = 0; t < GE::WG; ++t) {
        const int grp = t / GE::G, g = t % GE::G;
        const float2(&x)[16] = *reinterpret_cast<float2(*)[16]>(xs[t].data());
        if (complete) {
          store_valid<N>(x, ds, Ns, segof(t) * H, 0, H, g);
        } else {
          const int slot = tile == t_first ? 0 : 1;
          store_valid<N>(x, ws.data() + ((b * 2 + slot) * GE::SEGS + grp) * (int64_t)N, (int64_t)H, 0, 0, H, g);
        }
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
      for (int t = 0; t < GE::WG; ++t)
        load_window<N>(*reinterpret_cast<float2(*)[16]>(xs[t].data()), gy + (int64_t)r * Ns, Ns, segof(t) * H, N,
                       t % GE::G);
      fwd_from<N, 0>(xs, G, tw);
      for (int t = 0; t < GE::WG; ++t) {
        float2 f[16];
        load_spectrum<N>(f, F.data(), r, t % GE::G);
        acc_conj_product(*reinterpret_cast<float2(*)[16]>(acc[t].data()),
                         *reinterpret_cast<float2(*)[16]>(xs[t].data()), f);
        float2 a[16];
        for (int i = 0; i < 16; ++i) a[i] = A[t][i];
        product_pass<N>(*reinterpret_cast<float2(*)[16]>(xs[t].data()), a);
      }
      exchange_phase<N, GE::P - 2, GE::P - 1, GE::P - 2>(xs, G);
      inv_from<N, GE::P - 2>(xs, G, tw);
      for (int t = 0; t < GE::WG; ++t)
        add_lags<N>(part.data() + ((b * GE::SEGS + t / GE::G) * (int64_t)K + r) * M,
                    *reinterpret_cast<float2(*)[16]>(xs[t].data()), M, t % GE::G);
      ++r;
    }
    finish_tile();
  }
  // split-tile fixup, exactly as the device kernel
  for (int64_t bnd = 1; bnd < P; ++bnd) {
    const int64_t ub = first_unit(U, P, bnd);
    if (ub % K == 0) continue;
    const int64_t t = ub / K;
    if (first_unit(U, P, bnd - 1) > t * K) continue;
    const int64_t blo = owner_of_unit(U, P, t * K), bhi = owner_of_unit(U, P, (t + 1) * K - 1);
    for (int i = 0; i < GE::SEGS * H; ++i) {
      const int sg = i / H, p = i - sg * H;
      const int64_t o = (t * GE::SEGS + sg) * H + p;
      if (o >= Ns) continue;
      float2 a = make_float2(0.f, 0.f);
      for (int64_t bb = blo; bb <= bhi; ++bb) {
        const int slot = first_unit(U, P, bb) / K == t ? 0 : 1;
        a = cadd(a, ws[((bb * 2 + slot) * GE::SEGS + sg) * (int64_t)N + p]);
      }
      ds[o] = a;
    }
  }
  const int64_t KM = (int64_t)K * M, nslots = P * GE::SEGS, nch = dh_chunks(nslots);
  for (int64_t i = 0; i < KM; ++i) {
    float2 a = make_float2(0.f, 0.f);
    for (int64_t c = 0; c < nch; ++c) {
      float2 cs = make_float2(0.f, 0.f);
      for (int64_t sl = c * DH_CHUNK; sl < std::min<int64_t>(nslots, (c + 1) * DH_CHUNK); ++sl)
        cs = cadd(cs, part[sl * KM + i]);
      a = cadd(a, cs);
    }
    dh[i] = a;
  }
  return G.guards_ok() ? 0 : 3;
}

// Batched: the same unit table, equal shares per workgroup, binary search for
// the first item and the walk across items as the device kernel.
struct EmuItem {
  const float2* s;
  float2* y;
  std::vector<float2> F;
  int64_t Ns, unit_begin, units, tile_begin = 0, ntiles = 0;
  int K, M, N, D, H, nf;
  int shift_mask = 0;
};

template <int N>
struct RangeN {
  static int run(EmuItem* itp, int64_t a, int64_t b) {
    EmuItem& it = *itp;
    static thread_local Group<N>* G = nullptr;
    if (!G) { G = new Group<N>(); G->poison(); }
    auto tw = lane_twiddles<N>(build_twiddles<N>());
    forward_range<N>(it.s, it.Ns, it.F.data(), it.y, it.K, it.D, it.H, a, b, *G, tw, it.nf, false, false, nullptr,
                     it.shift_mask);
    return G->guards_ok() ? 0 : 3;
  }
};
template <int N>
struct SpecN {
  static int run(EmuItem* itp, const float2* h) {
    EmuItem& it = *itp;
    bool guards = true;
    it.F = spectra<N>(h, it.K, it.M, build_twiddles<N>(), &guards, false, false, it.y, 8, it.Ns, it.D,
                      it.shift_mask);
    return guards ? 0 : 2;
  }
};

// LDS exchange analysis for one (exchange E, pattern K) over a whole workgroup.
template <int N, int E, int K>
void pattern(std::map<int, int>& seen, int64_t* out, bool writer, std::vector<int>& cells) {
  using GE = Geo<N>;
  constexpr int RK = GE::radix(K);
  for (int j = 0; j < GE::slots(K); ++j) {
    for (int a = 0; a < RK; ++a) {
      std::vector<int> addr(GE::WG);
      for (int t = 0; t < GE::WG; ++t) {
        const int grp = t / GE::G, g = t % GE::G;
        addr[t] = lds_base<N, E, K>(grp, g) + lds_off<N, E, K>(j, a);
        if (addr[t] < 0 || addr[t] >= GE::LDS) out[2]++;
        if (addr[t] + 1 > out[3]) out[3] = addr[t] + 1;
        if (writer) {
          if (seen.count(addr[t])) out[4]++;
          seen[addr[t]] = 1;
        } else {
          cells.push_back(addr[t]);
        }
      }
      for (int lanes = 16; lanes <= 32; lanes *= 2) {
        for (int base = 0; base < GE::WG; base += lanes) {
          std::map<int, int> cnt;
          int worst = 0;
          for (int t = base; t < base + lanes; ++t) worst = std::max(worst, ++cnt[((addr[t] % lanes) + lanes) % lanes]);
          int64_t& w = out[lanes == 16 ? 0 : 1];
          if (worst > w) w = worst;
        }
      }
    }
  }
}

template <int N, int E>
void exchange_report(int64_t* out) {
  // forward direction writes pattern E, reads pattern E+1; inverse the reverse
  std::map<int, int> w1, w2;
  std::vector<int> r1, r2, dummy;
  pattern<N, E, E>(w1, out, true, dummy);
  pattern<N, E, E + 1>(w1, out, false, r1);
  pattern<N, E, E + 1>(w2, out, true, dummy);
  pattern<N, E, E>(w2, out, false, r2);
  for (int a : r1)
    if (!w1.count(a)) out[5]++;
  for (int a : r2)
    if (!w2.count(a)) out[5]++;
  if ((int64_t)r1.size() != (int64_t)w1.size()) out[5]++;
  if constexpr (E + 1 < Geo<N>::P - 1) exchange_report<N, E + 1>(out);
}

template <int N>
void lds_report(int64_t* out) {
  for (int i = 0; i < 8; ++i) out[i] = 0;
  exchange_report<N, 0>(out);
  out[6] = Geo<N>::LDS;
  out[7] = Geo<N>::TW_TOTAL;
}

template <template <int> class F, typename... A>
int dispatch(int N, A... a) {
  switch (N) {
    case 256: return F<256>::run(a...);
    case 512: return F<512>::run(a...);
    case 1024: return F<1024>::run(a...);
    case 2048: return F<2048>::run(a...);
    case 4096: return F<4096>::run(a...);
    case 8192: return F<8192>::run(a...);
  }
  return -1;
}

template <int N>
struct RunFwd {
  static int run(const float2* s, int64_t Ns, const float2* h, int K, int M, int D, int H, int grid, float2* y,
                 int post, const Stencil* st) {
    return forward<N>(s, Ns, h, K, M, D, H, grid, y, post, st);
  }
};
template <int N>
struct RunBwd {
  static int run(const float2* s, int64_t Ns, const float2* gy, const float2* h, int K, int M, int D, int H, int grid,
                 float2* ds, float2* dh) {
    return backward<N>(s, Ns, gy, h, K, M, D, H, grid, ds, dh);
  }
};
template <int N>
struct RunSpec {
  static int run(const float2* h, int K, int M, float2* out) {
    bool guards = true;
    std::vector<float2> F = spectra<N>(h, K, M, build_twiddles<N>(), &guards);
    for (int r = 0; r < K; ++r)
      for (int reg = 0; reg < 16; ++reg)
        for (int g = 0; g < Geo<N>::G; ++g)
          out[(int64_t)r * N + spectrum_index<N>(g, reg)] = F[(int64_t)r * N + spectrum_offset<N>(reg, g)];
    return guards ? 0 : 2;
  }
};
template <int N>
struct RunLds {
  static int run(int64_t* out) {
    lds_report<N>(out);
    return 0;
  }
};
// Exchange E is wave-local when every LDS cell is read (pass E+1 layout) by a
// lane of the same wave that wrote it (pass E layout); out[E] = 1 or 0.
template <int N, int E>
void wave_locality(int32_t* out) {
  using GE = Geo<N>;
  std::map<int, int> writer;
  for (int j = 0; j < GE::slots(E); ++j)
    for (int a = 0; a < GE::radix(E); ++a)
      for (int t = 0; t < GE::WG; ++t)
        writer[lds_base<N, E, E>(t / GE::G, t % GE::G) + lds_off<N, E, E>(j, a)] = t / 64;
  int local = 1;
  for (int j = 0; j < GE::slots(E + 1); ++j)
    for (int a = 0; a < GE::radix(E + 1); ++a)
      for (int t = 0; t < GE::WG; ++t) {
        auto it = writer.find(lds_base<N, E, E + 1>(t / GE::G, t % GE::G) + lds_off<N, E, E + 1>(j, a));
        if (it == writer.end() || it->second != t / 64) local = 0;
      }
  out[E] = local;
  if constexpr (E + 1 < GE::P - 1) wave_locality<N, E + 1>(out);
}

template <int N>
struct RunWaveLocal {
  static int run(int32_t* out) {
    wave_locality<N, 0>(out);
    return 0;
  }
};

template <int N>
struct RunGeo {
  static int run(int32_t* out) {
    using GE = Geo<N>;
    out[0] = GE::G;
    out[1] = GE::P;
    out[2] = GE::R0;
    out[3] = GE::WG;
    out[4] = GE::SEGS;
    out[5] = GE::LDS;
    out[6] = GE::TWR;
    return 0;
  }
};

}  // namespace emu
}  // namespace ols

extern "C" {

// y[K][Ns] (interleaved floats) = forward overlap-and-save through the kernel
// dataflow.  Returns 0 on success, 2/3 if an LDS guard band was touched, -1 for
// an unsupported N.
int ols_emu_forward(int N, const float* s, int64_t Ns, const float* h, int K, int M, int D, int H, int grid, float* y) {
  return ols::emu::dispatch<ols::emu::RunFwd>(N, (const float2*)s, Ns, (const float2*)h, K, M, D, H, grid, (float2*)y,
                                              0, (const ols::Stencil*)nullptr);
}

// As ols_emu_forward with the flags of ols_plan_ex (1: first difference folded
// into the spectra, 2: power |y|^2 stored as float [K][Ns], 4: R2R, s float
// [Ns], h float [K][M], y float [K][Ns]).
int ols_emu_forward_post(int N, const float* s, int64_t Ns, const float* h, int K, int M, int D, int H, int grid,
                         int post, float* y) {
  return ols::emu::dispatch<ols::emu::RunFwd>(N, (const float2*)s, Ns, (const float2*)h, K, M, D, H, grid, (float2*)y,
                                              post, (const ols::Stencil*)nullptr);
}

// As ols_emu_forward_post with the non-local stencil stage (J phases, left
// and right reach, weights w[J][left + 1 + right]); y holds [K][J*Ns] outputs.
// packed = 1 takes the packed store form where the library would (J <= 2, y
// aligned to J elements), 0 never.  Returns 1 for an invalid stencil.
int ols_emu_forward_stencil(int N, const float* s, int64_t Ns, const float* h, int K, int M, int D, int H, int grid,
                            int post, int J, int L, int R, const float* w, int packed, float* y) {
  if (J < 1 || J > ols::STENCIL_MAX_PHASES || L < 0 || R < 0 || L + 1 + R > ols::STENCIL_MAX_TAPS) return 1;
  ols::Stencil st{};
  const uintptr_t el = (uintptr_t)J * ((post & 6) ? 4 : 8);
  st.packed = packed && J <= 2 && (uintptr_t)y % el == 0;
  st.J = J;
  st.L = L;
  st.T = L + 1 + R;
  for (int j = 0; j < J; ++j)
    for (int d = 0; d < st.T; ++d) st.w[j][d] = w[j * st.T + d];
  return ols::emu::dispatch<ols::emu::RunFwd>(N, (const float2*)s, Ns, (const float2*)h, K, M, D, H, grid, (float2*)y,
                                              post, (const ols::Stencil*)&st);
}

// First kept position of a plan with a stencil reaching L back and R ahead
// (the host plan code's rule; the hop is N - D - R).
int ols_emu_stencil_delay(int N, int Meff, int L, int R) { return ols::stencil_delay(N, Meff, L, R); }

// Default hop of such a plan.
int ols_emu_stencil_hop(int N, int D, int R) { return ols::stencil_hop(N, D, R); }

// Batched geometry for an item with output y and N_s samples: out[0] = D,
// out[1] = H, out[2] = the mask of its per-row filter delays (0: rows on the
// 128-byte grid); and the delay of row r.
void ols_emu_batch_geometry(int N, int M, const void* y, int64_t Ns, int32_t* out) {
  out[0] = ols::default_delay(N, M);
  const ols::RowShift rs = ols::batch_row_shift(y, Ns, N, out[0]);
  out[2] = rs.mask;
  out[1] = rs.H;
}
int ols_emu_row_shift(const void* y, int64_t Ns, int D, int r, int mask) { return ols::row_delay(y, 8, Ns, D, r, mask); }

// The single-signal forward's rule for a call: out[0] = H, out[1] = mask,
// for outputs of el bytes (8 complex64, 4 float32) and the plan's D, H.
void ols_emu_row_shift_geometry(const void* y, int64_t Ns, int N, int D, int H, int el, int32_t* out) {
  const ols::RowShift rs = ols::row_shift_geometry(y, Ns, N, D, H, el, true);
  out[0] = rs.H;
  out[1] = rs.mask;
}

// Adjoint through the kernel dataflow: ds[N_s], dh[K][M].
int ols_emu_backward(int N, const float* s, int64_t Ns, const float* gy, const float* h, int K, int M, int D, int H,
                     int grid, float* ds, float* dh) {
  return ols::emu::dispatch<ols::emu::RunBwd>(N, (const float2*)s, Ns, (const float2*)gy, (const float2*)h, K, M, D,
                                              H, grid, (float2*)ds, (float2*)dh);
}

// Batched forward through the kernel dataflow.  Per item: s, y (host), N_s,
// K, M, N (must be given, 256..4096), D, H; H = 0 takes the library's
// geometry (default delay, and the row shift of rows off the 128-byte line grid).
// grid = persistent workgroups.
int ols_emu_batched(int n, const float* const* s, float* const* y, const int64_t* Ns, const float* const* h,
                    const int* K, const int* M, const int* N, const int* D, const int* H, int grid) {
  using namespace ols::emu;
  std::vector<EmuItem> items(n);
  int64_t units = 0, tiles = 0;
  for (int i = 0; i < n; ++i) {
    EmuItem& it = items[i];
    it.s = (const float2*)s[i];
    it.y = (float2*)y[i];
    it.Ns = Ns[i];
    it.K = K[i];
    it.M = M[i];
    it.N = N[i];
    if (H[i] == 0) {
      it.D = ols::default_delay(it.N, it.M);
      const ols::RowShift rs = ols::batch_row_shift(it.y, it.Ns, it.N, it.D);
      it.shift_mask = rs.mask;
      it.H = rs.H;
    } else {
      it.D = D[i];
      it.H = H[i];
    }
    it.nf = ols::choose_nf_batched(it.N, it.K);
    const int segs = 4096 / it.N;
    const int64_t nseg = (it.Ns + it.H - 1) / it.H;
    it.ntiles = (nseg + segs - 1) / segs;
    it.units = it.ntiles * ((it.K + it.nf - 1) / it.nf);
    if (dispatch<SpecN>(it.N, &it, (const float2*)h[i]) != 0) return 2;
  }
  // the plan's kernel order: items by class (N, filters per unit), stable
  std::stable_sort(items.begin(), items.end(), [](const EmuItem& u, const EmuItem& v) {
    return u.N != v.N ? u.N < v.N : u.nf < v.nf;
  });
  for (EmuItem& it : items) {
    it.unit_begin = units;
    units += it.units;
    it.tile_begin = tiles;
    tiles += it.ntiles;
  }
  // the device schedule (first_batch_tile, next_batch_tile,
  // batch_workgroup_order): chunks of tiles dealt round-robin to the grid,
  // each workgroup taking its tiles in runs of one class
  const int64_t P = grid;
  for (int64_t blk = 0; blk < P; ++blk) {
    int i = 0;
    int64_t t = ols::first_batch_tile(ols::batch_workgroup_order(blk, P));
    int runs = 0;
    while (t < tiles) {
      while (i + 1 < n && items[i + 1].tile_begin <= t) ++i;
      const int N = items[i].N, nf = items[i].nf;
      ++runs;
      for (;;) {
        EmuItem& it = items[i];
        if (t < it.tile_begin || t >= it.tile_begin + it.ntiles) return 4;  // walk invariant
        const int64_t per_tile = it.units / it.ntiles;
        const int64_t a = (t - it.tile_begin) * per_tile;
        if (dispatch<RangeN>(it.N, &it, a, a + per_tile) != 0) return 3;
        t = ols::next_batch_tile(t, P);
        if (t >= tiles) break;
        while (i + 1 < n && items[i + 1].tile_begin <= t) ++i;
        if (items[i].N != N || items[i].nf != nf) break;
      }
    }
    if (runs > 10) return 5;  // at most one run per class (5 lengths x 2)
  }
  (void)units;
  return 0;
}

// Natural-order filter spectra out[K][N] = FFT_N(pad h_r) / N through the kernel dataflow.
int ols_emu_spectra(int N, const float* h, int K, int M, float* out) {
  return ols::emu::dispatch<ols::emu::RunSpec>(N, (const float2*)h, K, M, (float2*)out);
}

// out[0] worst bank multiplicity for 16-lane groups / 16 slots (32 banks),
// out[1] for 32-lane groups / 32 slots (64 banks), out[2] out-of-range LDS
// addresses, out[3] highest address + 1, out[4] double writes within one
// exchange, out[5] reads of cells not written by the exchange, out[6] LDS
// size (float2), out[7] twiddle table size.
int ols_emu_lds_report(int N, int64_t* out) { return ols::emu::dispatch<ols::emu::RunLds>(N, out); }

// The library's FFT-length cost model (exact integer comparison) for K
// filters of M taps and lengths up to max_n; 0 if none fits.
int ols_emu_cost_model(int K, int M, int max_n) { return ols::cost_model_fft_length(K, M, max_n); }

// out[0..6] = G, P, R0, WG, SEGS, LDS (float2), TWR
int ols_emu_geometry(int N, int32_t* out) { return ols::emu::dispatch<ols::emu::RunGeo>(N, out); }

// out[E] = 1 if exchange E (between passes E and E+1) keeps every value in
// the wave that wrote it, for E = 0 .. P-2.
int ols_emu_wave_local(int N, int32_t* out) { return ols::emu::dispatch<ols::emu::RunWaveLocal>(N, out); }

}  // extern "C"
