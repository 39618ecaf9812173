// Per-wavefront form of the fused pass (forward FFT along the last axis, spectral
// multiply, inverse FFT) for complex lines of a power-of-two length.
//
// One line of M points is spread over P = M / E lanes of a 64-lane wavefront; lane j of
// the line holds points j + P m (m < E) in registers.  This is the layout of the input
// as loaded from HBM (consecutive lanes read consecutive points), of the spectrum after
// the forward transform and of the output before the store, so the forward transform,
// the multiplication by the Green's spectrum (or the spectral curl) and the inverse
// transform follow each other in registers.  The FFT is a Stockham radix schedule: the
// first stage is a radix-E butterfly over a lane's own registers, the later stages take
// their inputs from the other lanes of the line through a per-wave LDS buffer, and the
// last stage leaves the outputs in natural order in the lane layout above.  Nothing is
// shared between wavefronts, so there is no workgroup barrier: the LDS exchanges are
// ordered within the wave only.  L = 64 / P lines share a wavefront, W wavefronts a
// workgroup (one tile of W * L lines).
#pragma once
#include "fm_device.h"

namespace fm {

template <typename T, int M, int E_>
struct WaveShape {
  static constexpr int E = E_;
  static constexpr int P = M / E;
  static constexpr int L = 64 / P;
};

// LDS ordering between the lanes of one wavefront: every LDS access of the wave issued
// before the call is performed before any issued after it (LDS operations of a
// wavefront are performed in order; the fences keep the compiler from moving accesses
// across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage s of the wave FFT (sign S) and all later stages.  Before the stage, v[i R + r]
// holds input r of the lane's butterfly i (t = j + P i), i.e. point t + r M / R; the
// first stage's inputs are the lane layout itself (one butterfly, t = j).  After the
// last stage v[m] holds output j + P m.
template <typename T, int M, int E, int s, int S, class TW>
__device__ __forceinline__ void wave_stages(cpx<T> (&v)[E], int j, cpx<T>* buf, TW tw) {
  constexpr int P = M / E;
  constexpr int R = wave_radix(M, s, E);
  if constexpr (R != 0) {
    constexpr int Ns = wave_ns(M, s, E);
    constexpr int NB = E / R;  // butterflies per lane
    if constexpr (s > 0) {
      // W_{Ns R}^{k r}, k = t mod Ns (table: offset + (r - 1) Ns + k)
      constexpr int off = wave_tw_offset(M, s, E);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int k = (j + P * i) & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const auto& g = tw[off + (r - 1) * Ns + k];
          const cpx<T> w = {g.x, S > 0 ? -g.y : g.y};
          v[i * R + r] = cmul(v[i * R + r], w);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) SmallDft<R, S, T>::run(&v[i * R]);
    constexpr int R2 = wave_radix(M, s + 1, E);
    if constexpr (R2 == 0) {
      // last stage: output q of butterfly i is point t + q Ns = j + P (i + NB q)
      cpx<T> nat[E];
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int q = 0; q < R; ++q) nat[i + NB * q] = v[i * R + q];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = nat[e];
    } else {
      // exchange through the wave's LDS line: output q of butterfly t goes to
      // (t - k) R + k + q Ns; the next stage reads point t' + r M / R2
      constexpr int NB2 = E / R2;
      constexpr int MR2 = M / R2;
      wave_lds_sync();  // the previous exchange's reads are done
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int t = j + P * i;
        const int k = t & (Ns - 1);
        const int base = (t - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) buf[pad16(base + q * Ns)] = v[i * R + q];
      }
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < NB2; ++i) {
        const int t = j + P * i;
#pragma unroll
        for (int r = 0; r < R2; ++r) v[i * R2 + r] = buf[pad16(t + r * MR2)];
      }
      wave_stages<T, M, E, s + 1, S, TW>(v, j, buf, tw);
    }
  }
}

// One tile of the fused pass: W wavefronts of L lines each.  KIND is K_F_C2C (Poisson:
// times the Green's spectrum) or K_F_CURL (three components per line: u = G i w x f).
template <typename T, int M, int KIND, int EV>
__device__ __forceinline__ void wave_tile(const PassDesc& d, const void* in, void* out, char* smem,
                                          int tile) {
  using WS = WaveShape<T, M, EV>;
  constexpr int E = WS::E, P = WS::P, L = WS::L;
  constexpr int NCL = KIND == K_F_CURL ? 3 : 1;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int j = lane % P;
  const int l = wave * L + lane / P;  // line of the tile
  const TileIdx ti = tile_index(d, tile);
  if (l >= ti.nl) return;  // no workgroup barrier follows
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem) + (size_t)(wave * L + lane / P) * fft_line_stride(M);
  const GTab<T> tw = gptr<cpx<T>>(E == 16 ? d.wtw : (E == 8 ? d.wtw8 : d.wtw32));
  const int b = ti.b0 + l;
  const int comp0 = NCL == 3 ? 0 : ti.comp;
  const int64_t line_off = (int64_t)ti.c * d.in_s_c + (int64_t)b * d.in_s_b;

  // the Green's row of the line, folded: G[fold(k)] for k = j + P m (coalesced; the upper
  // half of a row reads the lower half again, from cache)
  const auto* G = gptr<T>(d.g.G);
  const int64_t grow = ((int64_t)fold_index(ti.c, d.g.fold_c) * d.g.F_b + fold_index(b, d.g.fold_b)) *
                       (int64_t)d.g.F_line;
  // Poisson: the row is loaded ahead of the transforms (its latency hides behind them);
  // the curl loads it after its three forward transforms, when registers are free
  T g[E];
  if constexpr (KIND != K_F_CURL) {
#pragma unroll
    for (int m = 0; m < E; ++m) g[m] = G[grow + fold_index(j + P * m, d.g.fold_line)];
  }

  cpx<T> v[NCL][E];
#pragma unroll
  for (int q = 0; q < NCL; ++q) {
    const auto* src = gptr<cpx<T>>(in) + (int64_t)(comp0 + q) * d.in_s_comp + line_off;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int n = j + P * m;
      v[q][m] = cpx<T>{T(0), T(0)};
      if (n < d.n_data) {
        const auto& z = src[n];
        v[q][m] = cpx<T>{z.x, z.y};
      }
    }
    wave_stages<T, M, E, 0, -1>(v[q], j, buf, tw);
  }
  if constexpr (KIND == K_F_CURL) {
#pragma unroll
    for (int m = 0; m < E; ++m) g[m] = G[grow + fold_index(j + P * m, d.g.fold_line)];
    T wc, mc, wb, mb;
    curl_factor<T>(d.g.csym, curl_wave<T>(ti.c, d.g.dtab_c), wc, mc);
    if constexpr (sizeof(T) == 8 && E == 16) {
      // no symmetric b direction in this instance (its registers are full; the planner
      // keeps such passes off it)
      wb = curl_wave<T>(b, d.g.dtab_b);
      mb = T(0);
    } else {
      curl_factor<T>(d.g.csym_b, curl_wave<T>(b, d.g.dtab_b), wb, mb);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const T wl = curl_wave<T>(j + P * m, d.g.dtab_line);
      const T wx = d.g.axis_line == 0 ? wl : (d.g.axis_b == 0 ? wb : wc);
      const T wy = d.g.axis_line == 1 ? wl : (d.g.axis_b == 1 ? wb : wc);
      const T wz = d.g.axis_line == 2 ? wl : (d.g.axis_b == 2 ? wb : wc);
      curl_point<T>(g[m], wx, wy, wz, d.g.axis_c, mc, d.g.axis_b, mb, v[0][m], v[1][m], v[2][m]);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[0][m] = {v[0][m].x * g[m], v[0][m].y * g[m]};
  }
#pragma unroll
  for (int q = 0; q < NCL; ++q) {
    wave_stages<T, M, E, 0, +1>(v[q], j, buf, tw);
    auto* dst = (__attribute__((address_space(1))) cpx<T>*)(out) +
                (int64_t)(comp0 + q) * d.out_s_comp + (int64_t)ti.c * d.out_s_c + (int64_t)b * d.out_s_b;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int n = j + P * m;
      if (n < d.out_n) {
        dst[n].x = v[q][m].x;
        dst[n].y = v[q][m].y;
      }
    }
  }
}

// Tiles in the XCD-aware order of the other pass kernels; a grid of one workgroup per
// tile gives each workgroup one or two tiles.
// Occupancy targets of the three-component (curl) kernels: 16 values per lane (1024-point
// lines) keep one wave per SIMD, where FP32 fits without spilling (two waves spill some
// 300 bytes per lane and ran 20 % slower on the 512^3 Biot-Savart pass) and FP64 takes the
// 512 architectural and accumulation registers; 8 FP32 values fit the 168 of three (FP64
// would spill there and keeps the compiler's choice).
template <typename T, int KIND, int E>
constexpr int wave_min_waves() {
  return KIND == K_F_CURL ? (E == 16 ? 1 : (sizeof(T) == 4 ? 3 : 1)) : 1;
}

template <typename T, int M, int KIND, int E>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(wave_min_waves<T, KIND, E>())))
void wave_pass_kernel(const PassDesc* __restrict__ dp, const void* in, void* out) {
  extern __shared__ __align__(16) char smem[];
  const PassDesc& d = *dp;
  for (int k = 0;; ++k) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, k, d.tiles);
    if (tile < 0) return;
    wave_tile<T, M, KIND, E>(d, in, out, smem, tile);
  }
}

// ---------------------------------------------------------------------------------
// Per-wavefront form of the plain passes (one axis, forward or inverse, any gather and
// scatter).  The tile is staged in LDS as in the LDS-tile kernel, so strided lines are
// still loaded and stored in coalesced rows, but each wavefront then transforms its own
// FFT lines in registers with the schedule above: three workgroup barriers per tile
// instead of one per radix stage.  Four wavefronts of L = 64 / P FFT lines each; a
// packed kind (two real lines per FFT) holds 2 L tile lines per wavefront, so a tile is
// B = 4 L (or 8 L) lines, a power of two.  The raw lines of wavefront w sit inside the
// LDS region of its own FFT lines: all its raw values are read before its first exchange
// write, and no other wavefront touches the region until the next workgroup barrier.
//
// A persistent grid: each workgroup loops over its tiles, and the input of its next
// tile is loaded into registers while the current one is transformed and stored.  The
// stage twiddles (and the real-to-real post-twiddles) are copied to LDS once, so the
// transform issues no global load that would wait for that prefetch (vector-memory
// loads complete in order).  Every per-thread address that does not depend on the tile
// is formed once: in the strided (across-lines) walk a thread owns tile line tid mod B
// and rows tid / B + u kThreads / B.
// ---------------------------------------------------------------------------------
template <typename T, int M, int KIND, int E_>
struct WavePlain {
  static constexpr int E = E_;
  static constexpr int P = M / E;                         // lanes per FFT line
  static constexpr int L = 64 / P;                        // FFT lines per wavefront
  static constexpr int PK = gather_of(KIND) == G_CPLX ? 1 : 2;  // tile lines per FFT line
  static constexpr int RW = L * PK;                       // tile lines per wavefront
  static constexpr int B = 4 * RW;                        // tile lines
  static constexpr int STEP = kThreads / B;               // rows per value, strided walk
  static constexpr int LS = fft_line_stride(M);
  static constexpr bool CIN = in_cplx_of(KIND);
  using In = typename std::conditional<CIN, cpx<T>, T>::type;
  static constexpr int REGION = L * LS * (CIN ? 1 : 2);   // a wavefront's LDS, in In units
  // input values per thread: B in_n / kThreads with in_n <= M + 1 (a node-centred periodic
  // line keeps its duplicate end point), or M / 2 + 1 for the packed half spectra and
  // real-to-real lines
  static constexpr int U = KIND == K_R2C ? 2 * E + 1 : E + 1;
  static constexpr int NTW = wave_tw_size(M, E);          // stage twiddles
  static constexpr int NPOST = KIND == K_R2R ? 2 * M : 0; // real-to-real post-twiddles
  static constexpr int NSLOT = KIND == K_R2R ? M : 0;     // real-to-real gather slots
};

// Input values of one tile into registers (strided walk: only rows below in_n).
template <class WP, class Stage>
__device__ __forceinline__ void wp_fetch(Stage& r, const PassDesc& d,
                                         const void* in, const TileIdx& ti, bool lc) {
  using In = typename WP::In;
  const char* base = reinterpret_cast<const char*>(in) +
                     ((int64_t)ti.comp * d.in_s_comp + (int64_t)ti.c * d.in_s_c +
                      (int64_t)ti.b0 * d.in_s_b) * (int64_t)sizeof(In);
  const int tid = (int)threadIdx.x;
  if (lc) {
    const int total = ti.nl * d.in_n;
#pragma unroll
    for (int u = 0; u < WP::U; ++u) {
      const int e = tid + u * kThreads;
      if (e < total) {
        const uint32_t l = fdiv((uint32_t)e, d.mag_in);
        const uint32_t i = (uint32_t)e - l * (uint32_t)d.in_n;
        r.set(u, *reinterpret_cast<const In*>(base + (l * (uint32_t)d.in_s_b + i) * (uint32_t)sizeof(In)));
      }
    }
  } else {
    const int l = tid % WP::B, i0 = tid / WP::B;
    if (l < ti.nl) {
      const uint32_t o0 = ((uint32_t)l * (uint32_t)d.in_s_b + (uint32_t)i0 * (uint32_t)d.in_s_line) *
                          (uint32_t)sizeof(In);
      const uint32_t ds = (uint32_t)WP::STEP * (uint32_t)d.in_s_line * (uint32_t)sizeof(In);
#pragma unroll
      for (int u = 0; u < WP::U; ++u)
        if (i0 + u * WP::STEP < d.in_n) r.set(u, *reinterpret_cast<const In*>(base + o0 + (uint32_t)u * ds));
    }
  }
}

// Registers -> raw tile: tile line l at (l / RW) REGION + (l mod RW) rs.
template <class WP, class Stage>
__device__ __forceinline__ void wp_commit(const Stage& r, const PassDesc& d,
                                          const TileIdx& ti, char* smem, bool lc) {
  using In = typename WP::In;
  In* raw = reinterpret_cast<In*>(smem);
  const int rs = d.wave_rs, tid = (int)threadIdx.x;
  if (lc) {
    const int total = ti.nl * d.in_n;
#pragma unroll
    for (int u = 0; u < WP::U; ++u) {
      const int e = tid + u * kThreads;
      if (e < total) {
        const int l = (int)fdiv((uint32_t)e, d.mag_in);
        const int i = e - l * d.in_n;
        raw[(l / WP::RW) * WP::REGION + (l % WP::RW) * rs + i] = r.get(u);
      }
    }
  } else {
    const int l = tid % WP::B, i0 = tid / WP::B;
    if (l < ti.nl) {
      In* row = raw + (l / WP::RW) * WP::REGION + (l % WP::RW) * rs + i0;
#pragma unroll
      for (int u = 0; u < WP::U; ++u)
        if (i0 + u * WP::STEP < d.in_n) row[u * WP::STEP] = r.get(u);
    }
  }
}

// Real-to-real gather: slot m of the symmetric extension of line pair (2f, 2f + 1) is
// W_m (x_{2f}[s_m] + i x_{2f+1}[s_m]), with the source index s_m and the complex weight
// W_m (end-point weight, mirror sign, pre-twiddle) the same for every line and tile:
// a table of M entries built in LDS once per workgroup.
template <typename T>
struct R2RSlot {
  T wx, wy;
  int idx, pad;
};

template <typename T, int M, int KIND, int E>
__device__ __forceinline__ void wp_transform(const PassDesc& d, const TileIdx& ti, char* smem,
                                             const cpx<T>* ltw, const R2RSlot<T>* slots) {
  using WP = WavePlain<T, M, KIND, E>;
  using In = typename WP::In;
  constexpr int P = WP::P, L = WP::L, PK = WP::PK;
  constexpr int S = (KIND == K_C2C_I || KIND == K_C2R) ? +1 : -1;
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int j = lane % P, lf = lane / P;  // lane of the line, line of the wavefront
  const int f = wave * L + lf;            // FFT line of the tile
  if (f >= (ti.nl + PK - 1) / PK) return;
  cpx<T>* line = reinterpret_cast<cpx<T>*>(smem) + (size_t)f * WP::LS;
  const In* raw = reinterpret_cast<const In*>(smem) + wave * WP::REGION;
  const int nlw = ti.nl - wave * WP::RW;  // tile lines from the wavefront's first
  const int rs = d.wave_rs;
  cpx<T> v[E];
  if constexpr (gather_of(KIND) == G_CPLX) {
    const GatherCplx<T> g{raw, rs, d.n_data};
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = g(lf, j + P * k);
  } else if constexpr (gather_of(KIND) == G_REAL2) {
    const GatherReal2<T> g{raw, rs, d.n_data, nlw};
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = g(lf, j + P * k);
  } else if constexpr (gather_of(KIND) == G_HERM2) {
    const GatherHerm2<T> g{raw, rs, M, nlw};
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = g(lf, j + P * k);
  } else {
    const T* r0 = raw + (2 * lf) * rs;
    const T* r1 = (2 * lf + 1 < nlw) ? r0 + rs : nullptr;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const R2RSlot<T> sl = slots[j + P * k];
      const T a = r0[sl.idx];
      const T b = r1 ? r1[sl.idx] : T(0);
      v[k] = cpx<T>{a * sl.wx - b * sl.wy, a * sl.wy + b * sl.wx};
    }
  }
  wave_stages<T, M, E, 0, S>(v, j, line, ltw);
  wave_lds_sync();  // the last exchange's reads are done
#pragma unroll
  for (int k = 0; k < E; ++k) line[pad16(j + P * k)] = v[k];
}

// One output element (line l, index j) with the last pass's fix-ups.
template <bool FIX, typename O>
__device__ __forceinline__ void wp_put(O* o, const PassDesc& d, const TileIdx& ti, int l, uint32_t off,
                                       O w, bool czero, bool cdup) {
  if constexpr (FIX) {
    const Fixup& fx = d.fix;
    const int b = ti.b0 + l;
    if (czero || (fx.b_zero_lo && b == 0) || (fx.b_zero_hi && b == fx.b_last)) w = O{};
    o[off] = w;
    const bool bdup = fx.b_dup && b == 0;
    if (bdup) o[off + (int64_t)fx.b_last * d.out_s_b] = w;
    if (cdup) {
      o[off + (int64_t)fx.c_last * d.out_s_c] = w;
      if (bdup) o[off + (int64_t)fx.b_last * d.out_s_b + (int64_t)fx.c_last * d.out_s_c] = w;
    }
  } else {
    (void)d; (void)ti; (void)l; (void)czero; (void)cdup;
    o[off] = w;
  }
}

template <typename T, int M, int KIND, int E, bool FIX>
__device__ __forceinline__ void wp_store(const PassDesc& d, void* out, const TileIdx& ti,
                                         const char* smem, const cpx<T>* lpost, bool lc) {
  using WP = WavePlain<T, M, KIND, E>;
  constexpr int SC = scatter_of(KIND);
  using O = typename std::conditional<SC == S_CPLX || SC == S_R2C2, cpx<T>, T>::type;
  constexpr int LS = WP::LS;
  const cpx<T>* buf = reinterpret_cast<const cpx<T>*>(smem);
  O* o = reinterpret_cast<O*>(out) + (int64_t)ti.comp * d.out_s_comp + (int64_t)ti.c * d.out_s_c +
         (int64_t)ti.b0 * d.out_s_b;
  auto val = [&](int l, int j) -> O {
    if constexpr (SC == S_CPLX) {
      return buf[l * LS + pad16(j < M ? j : j - M)];
    } else if constexpr (SC == S_R2C2) {
      const cpx<T>* z = buf + (l >> 1) * LS;
      const cpx<T> zk = z[pad16(j)], zm = z[pad16(j == 0 ? 0 : M - j)];
      if (l & 1) return cpx<T>{T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
      return cpx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    } else if constexpr (SC == S_REAL2) {
      const cpx<T> z = buf[(l >> 1) * LS + pad16(j < M ? j : j - M)];
      return (l & 1) ? z.y : z.x;
    } else {
      return scatter_r2r<T>(buf, LS, d.r2r, lpost, l, j);
    }
  };
  bool czero = false, cdup = false;
  if constexpr (FIX) {
    czero = (d.fix.c_zero_lo && ti.c == 0) || (d.fix.c_zero_hi && ti.c == d.fix.c_last);
    cdup = d.fix.c_dup && ti.c == 0;
  }
  const int tid = (int)threadIdx.x;
  if (lc) {
    const int total = ti.nl * d.out_n;
    for (int e0 = tid; e0 < total; e0 += 4 * kThreads) {
      O w[4];
      int ll[4];
      uint32_t off[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + q * kThreads;
        ll[q] = -1;
        if (e < total) {
          const int l = (int)fdiv((uint32_t)e, d.mag_out);
          const int j = e - l * d.out_n;
          ll[q] = l;
          off[q] = (uint32_t)l * (uint32_t)d.out_s_b + (uint32_t)j;
          w[q] = val(l, j);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (ll[q] >= 0) wp_put<FIX>(o, d, ti, ll[q], off[q], w[q], czero, cdup);
    }
  } else {
    const int l = tid % WP::B, j0 = tid / WP::B;
    if (l >= ti.nl) return;
    const uint32_t ob = (uint32_t)l * (uint32_t)d.out_s_b;
    const uint32_t sl = (uint32_t)d.out_s_line;
    for (int jb = j0; jb < d.out_n; jb += 4 * WP::STEP) {
      O w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jb + q * WP::STEP;
        if (j < d.out_n) w[q] = val(l, j);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = jb + q * WP::STEP;
        if (j < d.out_n) wp_put<FIX>(o, d, ti, l, ob + (uint32_t)j * sl, w[q], czero, cdup);
      }
    }
  }
}

// Occupancy targets of the plain per-wavefront kernels that fit them without spilling:
// FP32 with 8 values per lane four waves per SIMD (128 VGPRs), with 16 three (168); FP64
// keeps the compiler's choice.
template <typename T, int KIND, int E>
constexpr int wave_plain_min_waves() {
  return sizeof(T) == 4 ? (E == 8 ? 4 : 3) : 1;
}

template <typename T, int M, int KIND, int E>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(wave_plain_min_waves<T, KIND, E>())))
void wave_plain_kernel(const PassDesc* __restrict__ dp, const void* in, void* out) {
  using WP = WavePlain<T, M, KIND, E>;
  using In = typename WP::In;
  extern __shared__ __align__(16) char smem[];
  const PassDesc& d = *dp;
  int k = 0;
  int tile = xcd_tile(blockIdx.x, gridDim.x, k, d.tiles);
  if (tile < 0) return;
  const bool lc_in = d.in_s_line == 1, lc_out = d.out_s_line == 1;
  // the first tile's input is requested before the tables are copied, so that its HBM
  // latency and the tables' overlap (the copy waits for both: loads complete in order)
  TileIdx ti = tile_index(d, tile);
  RegStage<T, In, WP::U> r;
  wp_fetch<WP>(r, d, in, ti, lc_in);
  // tables into LDS, per-thread real-to-real gather weights
  cpx<T>* ltw = reinterpret_cast<cpx<T>*>(smem + d.tab_off);
  cpx<T>* lpost = ltw + WP::NTW;
  {
    const GTab<T> gtw = gptr<cpx<T>>(E == 16 ? d.wtw : d.wtw8);
    for (int i = (int)threadIdx.x; i < WP::NTW; i += kThreads) ltw[i] = cpx<T>{gtw[i].x, gtw[i].y};
    if constexpr (WP::NPOST > 0) {
      const GTab<T> g4 = gptr<cpx<T>>(d.tw);
      for (int i = (int)threadIdx.x; i < WP::NPOST; i += kThreads) lpost[i] = cpx<T>{g4[i].x, g4[i].y};
    }
  }
  R2RSlot<T>* slots = reinterpret_cast<R2RSlot<T>*>(lpost + WP::NPOST);
  if constexpr (KIND == K_R2R) {
    const GatherR2R<T, GTab<T>> g{nullptr, 0, d.in_n, 2, d.r2r, gptr<cpx<T>>(d.tw)};
    for (int m = (int)threadIdx.x; m < M; m += kThreads) {
      R2RSlot<T> sl;
      const cpx<T> w = g.weight(m, sl.idx);
      sl.wx = w.x;
      sl.wy = w.y;
      sl.pad = 0;
      slots[m] = sl;
    }
  }
  for (;;) {
    wp_commit<WP>(r, d, ti, smem, lc_in);
    __syncthreads();
    const int next = xcd_tile(blockIdx.x, gridDim.x, ++k, d.tiles);
    const TileIdx tn = next >= 0 ? tile_index(d, next) : ti;
    if (next >= 0) wp_fetch<WP>(r, d, in, tn, lc_in);  // in flight during the transform
    wp_transform<T, M, KIND, E>(d, ti, smem, ltw, slots);
    __syncthreads();
    if (d.has_fix) wp_store<T, M, KIND, E, true>(d, out, ti, smem, lpost, lc_out);
    else wp_store<T, M, KIND, E, false>(d, out, ti, smem, lpost, lc_out);
    if (next < 0) return;
    __syncthreads();  // the stores' LDS reads are done before the next commit
    ti = tn;
  }
}

}  // namespace fm
