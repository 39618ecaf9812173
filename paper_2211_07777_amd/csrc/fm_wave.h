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
template <typename T, int M, int E, int s, int S>
__device__ __forceinline__ void wave_stages(cpx<T> (&v)[E], int j, cpx<T>* buf, GTab<T> tw) {
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
      wave_stages<T, M, E, s + 1, S>(v, j, buf, tw);
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
  const GTab<T> tw = gptr<cpx<T>>(E == 16 ? d.wtw : d.wtw8);
  const int b = ti.b0 + l;
  const int comp0 = NCL == 3 ? 0 : ti.comp;
  const int64_t line_off = (int64_t)ti.c * d.in_s_c + (int64_t)b * d.in_s_b;

  // the Green's row of the line, folded: G[fold(k)] for k = j + P m (coalesced; the upper
  // half of a row reads the lower half again, from cache)
  const auto* G = gptr<T>(d.g.G);
  const int64_t grow = ((int64_t)fold_index(ti.c, d.g.fold_c) * d.g.F_b + fold_index(b, d.g.fold_b)) *
                       (int64_t)d.g.F_line;
  T g[E];
#pragma unroll
  for (int m = 0; m < E; ++m) g[m] = G[grow + fold_index(j + P * m, d.g.fold_line)];

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
    const T wc = curl_wave<T>(ti.c, d.g.dtab_c);
    const T wb = curl_wave<T>(b, d.g.dtab_b);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const T wl = curl_wave<T>(j + P * m, d.g.dtab_line);
      const T wx = d.g.axis_line == 0 ? wl : (d.g.axis_b == 0 ? wb : wc);
      const T wy = d.g.axis_line == 1 ? wl : (d.g.axis_b == 1 ? wb : wc);
      const T wz = d.g.axis_line == 2 ? wl : (d.g.axis_b == 2 ? wb : wc);
      const cpx<T> fx = v[0][m], fy = v[1][m], fz = v[2][m];
      // u_hat = G i (w x f_hat)
      const cpx<T> cx = {wy * fz.x - wz * fy.x, wy * fz.y - wz * fy.y};
      const cpx<T> cy = {wz * fx.x - wx * fz.x, wz * fx.y - wx * fz.y};
      const cpx<T> cz = {wx * fy.x - wy * fx.x, wx * fy.y - wy * fx.y};
      v[0][m] = {-g[m] * cx.y, g[m] * cx.x};
      v[1][m] = {-g[m] * cy.y, g[m] * cy.x};
      v[2][m] = {-g[m] * cz.y, g[m] * cz.x};
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
// Occupancy targets of the three-component (curl) kernels: 16 values per lane need the
// 256 VGPRs of two waves per SIMD; 8 FP32 values fit the 168 of three (FP64 would spill
// there and keeps the compiler's choice).
template <typename T, int KIND, int E>
constexpr int wave_min_waves() {
  return KIND == K_F_CURL ? (E == 16 ? 2 : (sizeof(T) == 4 ? 3 : 1)) : 1;
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
// FFT lines in registers with the schedule above: two workgroup barriers per tile
// instead of one per radix stage.  Four wavefronts of L = 64 / P FFT lines each; a
// packed kind (two real lines per FFT) holds 2 L tile lines per wavefront.  The raw
// lines of wavefront w sit inside the LDS region of its own FFT lines: all its raw
// values are read before its first exchange write, and no other wavefront touches the
// region until the next workgroup barrier.
// ---------------------------------------------------------------------------------
template <typename T, int M, int KIND, int E_>
struct WavePlain {
  static constexpr int E = E_;
  static constexpr int P = M / E;                         // lanes per FFT line
  static constexpr int L = 64 / P;                        // FFT lines per wavefront
  static constexpr int PK = gather_of(KIND) == G_CPLX ? 1 : 2;  // tile lines per FFT line
  static constexpr int RW = L * PK;                       // tile lines per wavefront
  static constexpr int LS = fft_line_stride(M);
  static constexpr bool CIN = in_cplx_of(KIND);
  using In = typename std::conditional<CIN, cpx<T>, T>::type;
  static constexpr int REGION = L * LS * (CIN ? 1 : 2);   // a wavefront's LDS, in In units
  static constexpr int U = KIND == K_R2C ? 2 * E : E + 1; // input values per thread
};

// Registers -> raw tile: tile line l at (l / RW) REGION + (l mod RW) rs.
template <class WP, class Stage>
__device__ __forceinline__ void commit_wave(const Stage& v, const PassDesc& d, const TileIdx& ti,
                                            char* smem) {
  using In = typename WP::In;
  const TileWalk w = in_walk(d, ti);
  In* raw = reinterpret_cast<In*>(smem);
  const int rs = d.wave_rs;
#pragma unroll
  for (int u = 0; u < WP::U; ++u) {
    int l, i;
    if (w.at((int)threadIdx.x + u * kThreads, l, i))
      raw[(l / WP::RW) * WP::REGION + (l % WP::RW) * rs + i] = v.get(u);
  }
}

template <typename T, int M, int KIND, int E>
__device__ __forceinline__ void wave_plain_tile(const PassDesc& d, const void* in, void* out,
                                                char* smem, int tile) {
  using WP = WavePlain<T, M, KIND, E>;
  using In = typename WP::In;
  constexpr int P = WP::P, L = WP::L, PK = WP::PK;
  constexpr int S = (KIND == K_C2C_I || KIND == K_C2R) ? +1 : -1;
  const TileIdx ti = tile_index(d, tile);
  {
    RegStage<T, In, WP::U> st;
    fetch<WP::U, 1, false, In>(st, d, in, ti);
    commit_wave<WP>(st, d, ti, smem);
  }
  __syncthreads();
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int j = lane % P, lf = lane / P;  // lane of the line, line of the wavefront
  const int f = wave * L + lf;            // FFT line of the tile
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);
  const GTab<T> tw4 = gptr<cpx<T>>(d.tw);
  if (f < (ti.nl + PK - 1) / PK) {
    const In* raw = reinterpret_cast<const In*>(smem) + wave * WP::REGION;
    const int nlw = ti.nl - wave * WP::RW;  // tile lines from the wavefront's first
    const int rs = d.wave_rs;
    cpx<T> v[E];
    if constexpr (gather_of(KIND) == G_CPLX) {
      const GatherCplx<T> g{raw, rs, d.n_data};
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = g(lf, j + P * m);
    } else if constexpr (gather_of(KIND) == G_REAL2) {
      const GatherReal2<T> g{raw, rs, d.n_data, nlw};
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = g(lf, j + P * m);
    } else if constexpr (gather_of(KIND) == G_HERM2) {
      const GatherHerm2<T> g{raw, rs, M, nlw};
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = g(lf, j + P * m);
    } else {
      const GatherR2R<T, GTab<T>> g{raw, rs, d.in_n, nlw, d.r2r, tw4};
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = g(lf, j + P * m);
    }
    cpx<T>* line = buf + (size_t)f * WP::LS;
    wave_stages<T, M, E, 0, S>(v, j, line, gptr<cpx<T>>(E == 16 ? d.wtw : d.wtw8));
    wave_lds_sync();  // the last exchange's reads are done
#pragma unroll
    for (int m = 0; m < E; ++m) line[pad16(j + P * m)] = v[m];
  }
  __syncthreads();
  plain_store<T, M, KIND>(d, out, ti, buf, tw4);
}

template <typename T, int M, int KIND, int E>
__global__ __launch_bounds__(kThreads) void wave_plain_kernel(const PassDesc* __restrict__ dp,
                                                              const void* in, void* out) {
  extern __shared__ __align__(16) char smem[];
  const PassDesc& d = *dp;
  for (int k = 0;; ++k) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, k, d.tiles);
    if (tile < 0) return;
    if (k > 0) __syncthreads();  // the previous tile's LDS reads are finished
    wave_plain_tile<T, M, KIND, E>(d, in, out, smem, tile);
  }
}

}  // namespace fm
