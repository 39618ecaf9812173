// Device code of the Fourier-convolution solver for gfx950.
//
// Every step of a solve is one "line pass" (fm_pass.h): a workgroup loads a tile of B
// lines with coalesced accesses into LDS, builds the FFT inputs in registers (zero
// padding of unbounded directions, symmetric extension and pre-twiddle for DCT/DST,
// two real lines packed into one complex line), runs a mixed-radix Stockham FFT in LDS,
// and writes the post-processed lines into the next layout (transposed), again
// coalesced.  Pass 3 fuses the forward transform of the last axis, the multiplication
// by the Green's spectrum (or by the Green's spectrum times the spectral curl) and the
// inverse transform.  Twiddle tables and the Green's spectrum are generated in FP64.
#include <hip/hip_runtime.h>

#include "fm_pass.h"

namespace fm {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by S*i (S = +1 or -1)
template <int S, typename T>
__device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return S > 0 ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// ---------------------------------------------------------------------------------
// Small DFTs: v[q] <- sum_r v[r] exp(S 2 pi i r q / R)
// ---------------------------------------------------------------------------------
template <int R, int S, typename T>
struct SmallDft;

template <int S, typename T>
struct SmallDft<2, S, T> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int S, typename T>
struct SmallDft<4, S, T> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    const cpx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cpx<T> t2 = cadd(v[1], v[3]), t3 = mul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <int S, typename T>
struct SmallDft<8, S, T> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    SmallDft<4, S, T>::run(e);
    SmallDft<4, S, T>::run(o);
    const T c = T(0.70710678118654752440);
    // o[q] *= exp(S 2 pi i q / 8)
    const cpx<T> o1 = {c * (o[1].x - S * o[1].y), c * (S * o[1].x + o[1].y)};
    const cpx<T> o2 = mul_si<S>(o[2]);
    const cpx<T> o3 = {c * (-o[3].x - S * o[3].y), c * (S * o[3].x - o[3].y)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// odd radices: pair r with R - r
template <int R>
struct OddRoots;
template <>
struct OddRoots<3> {
  static constexpr double c[1] = {-0.5};
  static constexpr double s[1] = {0.86602540378443864676};
};
template <>
struct OddRoots<5> {
  static constexpr double c[2] = {0.30901699437494742410, -0.80901699437494742410};
  static constexpr double s[2] = {0.95105651629515357212, 0.58778525229247312917};
};
template <>
struct OddRoots<7> {
  static constexpr double c[3] = {0.62348980185873353053, -0.22252093395631440429,
                                  -0.90096886790241912624};
  static constexpr double s[3] = {0.78183148246802980871, 0.97492791218182360702,
                                  0.43388373911755812048};
};

template <int R, int S, typename T>
struct OddDft {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    constexpr int H = (R - 1) / 2;
    cpx<T> a[H], d[H];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      a[r - 1] = cadd(v[r], v[R - r]);
      d[r - 1] = csub(v[r], v[R - r]);
    }
    cpx<T> out[R];
    cpx<T> s0 = v[0];
#pragma unroll
    for (int r = 0; r < H; ++r) s0 = cadd(s0, a[r]);
    out[0] = s0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      cpx<T> re = v[0], im = {T(0), T(0)};
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        const int e = (r * q) % R;  // angle index; cos even, sin odd in e
        const int ee = e <= H ? e : R - e;
        const T cc = T(OddRoots<R>::c[ee - 1]);
        const T ss = T(e <= H ? OddRoots<R>::s[ee - 1] : -OddRoots<R>::s[ee - 1]);
        re.x += cc * a[r - 1].x;
        re.y += cc * a[r - 1].y;
        im.x += ss * d[r - 1].x;
        im.y += ss * d[r - 1].y;
      }
      // out[q] = re + S i im, out[R-q] = re - S i im
      const cpx<T> sim = mul_si<S>(im);
      out[q] = cadd(re, sim);
      out[R - q] = csub(re, sim);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = out[q];
  }
};
template <int S, typename T>
struct SmallDft<3, S, T> : OddDft<3, S, T> {};
template <int S, typename T>
struct SmallDft<5, S, T> : OddDft<5, S, T> {};
template <int S, typename T>
struct SmallDft<7, S, T> : OddDft<7, S, T> {};

// ---------------------------------------------------------------------------------
// One Stockham radix-R stage over F lines of length M held in LDS (line stride ls).
// Butterfly t of a line reads x[t + r M/R], twiddles by W_{Ns R}^{(t mod Ns) r}, and
// writes to (t - t mod Ns) R + t mod Ns + q Ns.  The first stage reads through
// `load` (the gather), later stages read LDS.
// ---------------------------------------------------------------------------------
template <typename T, int R, int S, class Load>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, int ls, int F, int M, int Ns,
                                          const cpx<T>* __restrict__ tw, Load& load) {
  constexpr int NB = (kElems + R - 1) / R;
  cpx<T> v[NB][R];
  int lin[NB], tt[NB];
  const int MR = M / R;
  const int total = F * MR;
  const int twstep = 4 * (MR / Ns);  // 4M table: W_{Ns R}^e = tw[4 e M / (Ns R)]
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int u = (int)threadIdx.x + i * kThreads;
    lin[i] = -1;
    tt[i] = 0;
    if (u < total) {
      const int line = u / MR;
      const int t = u - line * MR;
      const int k = t % Ns;
      lin[i] = line;
      tt[i] = t;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cpx<T> a = load(line, t + r * MR);
        if (r > 0 && k > 0) {
          cpx<T> w = tw[k * r * twstep];
          if (S > 0) w.y = -w.y;
          a = cmul(a, w);
        }
        v[i][r] = a;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (lin[i] >= 0) {
      SmallDft<R, S, T>::run(v[i]);
      const int t = tt[i];
      const int k = t % Ns;
      const int base = lin[i] * ls + (t - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[base + q * Ns] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename T, int S, class Load>
__device__ __forceinline__ void fft_stage_dispatch(int R, cpx<T>* buf, int ls, int F, int M,
                                                   int Ns, const cpx<T>* tw, Load& load) {
  switch (R) {
    case 8: fft_stage<T, 8, S>(buf, ls, F, M, Ns, tw, load); break;
    case 4: fft_stage<T, 4, S>(buf, ls, F, M, Ns, tw, load); break;
    case 2: fft_stage<T, 2, S>(buf, ls, F, M, Ns, tw, load); break;
    case 3: fft_stage<T, 3, S>(buf, ls, F, M, Ns, tw, load); break;
    case 5: fft_stage<T, 5, S>(buf, ls, F, M, Ns, tw, load); break;
    case 7: fft_stage<T, 7, S>(buf, ls, F, M, Ns, tw, load); break;
    default: break;
  }
}

// Full FFT of F lines; result in buf in natural order.
template <typename T, int S, class Load>
__device__ void fft_lines(cpx<T>* buf, int ls, int F, const PassDesc& d, const cpx<T>* tw,
                          Load& load0) {
  auto lds = [buf, ls](int line, int idx) { return buf[line * ls + idx]; };
  int Ns = 1;
  for (int s = 0; s < d.nstages; ++s) {
    const int R = d.radix[s];
    if (s == 0) fft_stage_dispatch<T, S>(R, buf, ls, F, d.M, Ns, tw, load0);
    else fft_stage_dispatch<T, S>(R, buf, ls, F, d.M, Ns, tw, lds);
    Ns *= R;
  }
}

// ---------------------------------------------------------------------------------
// Gathers: value of slot m of FFT line f, from the raw tile in LDS.
// ---------------------------------------------------------------------------------
template <typename T>
struct GatherCplx {  // complex lines, zero padded beyond n_data
  const cpx<T>* raw;
  int rs, n_data;
  __device__ cpx<T> operator()(int f, int m) const {
    return m < n_data ? raw[f * rs + m] : cpx<T>{T(0), T(0)};
  }
};

template <typename T>
struct GatherReal2 {  // two real lines packed as re + i im, zero padded
  const T* raw;
  int rs, n_data, nl;
  __device__ cpx<T> operator()(int f, int m) const {
    if (m >= n_data) return {T(0), T(0)};
    const int l = 2 * f;
    const T a = raw[l * rs + m];
    const T b = (l + 1 < nl) ? raw[(l + 1) * rs + m] : T(0);
    return {a, b};
  }
};

template <typename T>
struct GatherHerm2 {  // two Hermitian half-spectra -> one full spectrum
  const cpx<T>* raw;
  int rs, M, nl;
  __device__ cpx<T> operator()(int f, int m) const {
    const int l = 2 * f;
    const bool hi = 2 * m > M;
    const int mm = hi ? M - m : m;
    cpx<T> x1 = raw[l * rs + mm];
    cpx<T> x2 = (l + 1 < nl) ? raw[(l + 1) * rs + mm] : cpx<T>{T(0), T(0)};
    if (mm == 0 || 2 * mm == M) {  // modes that are real for real data
      x1.y = T(0);
      x2.y = T(0);
    }
    if (!hi) return {x1.x - x2.y, x1.y + x2.x};   // X1 + i X2
    return {x1.x + x2.y, -x1.y + x2.x};           // conj(X1) + i conj(X2)
  }
};

template <typename T>
__device__ __forceinline__ int r2r_weight(const R2R& r, int p) {
  return p == r.plo ? r.wlo : (p == r.phi ? r.whi : 2);
}

template <typename T>
struct GatherR2R {  // symmetric extension of two real lines, with pre-twiddle
  const T* raw;
  int rs, in_n, nl;
  R2R r;
  const cpx<T>* tw;  // 4M table
  __device__ cpx<T> operator()(int f, int m) const {
    const int M = 2 * r.nh;
    const int l = 2 * f;
    const T eps = r.b2 ? T(-1) : T(1);          // wrap factor of a full period
    const T sigma = r.sin ? -eps : eps;          // sign of the mirrored sample
    T re = T(0), im = T(0);
    auto add = [&](int p, T coef) {
      if (p < r.plo || p > r.phi) return;
      const int j = r.in_rev ? r.in_base - p : p - r.in_base;
      if (j < 0 || j >= in_n) return;
      const T c = coef * T(r2r_weight<T>(r, p)) * T(0.5);
      re += c * raw[l * rs + j];
      if (l + 1 < nl) im += c * raw[(l + 1) * rs + j];
    };
    if (r.a2 == 0) {
      if (m == 0) add(0, T(1) + sigma * eps);
      else if (m == r.nh) add(r.nh, T(1) + sigma);
      else if (m < r.nh) add(m, T(1));
      else add(M - m, sigma);
    } else {
      if (m < r.nh) add(m, T(1));
      else add(M - 1 - m, sigma);
    }
    cpx<T> z = {re, im};
    if (r.b2) z = cmul(z, tw[2 * m]);  // exp(-i pi m b / nh), b = 1/2
    return z;
  }
};

// ---------------------------------------------------------------------------------
// Scatters: value of output element j of tile line l, from the FFT buffer.
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T scatter_r2r(const cpx<T>* buf, int ls, const R2R& r,
                                         const cpx<T>* tw, int l, int j) {
  const int q = r.out_rev ? r.out_base - j : j + r.out_base;
  if (q < r.qlo || q > r.qhi) return T(0);
  cpx<T> Y = buf[(l >> 1) * ls + q];
  if (r.a2) Y = cmul(Y, tw[2 * q + r.b2]);  // exp(-i pi a (q + b) / nh), a = 1/2
  if (!r.sin) return (l & 1) ? Y.y : Y.x;
  return (l & 1) ? Y.x : -Y.y;
}

// ---------------------------------------------------------------------------------
// Coalesced tile load / store
// ---------------------------------------------------------------------------------
template <typename E>
__device__ __forceinline__ void load_tile(const E* __restrict__ in, int64_t s_line, int64_t s_b,
                                          int nl, int n, E* raw, int rs) {
  const int total = nl * n;
  if (s_line == 1) {
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int l = e / n, i = e - l * n;
      raw[l * rs + i] = in[l * s_b + i];
    }
  } else {
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int i = e / nl, l = e - i * nl;
      raw[l * rs + i] = in[l * s_b + (int64_t)i * s_line];
    }
  }
}

template <typename E, class Val>
__device__ __forceinline__ void store_tile(E* __restrict__ out, int64_t s_line, int64_t s_b,
                                           int nl, int n, Val& val) {
  const int total = nl * n;
  if (s_line == 1) {
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int l = e / n, j = e - l * n;
      out[l * s_b + j] = val(l, j);
    }
  } else {
    for (int e = threadIdx.x; e < total; e += kThreads) {
      const int j = e / nl, l = e - j * nl;
      out[l * s_b + (int64_t)j * s_line] = val(l, j);
    }
  }
}

// Store with the output conventions of the batch axes (last pass): `out` points at
// (c, b0); writes 0 on odd faces and duplicates index 0 to index last when asked.
template <typename E, class Val>
__device__ __forceinline__ void store_tile_fix(E* __restrict__ out, int64_t s_line, int64_t s_b,
                                               int64_t s_c, int nl, int n, int b0, int c,
                                               const Fixup& fx, Val& val) {
  const bool czero = (fx.c_zero_lo && c == 0) || (fx.c_zero_hi && c == fx.c_last);
  const bool cdup = fx.c_dup && c == 0;
  const int total = nl * n;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    int l, j;
    if (s_line == 1) {
      l = e / n;
      j = e - l * n;
    } else {
      j = e / nl;
      l = e - j * nl;
    }
    const int b = b0 + l;
    E v = val(l, j);
    if (czero || (fx.b_zero_lo && b == 0) || (fx.b_zero_hi && b == fx.b_last)) v = E{};
    const int64_t o = l * s_b + (int64_t)j * s_line;
    out[o] = v;
    const bool bdup = fx.b_dup && b == 0;
    if (bdup) out[o + (int64_t)fx.b_last * s_b] = v;
    if (cdup) {
      out[o + (int64_t)fx.c_last * s_c] = v;
      if (bdup) out[o + (int64_t)fx.b_last * s_b + (int64_t)fx.c_last * s_c] = v;
    }
  }
}

__device__ __forceinline__ int fold_index(int k, int M) {
  if (M == 0) return k;
  const int r = M - k;
  return k < r ? k : r;
}

__device__ __forceinline__ double signed_wave(int k, int M, double dw) {
  // wavenumber of DFT mode k of length M; the Nyquist mode differentiates to 0
  if (2 * k == M) return 0.0;
  const int ks = (2 * k > M) ? k - M : k;
  return dw * (double)ks;
}

// ---------------------------------------------------------------------------------
// Plain pass on one tile
// ---------------------------------------------------------------------------------
template <typename T>
__device__ void plain_tile(const PassDesc& d, int tile, char* smem) {
  const int nbt = (d.nb + d.B - 1) / d.B;
  int t = tile;
  const int bt = t % nbt;
  t /= nbt;
  const int c = t % d.nc;
  const int comp = t / d.nc;
  const int b0 = bt * d.B;
  const int nl = min(d.B, d.nb - b0);
  const cpx<T>* tw = reinterpret_cast<const cpx<T>*>(d.tw);
  const int M = d.M;
  const int ls = M + 1;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);
  const int64_t in_off = comp * d.in_s_comp + c * d.in_s_c + b0 * d.in_s_b;
  const int64_t out_off = comp * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
  const int rs = d.in_n + 1;

  // 1) load the tile's lines
  if (d.in_cplx) {
    load_tile(reinterpret_cast<const cpx<T>*>(d.in) + in_off, d.in_s_line, d.in_s_b, nl, d.in_n,
              reinterpret_cast<cpx<T>*>(smem), rs);
  } else {
    load_tile(reinterpret_cast<const T*>(d.in) + in_off, d.in_s_line, d.in_s_b, nl, d.in_n,
              reinterpret_cast<T*>(smem), rs);
  }
  __syncthreads();

  // 2) FFT (first stage gathers from the raw tile, which aliases the FFT buffer)
  const int F = (d.gather == G_CPLX) ? nl : (nl + 1) / 2;
  if (d.gather == G_CPLX) {
    GatherCplx<T> g{reinterpret_cast<const cpx<T>*>(smem), rs, d.n_data};
    if (d.sign < 0) fft_lines<T, -1>(buf, ls, F, d, tw, g);
    else fft_lines<T, +1>(buf, ls, F, d, tw, g);
  } else if (d.gather == G_REAL2) {
    GatherReal2<T> g{reinterpret_cast<const T*>(smem), rs, d.n_data, nl};
    fft_lines<T, -1>(buf, ls, F, d, tw, g);
  } else if (d.gather == G_HERM2) {
    GatherHerm2<T> g{reinterpret_cast<const cpx<T>*>(smem), rs, M, nl};
    fft_lines<T, +1>(buf, ls, F, d, tw, g);
  } else {
    GatherR2R<T> g{reinterpret_cast<const T*>(smem), rs, d.in_n, nl, d.r2r, tw};
    fft_lines<T, -1>(buf, ls, F, d, tw, g);
  }

  // 3) write the lines into the output layout
  if (d.scatter == S_CPLX) {
    auto val = [&](int l, int j) { return buf[l * ls + (j < M ? j : j - M)]; };
    store_tile(reinterpret_cast<cpx<T>*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
  } else if (d.scatter == S_R2C2) {
    auto val = [&](int l, int k) {
      const cpx<T>* z = buf + (l >> 1) * ls;
      const cpx<T> zk = z[k], zm = z[k == 0 ? 0 : M - k];
      if (l & 1) return cpx<T>{T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
      return cpx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    };
    store_tile(reinterpret_cast<cpx<T>*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
  } else if (d.scatter == S_REAL2) {
    auto val = [&](int l, int j) {
      const cpx<T> z = buf[(l >> 1) * ls + (j < M ? j : j - M)];
      return (l & 1) ? z.y : z.x;
    };
    if (d.has_fix)
      store_tile_fix(reinterpret_cast<T*>(d.out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c, nl,
                     d.out_n, b0, c, d.fix, val);
    else
      store_tile(reinterpret_cast<T*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
  } else {
    auto val = [&](int l, int j) { return scatter_r2r<T>(buf, ls, d.r2r, tw, l, j); };
    if (d.has_fix)
      store_tile_fix(reinterpret_cast<T*>(d.out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c, nl,
                     d.out_n, b0, c, d.fix, val);
    else
      store_tile(reinterpret_cast<T*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
  }
}

// ---------------------------------------------------------------------------------
// Fused pass 3 on one tile: forward FFT, spectral multiply, inverse FFT.
// ---------------------------------------------------------------------------------
template <typename T>
__device__ void fused_tile(const PassDesc& d, int tile, char* smem) {
  const int nbt = (d.nb + d.B - 1) / d.B;
  int t = tile;
  const int bt = t % nbt;
  t /= nbt;
  const int c = t % d.nc;
  const int comp = t / d.nc;  // curl: always 0, all three components in the tile
  const int b0 = bt * d.B;
  const int nl = min(d.B, d.nb - b0);
  const cpx<T>* tw = reinterpret_cast<const cpx<T>*>(d.tw);
  const int M = d.M;
  const int ls = M + 1;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);
  const int rs = d.in_n + 1;
  const int ncl = d.g.curl ? 3 : 1;   // components held by the tile
  const T* G = reinterpret_cast<const T*>(d.g.G);
  const int fc = fold_index(c, d.g.fold_c);

  if (d.gather == G_R2R) {
    // ---- all-real-to-real problem: forward R2R -> spectrum in LDS -> inverse R2R
    const int64_t in_off = comp * d.in_s_comp + c * d.in_s_c + b0 * d.in_s_b;
    load_tile(reinterpret_cast<const T*>(d.in) + in_off, d.in_s_line, d.in_s_b, nl, d.in_n,
              reinterpret_cast<T*>(smem), rs);
    __syncthreads();
    const int F = (nl + 1) / 2;
    {
      GatherR2R<T> g{reinterpret_cast<const T*>(smem), rs, d.in_n, nl, d.r2r, tw};
      fft_lines<T, -1>(buf, ls, F, d, tw, g);
    }
    // spectrum (real) into its own LDS region, times the Green's spectrum
    const int ss = d.spec_n + 1;
    T* spec = reinterpret_cast<T*>(smem + (size_t)F * ls * sizeof(cpx<T>));
    for (int e = threadIdx.x; e < nl * d.spec_n; e += kThreads) {
      const int l = e / d.spec_n, j = e - l * d.spec_n;
      const T g = G[((int64_t)fc * d.g.F_b + fold_index(b0 + l, d.g.fold_b)) * d.g.F_line +
                    fold_index(j, d.g.fold_line)];
      spec[l * ss + j] = g * scatter_r2r<T>(buf, ls, d.r2r, tw, l, j);
    }
    __syncthreads();
    {
      GatherR2R<T> g{spec, ss, d.spec_n, nl, d.r2r2, tw};
      fft_lines<T, -1>(buf, ls, F, d, tw, g);
    }
    const int64_t out_off = comp * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
    auto val = [&](int l, int j) { return scatter_r2r<T>(buf, ls, d.r2r2, tw, l, j); };
    store_tile(reinterpret_cast<T*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
    return;
  }

  if (d.gather == G_REAL2) {
    // ---- only DFT axis of the problem: two real lines per FFT; the Green's spectrum
    // is real and even, so the product keeps the two lines separable
    const int64_t in_off = comp * d.in_s_comp + c * d.in_s_c + b0 * d.in_s_b;
    load_tile(reinterpret_cast<const T*>(d.in) + in_off, d.in_s_line, d.in_s_b, nl, d.in_n,
              reinterpret_cast<T*>(smem), rs);
    __syncthreads();
    const int F = (nl + 1) / 2;
    GatherReal2<T> g{reinterpret_cast<const T*>(smem), rs, d.n_data, nl};
    fft_lines<T, -1>(buf, ls, F, d, tw, g);
    // The two packed lines have their own Green rows: split Z into the two Hermitian
    // spectra X1 = (Z_k + conj Z_{M-k})/2, X2 = (Z_k - conj Z_{M-k})/(2i), scale each
    // by its (real, even) row, and pack again as Y1 + i Y2.  One thread owns the pair
    // (k, M-k).
    const int H = M / 2 + 1;
    for (int e = threadIdx.x; e < F * H; e += kThreads) {
      const int f = e / H, k = e - f * H;
      const int kk = fold_index(k, d.g.fold_line);
      const int l0 = 2 * f, l1 = min(2 * f + 1, nl - 1);
      const T g0 = G[((int64_t)fc * d.g.F_b + fold_index(b0 + l0, d.g.fold_b)) * d.g.F_line + kk];
      const T g1 = G[((int64_t)fc * d.g.F_b + fold_index(b0 + l1, d.g.fold_b)) * d.g.F_line + kk];
      const int km = (k == 0) ? 0 : M - k;
      const cpx<T> zk = buf[f * ls + k], zm = buf[f * ls + km];
      const cpx<T> x1 = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
      const cpx<T> x2 = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
      // Z'_k = g0 X1 + i g1 X2 ;  Z'_{M-k} = g0 conj(X1) + i g1 conj(X2)
      buf[f * ls + k] = {g0 * x1.x - g1 * x2.y, g0 * x1.y + g1 * x2.x};
      if (km != k) buf[f * ls + km] = {g0 * x1.x + g1 * x2.y, -g0 * x1.y + g1 * x2.x};
    }
    __syncthreads();
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + idx]; };
    fft_lines<T, +1>(buf, ls, F, d, tw, lds);
    const int64_t out_off = comp * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
    auto val = [&](int l, int j) {
      const cpx<T> z = buf[(l >> 1) * ls + (j < M ? j : j - M)];
      return (l & 1) ? z.y : z.x;
    };
    store_tile(reinterpret_cast<T*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
    return;
  }

  // ---- complex lines (C2C along the last axis), one or three components
  for (int q = 0; q < ncl; ++q) {
    const int cc = d.g.curl ? q : comp;
    const int64_t in_off = cc * d.in_s_comp + c * d.in_s_c + b0 * d.in_s_b;
    load_tile(reinterpret_cast<const cpx<T>*>(d.in) + in_off, d.in_s_line, d.in_s_b, nl, d.in_n,
              reinterpret_cast<cpx<T>*>(smem) + (size_t)q * nl * rs, rs);
  }
  __syncthreads();
  const int F = ncl * nl;
  {
    GatherCplx<T> g{reinterpret_cast<const cpx<T>*>(smem), rs, d.n_data};
    fft_lines<T, -1>(buf, ls, F, d, tw, g);
  }
  if (!d.g.curl) {
    for (int e = threadIdx.x; e < nl * M; e += kThreads) {
      const int l = e / M, k = e - l * M;
      const T g = G[((int64_t)fc * d.g.F_b + fold_index(b0 + l, d.g.fold_b)) * d.g.F_line +
                    fold_index(k, d.g.fold_line)];
      cpx<T> z = buf[l * ls + k];
      z.x *= g;
      z.y *= g;
      buf[l * ls + k] = z;
    }
  } else {
    const double wc = signed_wave(c, d.g.M_c, d.g.dw_c);
    for (int e = threadIdx.x; e < nl * M; e += kThreads) {
      const int l = e / M, k = e - l * M;
      const T g = G[((int64_t)fc * d.g.F_b + fold_index(b0 + l, d.g.fold_b)) * d.g.F_line +
                    fold_index(k, d.g.fold_line)];
      double w[3];
      w[d.g.axis_line] = signed_wave(k, d.g.M_line, d.g.dw_line);
      w[d.g.axis_b] = signed_wave(b0 + l, d.g.M_b, d.g.dw_b);
      w[d.g.axis_c] = wc;
      const T wx = T(w[0]), wy = T(w[1]), wz = T(w[2]);
      const cpx<T> fx = buf[(0 * nl + l) * ls + k];
      const cpx<T> fy = buf[(1 * nl + l) * ls + k];
      const cpx<T> fz = buf[(2 * nl + l) * ls + k];
      // u_hat = G * i (w x f_hat)
      const cpx<T> cx = {wy * fz.x - wz * fy.x, wy * fz.y - wz * fy.y};
      const cpx<T> cy = {wz * fx.x - wx * fz.x, wz * fx.y - wx * fz.y};
      const cpx<T> cz = {wx * fy.x - wy * fx.x, wx * fy.y - wy * fx.y};
      buf[(0 * nl + l) * ls + k] = {-g * cx.y, g * cx.x};
      buf[(1 * nl + l) * ls + k] = {-g * cy.y, g * cy.x};
      buf[(2 * nl + l) * ls + k] = {-g * cz.y, g * cz.x};
    }
  }
  __syncthreads();
  {
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + idx]; };
    fft_lines<T, +1>(buf, ls, F, d, tw, lds);
  }
  for (int q = 0; q < ncl; ++q) {
    const int cc = d.g.curl ? q : comp;
    const int64_t out_off = cc * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
    const cpx<T>* z = buf + (size_t)q * nl * ls;
    auto val = [&](int l, int j) { return z[l * ls + (j < M ? j : j - M)]; };
    store_tile(reinterpret_cast<cpx<T>*>(d.out) + out_off, d.out_s_line, d.out_s_b, nl, d.out_n, val);
  }
}

template <typename T>
__device__ __forceinline__ void run_tile(const PassDesc& d, int tile, char* smem) {
  if (d.fused) fused_tile<T>(d, tile, smem);
  else plain_tile<T>(d, tile, smem);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassDesc d) {
  extern __shared__ __align__(16) char smem[];
  run_tile<T>(d, blockIdx.x, smem);
}

// Batched form: tiles of many descriptors in one launch; prefix[i] = first tile of
// descriptor i, prefix[n] = total.
template <typename T>
__global__ __launch_bounds__(kThreads) void pass_kernel_batched(const PassDesc* __restrict__ ds,
                                                                const int* __restrict__ prefix,
                                                                int n) {
  extern __shared__ __align__(16) char smem[];
  const int tile = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  const PassDesc d = ds[lo];
  run_tile<T>(d, tile - prefix[lo], smem);
}

// ---------------------------------------------------------------------------------
// FP64 generation: twiddles, Green's spectrum samples, finalisation
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void twiddle_kernel(cpx<T>* out, int M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 4 * M) return;
  double s, c;
  sincospi((double)j / (2.0 * (double)M), &s, &c);  // angle 2 pi j / (4 M)
  out[j] = {T(c), T(-s)};
}

// K_nu(x) for nu = 0, 1 from K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt: the
// trapezoidal rule on this doubly-exponentially decaying analytic integrand converges
// geometrically (step 0.1 gives full double precision for the x used here); for large
// x the asymptotic expansion sqrt(pi/2x) e^-x sum_k a_k(nu) / x^k is used instead.
__device__ double bessel_k(int nu, double x) {
  if (x >= 25.0) {
    const double mu = 4.0 * nu * nu;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k <= 30; ++k) {
      term *= (mu - (2.0 * k - 1.0) * (2.0 * k - 1.0)) / (k * 8.0 * x);
      sum += term;
      if (fabs(term) < 1e-17 * fabs(sum)) break;
    }
    return sqrt(3.14159265358979323846 / (2.0 * x)) * exp(-x) * sum;
  }
  const double h = 0.1;
  // terms scaled by exp(x) to avoid underflow for larger x
  double sum = 0.5;  // t = 0: exp(-x (cosh 0 - 1)) cosh(0) = 1, half weight
  for (int j = 1; j < 2000; ++j) {
    const double tj = j * h;
    const double ch = cosh(tj);
    const double ex = x * (ch - 1.0);
    if (ex > 45.0 + tj) break;
    sum += exp(-ex) * (nu ? ch : 1.0);
  }
  return h * sum * exp(-x);
}



__device__ double green_value(const GreenGen& g, double rho, double k) {
  const double pi = 3.14159265358979323846;
  if (g.du == 3) {
    if (rho > 0.0) return -1.0 / (4.0 * pi * rho);
    const double s = -3.0 / (8.0 * pi * g.r_eq);
    return g.variant == 0 ? s * g.cellvol : s;
  }
  if (g.du == 2) {
    if (k == 0.0) {
      if (rho > 0.0) return log(rho) / (2.0 * pi);
      return (pi - 6.0 + 2.0 * log(pi * g.r_eq * g.r_eq / 2.0)) / (8.0 * pi);
    }
    if (rho > 0.0) return -bessel_k(0, k * rho) / (2.0 * pi);
    const double x = k * g.r_eq;
    return -(1.0 - x * bessel_k(1, x)) / (pi * x * x);
  }
  if (g.du == 1) {
    if (k == 0.0) return 0.5 * rho;
    return -exp(-k * rho) / (2.0 * k);
  }
  return k == 0.0 ? 0.0 : -1.0 / (k * k);
}

__global__ void green_sample_kernel(double* S, GreenGen g) {
  const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int idx[3];
  int64_t r = e;
  idx[2] = (int)(r % g.n[2]);
  r /= g.n[2];
  idx[1] = (int)(r % g.n[1]);
  idx[0] = (int)(r / g.n[1]);
  double r2 = 0.0, k2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (g.unb[a]) {
      const double dd = idx[a] * g.h[a];
      r2 += dd * dd;
    } else {
      const double w = g.dw[a] * (idx[a] + g.shift[a]);
      k2 += w * w;
    }
  }
  S[e] = green_value(g, sqrt(r2), sqrt(k2));
}

// table[f] = scale * S[f + off] (per axis offsets), converted to T
template <typename T>
__global__ void green_final_kernel(T* G, const double* S, int F0, int F1, int F2, int n1, int n2,
                                   int o0, int o1, int o2, double scale) {
  const int64_t total = (int64_t)F0 * F1 * F2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int64_t r = e;
  const int f2 = (int)(r % F2);
  r /= F2;
  const int f1 = (int)(r % F1);
  const int f0 = (int)(r / F1);
  const int64_t s = ((int64_t)(f0 + o0) * n1 + (f1 + o1)) * n2 + (f2 + o2);
  G[e] = T(scale * S[s]);
}

}  // namespace fm

// ---------------------------------------------------------------------------------
// Host launchers (internal to the library)
// ---------------------------------------------------------------------------------
namespace fm {

// Allow the pass kernels the full LDS of a gfx950 workgroup (set once per process).
template <typename T>
hipError_t allow_full_lds() {
  static hipError_t once = [] {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_kernel<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&pass_kernel_batched<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
  }();
  return once;
}

template <typename T>
hipError_t launch_pass(const PassDesc& d, hipStream_t st) {
  if (d.tiles <= 0) return hipSuccess;
  if (d.lds_bytes > kSoftLds) {
    const hipError_t e = allow_full_lds<T>();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(pass_kernel<T>, dim3(d.tiles), dim3(kThreads), d.lds_bytes, st, d);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_batched(const PassDesc* ds, const int* prefix, int n, int total_tiles,
                               int lds_bytes, hipStream_t st) {
  if (total_tiles <= 0) return hipSuccess;
  if (lds_bytes > kSoftLds) {
    const hipError_t e = allow_full_lds<T>();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(pass_kernel_batched<T>, dim3(total_tiles), dim3(kThreads), lds_bytes, st, ds,
                     prefix, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_twiddles(void* out, int M, hipStream_t st) {
  const int n = 4 * M;
  hipLaunchKernelGGL(twiddle_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<cpx<T>*>(out), M);
  return hipGetLastError();
}

hipError_t launch_green_sample(double* S, const GreenGen& g, hipStream_t st) {
  const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
  hipLaunchKernelGGL(green_sample_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     S, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_green_final(void* G, const double* S, const int F[3], const int n[3],
                              const int off[3], double scale, hipStream_t st) {
  const int64_t total = (int64_t)F[0] * F[1] * F[2];
  hipLaunchKernelGGL(green_final_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     st, reinterpret_cast<T*>(G), S, F[0], F[1], F[2], n[1], n[2], off[0], off[1],
                     off[2], scale);
  return hipGetLastError();
}

template hipError_t launch_pass<float>(const PassDesc&, hipStream_t);
template hipError_t launch_pass<double>(const PassDesc&, hipStream_t);
template hipError_t launch_pass_batched<float>(const PassDesc*, const int*, int, int, int, hipStream_t);
template hipError_t launch_pass_batched<double>(const PassDesc*, const int*, int, int, int, hipStream_t);
template hipError_t launch_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_green_final<float>(void*, const double*, const int*, const int*, const int*, double, hipStream_t);
template hipError_t launch_green_final<double>(void*, const double*, const int*, const int*, const int*, double, hipStream_t);

}  // namespace fm
