// Device templates of the Fourier-convolution solver for gfx950 (line passes).
//
// Every step of a solve is one "line pass" (fm_pass.h): a workgroup loads a tile of B
// lines with coalesced accesses into LDS, builds the FFT inputs in registers (zero
// padding of unbounded directions, symmetric extension and pre-twiddle for DCT/DST,
// two real lines packed into one complex line), runs a mixed-radix Stockham FFT in LDS,
// and writes the post-processed lines into the next layout (transposed), again
// coalesced.  Pass 3 fuses the forward transform of the last axis, the multiplication
// by the Green's spectrum (or by the Green's spectrum times the spectral curl) and the
// inverse transform.  Twiddle tables and the Green's spectrum are generated in FP64.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

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


// radix 16 = 4 x 4 with the inner twiddles W16^(n2 k1)
template <int S, typename T>
struct SmallDft<16, S, T> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    // cos / sin of 2 pi e / 16, e = 0..15
    constexpr double C[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                              0.38268343236508977173, 0.0, -0.38268343236508977173,
                              -0.70710678118654752440, -0.92387953251128675613, -1.0,
                              -0.92387953251128675613, -0.70710678118654752440,
                              -0.38268343236508977173, 0.0, 0.38268343236508977173,
                              0.70710678118654752440, 0.92387953251128675613};
    constexpr double Sn[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                               0.92387953251128675613, 1.0, 0.92387953251128675613,
                               0.70710678118654752440, 0.38268343236508977173, 0.0,
                               -0.38268343236508977173, -0.70710678118654752440,
                               -0.92387953251128675613, -1.0, -0.92387953251128675613,
                               -0.70710678118654752440, -0.38268343236508977173};
    cpx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cpx<T> col[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      SmallDft<4, S, T>::run(col);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) {
        const int e = n2 * k1;
        if (e == 0) {
          a[n2][k1] = col[k1];
        } else {
          const cpx<T> w = {T(C[e]), T(S * Sn[e])};
          a[n2][k1] = cmul(col[k1], w);
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cpx<T> row[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      SmallDft<4, S, T>::run(row);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = row[k2];
    }
  }
};

// radix 32 = 2 x 16: the DFTs of the even and the odd samples, joined with W32^k
template <int S, typename T>
struct SmallDft<32, S, T> {
  __device__ __forceinline__ static void run(cpx<T>* v) {
    // cos / sin of 2 pi k / 32, k = 0..15
    constexpr double C[16] = {1.0, 0.98078528040323044913, 0.92387953251128675613,
                              0.83146961230254523708, 0.70710678118654752440,
                              0.55557023301960222474, 0.38268343236508977173,
                              0.19509032201612826785, 0.0, -0.19509032201612826785,
                              -0.38268343236508977173, -0.55557023301960222474,
                              -0.70710678118654752440, -0.83146961230254523708,
                              -0.92387953251128675613, -0.98078528040323044913};
    constexpr double Sn[16] = {0.0, 0.19509032201612826785, 0.38268343236508977173,
                               0.55557023301960222474, 0.70710678118654752440,
                               0.83146961230254523708, 0.92387953251128675613,
                               0.98078528040323044913, 1.0, 0.98078528040323044913,
                               0.92387953251128675613, 0.83146961230254523708,
                               0.70710678118654752440, 0.55557023301960222474,
                               0.38268343236508977173, 0.19509032201612826785};
    cpx<T> e[16], o[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      e[m] = v[2 * m];
      o[m] = v[2 * m + 1];
    }
    SmallDft<16, S, T>::run(e);
    SmallDft<16, S, T>::run(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      cpx<T> t;
      if (k == 0) t = o[0];
      else if (k == 8) t = mul_si<S>(o[8]);
      else t = cmul(o[k], cpx<T>{T(C[k]), T(S * Sn[k])});
      v[k] = cadd(e[k], t);
      v[k + 16] = csub(e[k], t);
    }
  }
};

constexpr int gather_of(int k) {
  return (k == K_C2C_F || k == K_C2C_I || k == K_F_C2C || k == K_F_CURL) ? G_CPLX
         : (k == K_R2C || k == K_F_R2C)                                   ? G_REAL2
         : (k == K_C2R)                                                    ? G_HERM2
                                                                           : G_R2R;
}
constexpr int scatter_of(int k) {
  return k == K_C2C_F || k == K_C2C_I ? S_CPLX : k == K_R2C ? S_R2C2 : k == K_C2R ? S_REAL2 : S_R2R;
}
constexpr bool in_cplx_of(int k) {
  return k == K_C2C_F || k == K_C2C_I || k == K_C2R || k == K_F_C2C || k == K_F_CURL;
}
constexpr bool fused_of(int k) { return k >= K_F_C2C; }

// A table pointer of the descriptor as a global-memory pointer.  Descriptor pointers
// are generic; a generic load is a FLAT instruction, which counts against both the
// vector-memory and the LDS counters, so that every later LDS wait would also wait for
// it.  Global pointers give plain global loads.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const void* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}

// Twiddle tables are read through a pointer of type P: a generic pointer into LDS (the
// tables the persistent kernels stage) or a global-memory pointer (GTab).  Keeping the
// address space in the type makes the global reads plain global loads.
template <typename T>
using GTab = const __attribute__((address_space(1))) cpx<T>*;
template <typename T, class P>
__device__ __forceinline__ cpx<T> twid(P p, int i) {
  return cpx<T>{p[i].x, p[i].y};
}

// Position of FFT slot i in an LDS line (see fft_line_stride).
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Per-element loops over a tile take kChunk elements per thread at a time, so that
// their LDS reads are issued together.
constexpr int kChunk = 1;

// for e in [0, total) spread over the workgroup: v = ld(e) for a chunk of elements,
// then st(e, v) for the same chunk (all reads of a chunk precede its writes).
template <typename V, class Ld, class St>
__device__ __forceinline__ void chunked(int total, const Ld& ld, const St& st) {
  for (int e0 = threadIdx.x; e0 < total; e0 += kChunk * kThreads) {
    V v[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int e = e0 + u * kThreads;
      if (e < total) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int e = e0 + u * kThreads;
      if (e < total) st(e, v[u]);
    }
  }
}

template <typename T>
struct Prec {
  static constexpr int RMAX = max_radix((int)sizeof(T));
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint64_t mag) {
  return (uint32_t)(((uint64_t)n * mag) >> 32);
}

// ---------------------------------------------------------------------------------
// One Stockham radix-R stage over F lines of length M held in LDS (line stride ls).
// Butterfly t of a line reads x[t + r M/R], twiddles by W_{Ns R}^{(t mod Ns) r}, and
// writes to (t - t mod Ns) R + t mod Ns + q Ns.  The first stage reads through
// `load` (the gather), later stages read LDS.  Runtime-length form: twiddles from the
// 4M table; compile-time form: M, R, Ns are constants and twiddles come from the
// per-stage table (contiguous per butterfly).
// ---------------------------------------------------------------------------------
template <typename T, int EL, int R, int S, class P, class Load>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, int ls, int F, int M, int Ns, P tw,
                                          Load& load) {
  constexpr int NB = (EL + R - 1) / R;
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
          cpx<T> w = twid<T>(tw, k * r * twstep);
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
      const int base = (t - k) * R + k;
      cpx<T>* row = buf + lin[i] * ls;
#pragma unroll
      for (int q = 0; q < R; ++q) row[pad16(base + q * Ns)] = v[i][q];
    }
  }
  __syncthreads();
}

// Destination of the last stage's outputs: NoSink writes them to LDS (natural order);
// any other sink is called as sink(line, slot, value) for the kept slots instead.
struct NoSink {};

template <typename T, int M, int R, int Ns, int S, class P, class Load, class Sink>
__device__ __forceinline__ void fft_stage_ct(cpx<T>* buf, int ls, int F, P stw, Load& load,
                                             int keep, const Sink& sink) {
  constexpr int NB = (elems_per_thread((int)sizeof(T), M) + R - 1) / R;
  constexpr int MR = M / R;
  cpx<T> v[NB][R];
  int lin[NB], tt[NB];
  const int total = F * MR;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int u = (int)threadIdx.x + i * kThreads;
    lin[i] = -1;
    tt[i] = 0;
    if (u < total) {
      const int line = u / MR;
      const int t = u - line * MR;
      lin[i] = line;
      tt[i] = t;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = load(line, t + r * MR);
      if (Ns > 1) {
        const int k = t % Ns;
        const P w = stw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> ww = twid<T>(w, r - 1);
          if (S > 0) ww.y = -ww.y;
          v[i][r] = cmul(v[i][r], ww);
        }
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
      const int base = (t - k) * R + k;
      cpx<T>* row = buf + lin[i] * ls;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        // the last stage (Ns R = M) writes slot t + q Ns: only the first `keep` are read
        if constexpr (Ns * R == M && !std::is_same<Sink, NoSink>::value) {
          if (base + q * Ns < keep) sink(lin[i], base + q * Ns, v[i][q]);
        } else {
          if (Ns * R < M || base + q * Ns < keep) row[pad16(base + q * Ns)] = v[i][q];
        }
      }
    }
  }
  __syncthreads();
}

template <typename T, int M, int S, int s, int Ns, class P, class Load, class Sink>
__device__ __forceinline__ void stages_ct(cpx<T>* buf, int ls, int F, P stw, Load& load, int keep,
                                          const Sink& sink) {
  constexpr int R = radix_at(M, s, Prec<T>::RMAX);
  if constexpr (R != 0) {
    fft_stage_ct<T, M, R, Ns, S>(buf, ls, F, stw + stage_table_offset(M, s, Prec<T>::RMAX), load,
                                 keep, sink);
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + pad16(idx)]; };
    stages_ct<T, M, S, s + 1, Ns * R>(buf, ls, F, stw, lds, keep, sink);
  }
}

template <typename T, int EL, int S, class P, class Load>
__device__ __forceinline__ void fft_stage_dispatch(int R, cpx<T>* buf, int ls, int F, int M,
                                                   int Ns, P tw, Load& load) {
  switch (R) {
    case 8: fft_stage<T, EL, 8, S>(buf, ls, F, M, Ns, tw, load); break;
    case 4: fft_stage<T, EL, 4, S>(buf, ls, F, M, Ns, tw, load); break;
    case 2: fft_stage<T, EL, 2, S>(buf, ls, F, M, Ns, tw, load); break;
    case 3: fft_stage<T, EL, 3, S>(buf, ls, F, M, Ns, tw, load); break;
    case 5: fft_stage<T, EL, 5, S>(buf, ls, F, M, Ns, tw, load); break;
    case 7: fft_stage<T, EL, 7, S>(buf, ls, F, M, Ns, tw, load); break;
    default: break;
  }
}

// Full FFT of F lines; result in buf in natural order.  MC = compile-time length or 0.
// Compile-time lengths write only the first `keep` outputs of each line (the rest are
// cropped by the caller and never read).
template <typename T, int MC, int S, class P, class Load>
__device__ __forceinline__ void fft_lines(cpx<T>* buf, int ls, int F, const PassDesc& d, P stw,
                                          Load& load0, int keep = 1 << 30) {
  if constexpr (MC > 1) {
    stages_ct<T, MC, S, 0, 1>(buf, ls, F, stw, load0, keep, NoSink{});
  } else {
    constexpr int EL = elems_per_thread((int)sizeof(T), MC);
    const GTab<T> tw = gptr<cpx<T>>(d.tw);  // runtime lengths: the 4M table in global memory
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + pad16(idx)]; };
    int Ns = 1;
    for (int s = 0; s < d.nstages; ++s) {
      const int R = d.radix[s];
      if (s == 0) fft_stage_dispatch<T, EL, S>(R, buf, ls, F, d.M, Ns, tw, load0);
      else fft_stage_dispatch<T, EL, S>(R, buf, ls, F, d.M, Ns, tw, lds);
      Ns *= R;
    }
  }
}

// Twiddle tables seen by a tile: in LDS for persistent kernels (copied once per
// workgroup), else in global memory.
template <class P>
struct Tabs {
  P stw;  // stage twiddles of the compile-time length
  P tw;   // 4M table (persistent real-to-real kernels: its first 2M entries)
};

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

// GatherCplx and GatherReal2 reading contiguous input lines straight from global memory
// (p: the tile's first line, sb: the line stride in elements).
template <typename T>
struct GatherCplxG {
  const __attribute__((address_space(1))) cpx<T>* p;
  int64_t sb;
  int n_data;
  __device__ cpx<T> operator()(int f, int m) const {
    if (m >= n_data) return {T(0), T(0)};
    const auto& z = p[f * sb + m];
    return {z.x, z.y};
  }
};

template <typename T>
struct GatherReal2G {
  const __attribute__((address_space(1))) T* p;
  int64_t sb;
  int n_data, nl;
  __device__ cpx<T> operator()(int f, int m) const {
    if (m >= n_data) return {T(0), T(0)};
    const int l = 2 * f;
    const T a = p[l * sb + m];
    const T b = (l + 1 < nl) ? p[(l + 1) * sb + m] : T(0);
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

template <typename T, class P>
struct GatherR2R {  // symmetric extension of two real lines, with pre-twiddle
  const T* raw;
  int rs, in_n, nl;
  R2R r;
  P tw;  // 4M table
  // Branch-free: the mirrored source index and its weight are selected per lane, the
  // index is clamped into the line, and a sample outside the data gets weight 0.
  // slot m of the extension: its source index jc in the line and its real weight c
  __device__ __forceinline__ void source(int m, int& jc, T& c) const {
    const int nh = r.nh, M = 2 * nh;
    const T eps = r.b2 ? T(-1) : T(1);          // wrap factor of a full period
    const T sigma = r.sin ? -eps : eps;          // sign of the mirrored sample
    int p;
    T coef;
    if (r.a2 == 0) {  // whole-sample symmetry: p and M - p share a sample
      const bool hi = m > nh;
      p = hi ? M - m : m;
      coef = hi ? sigma : T(1);
      coef = (m == 0) ? T(1) + sigma * eps : coef;
      coef = (m == nh) ? T(1) + sigma : coef;
    } else {          // half-sample symmetry: p and M - 1 - p
      const bool hi = m >= nh;
      p = hi ? M - 1 - m : m;
      coef = hi ? sigma : T(1);
    }
    const int j = r.in_rev ? r.in_base - p : p - r.in_base;
    const bool ok = p >= r.plo && p <= r.phi && j >= 0 && j < in_n;
    jc = ok ? j : 0;
    const T w = T(p == r.plo ? r.wlo : (p == r.phi ? r.whi : 2));
    c = ok ? coef * w * T(0.5) : T(0);
  }
  // the complex weight of slot m (c times the pre-twiddle)
  __device__ __forceinline__ cpx<T> weight(int m, int& jc) const {
    T c;
    source(m, jc, c);
    cpx<T> z = {c, T(0)};
    if (r.b2) z = cmul(z, twid<T>(tw, 2 * m));
    return z;
  }
  __device__ cpx<T> operator()(int f, int m) const {
    const int l = 2 * f;
    int jc;
    T c;
    source(m, jc, c);
    const bool two = l + 1 < nl;
    const T a = raw[l * rs + jc];
    const T b = raw[(two ? l + 1 : l) * rs + jc];
    cpx<T> z = {c * a, two ? c * b : T(0)};
    if (r.b2) z = cmul(z, twid<T>(tw, 2 * m));  // exp(-i pi m b / nh), b = 1/2
    return z;
  }
};

// Write the symmetric extensions of a real-to-real tile into the FFT buffer (one LDS
// pass; the raw tile lives outside the buffer), so that the FFT stages read plain LDS.
template <typename T, int MC, class G>
__device__ __forceinline__ void extend_r2r(cpx<T>* buf, int ls, int F, int M, const G& g) {
  const int total = F * M;
  for (int e0 = threadIdx.x; e0 < total; e0 += kChunk * kThreads) {
    cpx<T> z[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int e = e0 + u * kThreads;
      if (e < total) {
        const int f = e / M, m = e - f * M;
        z[u] = g(f, m);
      }
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int e = e0 + u * kThreads;
      if (e < total) {
        const int f = e / M, m = e - f * M;
        buf[f * ls + pad16(m)] = z[u];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------
// Scatters: value of output element j of tile line l, from the FFT buffer.
// ---------------------------------------------------------------------------------
template <typename T, class P>
__device__ __forceinline__ T scatter_r2r(const cpx<T>* buf, int ls, const R2R& r, P tw, int l,
                                         int j) {
  const int q = r.out_rev ? r.out_base - j : j + r.out_base;
  const bool ok = q >= r.qlo && q <= r.qhi;   // outside: the coefficient is 0
  const int qc = ok ? q : r.qlo;
  cpx<T> Y = buf[(l >> 1) * ls + pad16(qc)];
  if (r.a2) Y = cmul(Y, twid<T>(tw, 2 * qc + r.b2));  // exp(-i pi a (q + b) / nh), a = 1/2
  const T v = r.sin ? ((l & 1) ? Y.x : -Y.y) : ((l & 1) ? Y.y : Y.x);
  return ok ? v : T(0);
}

// ---------------------------------------------------------------------------------
// Coalesced tile store.  Element e of the tile maps to (line l, index i):
// line-contiguous data walk along the line (l = e / n), otherwise across the B lines
// of the tile (i = e / B); divisions use host-computed multipliers.
// ---------------------------------------------------------------------------------
// Store with the output conventions of the batch axes (last pass): `out` points at
// (c, b0); writes 0 on odd faces and duplicates index 0 to index last when asked.
// Elements are taken kChunk at a time: all their LDS reads (inside `val`) are issued
// before the first global store, so that one LDS round trip serves the whole chunk.

template <bool FIX, typename E, class Val>
__device__ __forceinline__ void store_tile(E* __restrict__ out, int64_t s_line, int64_t s_b,
                                           int64_t s_c, int nl, int n, uint64_t mag_n, int B,
                                           uint64_t mag_B, int b0, int c, const Fixup& fx,
                                           Val& val) {
  bool czero = false, cdup = false;
  if (FIX) {
    czero = (fx.c_zero_lo && c == 0) || (fx.c_zero_hi && c == fx.c_last);
    cdup = fx.c_dup && c == 0;
  }
  const bool lc = (s_line == 1);
  const int total = lc ? nl * n : B * n;
  for (int e0 = threadIdx.x; e0 < total; e0 += kChunk * kThreads) {
    E v[kChunk];
    int lj[kChunk], jj[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int e = e0 + u * kThreads;
      int l = -1, j = 0;
      if (e < total) {
        if (lc) {
          l = (int)fdiv(e, mag_n);
          j = e - l * n;
        } else {
          j = (int)fdiv(e, mag_B);
          l = e - j * B;
          if (l >= nl) l = -1;
        }
      }
      lj[u] = l;
      jj[u] = j;
      if (l >= 0) v[u] = val(l, j);
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const int l = lj[u];
      if (l < 0) continue;
      const int64_t o = l * s_b + (int64_t)jj[u] * s_line;
      if (FIX) {
        const int b = b0 + l;
        E w = v[u];
        if (czero || (fx.b_zero_lo && b == 0) || (fx.b_zero_hi && b == fx.b_last)) w = E{};
        out[o] = w;
        const bool bdup = fx.b_dup && b == 0;
        if (bdup) out[o + (int64_t)fx.b_last * s_b] = w;
        if (cdup) {
          out[o + (int64_t)fx.c_last * s_c] = w;
          if (bdup) out[o + (int64_t)fx.b_last * s_b + (int64_t)fx.c_last * s_c] = w;
        }
      } else {
        out[o] = v[u];
      }
    }
  }
}

__device__ __forceinline__ int fold_index(int k, int M) {
  if (M == 0) return k;
  const int r = M - k;
  return k < r ? k : r;
}

template <typename T>
__device__ __forceinline__ T signed_wave(int k, int M, T dw) {
  // wavenumber of DFT mode k of length M; the Nyquist mode differentiates to 0
  if (2 * k == M) return T(0);
  const int ks = (2 * k > M) ? k - M : k;
  return dw * T(ks);
}

// u_hat = G i (w x f_hat) at one spectral point (Sec. V), in place.  The wavenumbers of
// the b and c directions (physical axes ab, ac) may be imaginary, i mb / i mc (symmetric
// directions, GreenRef::csym_b / csym; their real parts are then 0): their terms
// i m (e x f) are added under branches that are uniform across the wavefront.
template <typename T>
__device__ __forceinline__ void curl_imag(int a, T m, const cpx<T>& fx, const cpx<T>& fy,
                                          const cpx<T>& fz, cpx<T>& cx, cpx<T>& cy, cpx<T>& cz) {
  // i m (e_a x f): e_x x f = (0, -f_z, f_y), e_y x f = (f_z, 0, -f_x), e_z x f = (-f_y, f_x, 0)
  auto add = [m](cpx<T>& c, const cpx<T>& f, T sg) {  // c += sg i m f
    c.x -= sg * m * f.y;
    c.y += sg * m * f.x;
  };
  if (a == 0) {
    add(cy, fz, T(-1));
    add(cz, fy, T(1));
  } else if (a == 1) {
    add(cx, fz, T(1));
    add(cz, fx, T(-1));
  } else {
    add(cx, fy, T(-1));
    add(cy, fx, T(1));
  }
}

template <typename T>
__device__ __forceinline__ void curl_point(T g, T wx, T wy, T wz, int ac, T m, int ab, T mb,
                                           cpx<T>& fx, cpx<T>& fy, cpx<T>& fz) {
  cpx<T> cx = {wy * fz.x - wz * fy.x, wy * fz.y - wz * fy.y};
  cpx<T> cy = {wz * fx.x - wx * fz.x, wz * fx.y - wx * fz.y};
  cpx<T> cz = {wx * fy.x - wy * fx.x, wx * fy.y - wy * fx.y};
  if (m != T(0)) curl_imag<T>(ac, m, fx, fy, fz, cx, cy, cz);
  if (mb != T(0)) curl_imag<T>(ab, mb, fx, fy, fz, cx, cy, cz);
  fx = {-g * cx.y, g * cx.x};
  fy = {-g * cy.y, g * cy.x};
  fz = {-g * cz.y, g * cz.x};
}

// A direction's factor in the curl: (real, imaginary) = (w, 0) on a DFT direction,
// (0, -s w) on a symmetric or semi-unbounded one (s = GreenRef::csym or csym_b).
template <typename T>
__device__ __forceinline__ void curl_factor(int s, T w, T& re, T& im) {
  re = s ? T(0) : w;
  im = s ? T(-s) * w : T(0);
}

// Derivative factor of DFT mode k in the curl, from the direction's table: the spectral
// wavenumber (0 at the Nyquist mode) or the plan's central-difference symbol (Sec. V).
template <typename T>
__device__ __forceinline__ T curl_wave(int k, const void* tab) {
  return gptr<T>(tab)[k];
}

struct TileIdx {
  int b0, c, comp, nl;
};

__device__ __forceinline__ TileIdx tile_index(const PassDesc& d, int tile) {
  const int nbt = (d.nb + d.B - 1) / d.B;
  TileIdx ti;
  const int bt = tile % nbt;
  const int t = tile / nbt;
  ti.c = t % d.nc;
  ti.comp = t / d.nc;
  ti.b0 = bt * d.B;
  ti.nl = min(d.B, d.nb - ti.b0);
  return ti;
}

// ---------------------------------------------------------------------------------
// Plain pass on one tile
// ---------------------------------------------------------------------------------
template <typename T, int MC, bool FIX, class Val>
__device__ __forceinline__ void store_real(const PassDesc& d, void* out, const TileIdx& ti,
                                           int64_t out_off, Val& val) {
  store_tile<FIX>(reinterpret_cast<T*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c, ti.nl,
                  d.out_n, d.mag_out, d.B, d.mag_B, ti.b0, ti.c, d.fix, val);
}

// The FFT lines of a plain tile, in natural order in LDS (line f at buf + f ls), written
// into the output layout by the pass's scatter.
template <typename T, int MC, int KIND, class P>
__device__ __forceinline__ void plain_store(const PassDesc& d, void* out, const TileIdx& ti,
                                            const cpx<T>* buf, P tw) {
  const int scatter = KIND == K_ANY ? d.scatter : scatter_of(KIND);
  const int nl = ti.nl;
  const int M = MC > 1 ? MC : d.M;
  const int ls = fft_line_stride(M);
  const int64_t out_off = ti.comp * d.out_s_comp + ti.c * d.out_s_c + ti.b0 * d.out_s_b;
  if (scatter == S_CPLX) {
    auto val = [&](int l, int j) { return buf[l * ls + pad16(j < M ? j : j - M)]; };
    store_tile<false>(reinterpret_cast<cpx<T>*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c,
                      nl, d.out_n, d.mag_out, d.B, d.mag_B, ti.b0, ti.c, d.fix, val);
  } else if (scatter == S_R2C2) {
    auto val = [&](int l, int k) {
      const cpx<T>* z = buf + (l >> 1) * ls;
      const cpx<T> zk = z[pad16(k)], zm = z[pad16(k == 0 ? 0 : M - k)];
      if (l & 1) return cpx<T>{T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
      return cpx<T>{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
    };
    store_tile<false>(reinterpret_cast<cpx<T>*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c,
                      nl, d.out_n, d.mag_out, d.B, d.mag_B, ti.b0, ti.c, d.fix, val);
  } else if (scatter == S_REAL2) {
    auto val = [&](int l, int j) {
      const cpx<T> z = buf[(l >> 1) * ls + pad16(j < M ? j : j - M)];
      return (l & 1) ? z.y : z.x;
    };
    if (d.has_fix) store_real<T, MC, true>(d, out, ti, out_off, val);
    else store_real<T, MC, false>(d, out, ti, out_off, val);
  } else {
    auto val = [&](int l, int j) { return scatter_r2r<T>(buf, ls, d.r2r, tw, l, j); };
    if (d.out_cplx) {
      // the real-to-real spectrum handed on as complex values with a zero imaginary part
      // (the next axis is transformed as a full complex DFT)
      auto cval = [&](int l, int j) { return cpx<T>{val(l, j), T(0)}; };
      store_tile<false>(reinterpret_cast<cpx<T>*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c,
                        nl, d.out_n, d.mag_out, d.B, d.mag_B, ti.b0, ti.c, d.fix, cval);
    } else if (d.has_fix) {
      store_real<T, MC, true>(d, out, ti, out_off, val);
    } else {
      store_real<T, MC, false>(d, out, ti, out_off, val);
    }
  }
}

// DIRECT: forward complex or real-to-complex lines read by the first FFT stage straight
// from contiguous input lines at gin (the tile's first line) instead of the LDS raw tile.
template <typename T, int MC, int KIND, bool DIRECT = false, class P>
__device__ void plain_compute(const PassDesc& d, void* out, const TileIdx& ti, char* smem,
                              const Tabs<P>& tb, const void* gin = nullptr) {
  const int gather = KIND == K_ANY ? d.gather : gather_of(KIND);
  const int scatter = KIND == K_ANY ? d.scatter : scatter_of(KIND);
  const int sign = KIND == K_ANY ? d.sign : (KIND == K_C2C_I || KIND == K_C2R ? +1 : -1);
  const int nl = ti.nl;
  const P tw = tb.tw;
  const int M = MC > 1 ? MC : d.M;
  const int ls = fft_line_stride(M);
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);
  const int64_t out_off = ti.comp * d.out_s_comp + ti.c * d.out_s_c + ti.b0 * d.out_s_b;
  const int rs = d.in_n + 1;

  // 2) FFT (first stage gathers from the raw tile, which aliases the FFT buffer)
  const int F = (gather == G_CPLX) ? nl : (nl + 1) / 2;
  if constexpr (DIRECT && KIND == K_C2C_F) {
    GatherCplxG<T> g{gptr<cpx<T>>(gin), d.in_s_b, d.n_data};
    fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g);
  } else if constexpr (DIRECT && KIND == K_R2C) {
    GatherReal2G<T> g{gptr<T>(gin), d.in_s_b, d.n_data, nl};
    fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g);
  } else if (gather == G_CPLX) {
    GatherCplx<T> g{reinterpret_cast<const cpx<T>*>(smem), rs, d.n_data};
    // complex lines are written from their first out_n slots (cropped inverse)
    const int keep = scatter == S_CPLX ? min(d.out_n, M) : M;
    if constexpr (MC > 1) {
      if (scatter == S_CPLX && d.out_s_line == 1) {
        // contiguous output lines: the last stage stores them directly
        cpx<T>* o = reinterpret_cast<cpx<T>*>(out) + out_off;
        const int64_t sb = d.out_s_b;
        const int on = d.out_n;
        auto sink = [o, sb, on](int l, int j, const cpx<T>& v) {
          cpx<T>* r = o + l * sb;
          r[j] = v;
          if (j + MC < on) r[j + MC] = v;
        };
        if (sign < 0) stages_ct<T, MC, -1, 0, 1>(buf, ls, F, tb.stw, g, keep, sink);
        else stages_ct<T, MC, +1, 0, 1>(buf, ls, F, tb.stw, g, keep, sink);
        return;
      }
    }
    if (sign < 0) fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g, keep);
    else fft_lines<T, MC, +1>(buf, ls, F, d, tb.stw, g, keep);
  } else if (gather == G_REAL2) {
    GatherReal2<T> g{reinterpret_cast<const T*>(smem), rs, d.n_data, nl};
    fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g);
  } else if (gather == G_HERM2) {
    GatherHerm2<T> g{reinterpret_cast<const cpx<T>*>(smem), rs, M, nl};
    if constexpr (MC > 1) {
      if (scatter == S_REAL2 && !d.has_fix && d.out_s_line == 1) {
        // contiguous real output lines without fix-ups: FFT line f holds tile lines 2f
        // (real part) and 2f + 1 (imaginary part); the last stage stores them directly
        T* o = reinterpret_cast<T*>(out) + out_off;
        const int64_t sb = d.out_s_b;
        const int on = d.out_n;
        auto sink = [o, sb, on, nl](int f, int j, const cpx<T>& v) {
          T* r0 = o + (2 * f) * sb;
          r0[j] = v.x;
          if (j + MC < on) r0[j + MC] = v.x;
          if (2 * f + 1 < nl) {
            T* r1 = r0 + sb;
            r1[j] = v.y;
            if (j + MC < on) r1[j + MC] = v.y;
          }
        };
        stages_ct<T, MC, +1, 0, 1>(buf, ls, F, tb.stw, g, min(on, M), sink);
        return;
      }
    }
    fft_lines<T, MC, +1>(buf, ls, F, d, tb.stw, g, scatter == S_REAL2 ? min(d.out_n, M) : M);
  } else {
    // the first stage builds the symmetric extension as it reads the raw tile (every
    // read of a stage precedes its writes, so the raw tile may alias the FFT buffer)
    GatherR2R<T, P> g{reinterpret_cast<const T*>(smem + d.raw_off), rs, d.in_n, nl, d.r2r, tw};
    fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g);
  }

  // 3) write the lines into the output layout
  plain_store<T, MC, KIND>(d, out, ti, buf, tw);
}

// ---------------------------------------------------------------------------------
// Fused pass 3 on one tile: forward FFT, spectral multiply, inverse FFT.
// ---------------------------------------------------------------------------------
template <typename T, int MC, int KIND, class P>
__device__ void fused_compute(const PassDesc& d, void* out, const TileIdx& ti, char* smem,
                              const Tabs<P>& tb) {
  const int gather = KIND == K_ANY ? d.gather : gather_of(KIND);
  const bool curl = KIND == K_ANY ? (d.g.curl != 0) : (KIND == K_F_CURL);
  const int nl = ti.nl, b0 = ti.b0, c = ti.c, comp = ti.comp;  // curl: comp = 0
  const P tw = tb.tw;
  const int M = MC > 1 ? MC : d.M;
  const int ls = fft_line_stride(M);
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem);
  const int rs = d.in_n + 1;
  const int ncl = curl ? 3 : 1;   // components held by the tile
  // the tile's Green rows, staged in LDS with the tile: row l holds F_line values
  const T* gl = reinterpret_cast<const T*>(smem + d.g_off);
  const int FL = d.g.F_line;
  const Fixup nofix{};

  if (gather == G_R2R) {
    // ---- all-real-to-real problem: forward R2R -> spectrum in LDS -> inverse R2R
    const int F = (nl + 1) / 2;
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + pad16(idx)]; };
    {
      GatherR2R<T, P> g{reinterpret_cast<const T*>(smem + d.raw_off), rs, d.in_n, nl, d.r2r, tw};
      extend_r2r<T, MC>(buf, ls, F, M, g);
      fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, lds);
    }
    // spectrum (real) into its own LDS region (where the raw tile was), times the
    // Green's spectrum
    const int ss = d.spec_n + 1;
    T* spec = reinterpret_cast<T*>(smem + d.raw_off);
    chunked<T>(
        nl * d.spec_n,
        [&](int e) {
          const int l = (int)fdiv(e, d.mag_spec), j = e - l * d.spec_n;
          return gl[l * FL + fold_index(j, d.g.fold_line)] * scatter_r2r<T>(buf, ls, d.r2r, tw, l, j);
        },
        [&](int e, T v) {
          const int l = (int)fdiv(e, d.mag_spec), j = e - l * d.spec_n;
          spec[l * ss + j] = v;
        });
    __syncthreads();
    {
      GatherR2R<T, P> g{spec, ss, d.spec_n, nl, d.r2r2, tw};
      extend_r2r<T, MC>(buf, ls, F, M, g);
      fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, lds);
    }
    const int64_t out_off = comp * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
    auto val = [&](int l, int j) { return scatter_r2r<T>(buf, ls, d.r2r2, tw, l, j); };
    store_tile<false>(reinterpret_cast<T*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c, nl,
                      d.out_n, d.mag_out, d.B, d.mag_B, b0, c, nofix, val);
    return;
  }

  if (gather == G_REAL2) {
    // ---- only DFT axis of the problem: two real lines per FFT
    const int F = (nl + 1) / 2;
    GatherReal2<T> g{reinterpret_cast<const T*>(smem), rs, d.n_data, nl};
    fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g);
    // The two packed lines have their own Green rows: split Z into the two Hermitian
    // spectra X1 = (Z_k + conj Z_{M-k})/2, X2 = (Z_k - conj Z_{M-k})/(2i), scale each
    // by its (real, even) row, and pack again as Y1 + i Y2.  One thread owns the pair
    // (k, M-k).
    const int H = M / 2 + 1;
    struct Pair {
      cpx<T> a, b;
    };
    chunked<Pair>(
        F * H,
        [&](int e) {
          const int f = e / H, k = e - f * H;
          const int kk = fold_index(k, d.g.fold_line);
          const int l0 = 2 * f, l1 = min(2 * f + 1, nl - 1);
          const T g0 = gl[l0 * FL + kk];
          const T g1 = gl[l1 * FL + kk];
          const int km = (k == 0) ? 0 : M - k;
          const cpx<T> zk = buf[f * ls + pad16(k)], zm = buf[f * ls + pad16(km)];
          const cpx<T> x1 = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
          const cpx<T> x2 = {T(0.5) * (zk.y + zm.y), T(-0.5) * (zk.x - zm.x)};
          // Z'_k = g0 X1 + i g1 X2 ;  Z'_{M-k} = g0 conj(X1) + i g1 conj(X2)
          return Pair{{g0 * x1.x - g1 * x2.y, g0 * x1.y + g1 * x2.x},
                      {g0 * x1.x + g1 * x2.y, -g0 * x1.y + g1 * x2.x}};
        },
        [&](int e, const Pair& v) {
          const int f = e / H, k = e - f * H;
          const int km = (k == 0) ? 0 : M - k;
          buf[f * ls + pad16(k)] = v.a;
          if (km != k) buf[f * ls + pad16(km)] = v.b;
        });
    __syncthreads();
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + pad16(idx)]; };
    fft_lines<T, MC, +1>(buf, ls, F, d, tb.stw, lds);
    const int64_t out_off = comp * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
    auto val = [&](int l, int j) {
      const cpx<T> z = buf[(l >> 1) * ls + pad16(j < M ? j : j - M)];
      return (l & 1) ? z.y : z.x;
    };
    store_tile<false>(reinterpret_cast<T*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c, nl,
                      d.out_n, d.mag_out, d.B, d.mag_B, b0, c, nofix, val);
    return;
  }

  // ---- complex lines (C2C along the last axis), one or three components
  const int F = ncl * nl;
  {
    GatherCplx<T> g{reinterpret_cast<const cpx<T>*>(smem), rs, d.n_data};
    fft_lines<T, MC, -1>(buf, ls, F, d, tb.stw, g);
  }
  if (!curl) {
    // the multiplication by the Green's spectrum is the first inverse stage's load
    const int fl = d.g.fold_line;
    auto lds_g = [buf, ls, gl, FL, fl](int line, int idx) {
      const cpx<T> z = buf[line * ls + pad16(idx)];
      const T g = gl[line * FL + fold_index(idx, fl)];
      return cpx<T>{z.x * g, z.y * g};
    };
    if constexpr (MC > 1) {
      if (d.out_s_line == 1) {
        // contiguous output lines: the last inverse stage's lanes hold consecutive slots
        // of a line, so they store to global memory directly (no LDS pass, no store loop)
        cpx<T>* o = reinterpret_cast<cpx<T>*>(out) + comp * d.out_s_comp + c * d.out_s_c +
                    b0 * d.out_s_b;
        const int64_t sb = d.out_s_b;
        const int on = d.out_n;
        auto sink = [o, sb, on](int l, int j, const cpx<T>& v) {
          cpx<T>* r = o + l * sb;
          r[j] = v;
          if (j + MC < on) r[j + MC] = v;  // periodic duplicate beyond one period
        };
        stages_ct<T, MC, +1, 0, 1>(buf, ls, F, tb.stw, lds_g, min(on, M), sink);
        return;
      }
    }
    fft_lines<T, MC, +1>(buf, ls, F, d, tb.stw, lds_g, min(d.out_n, M));
  } else {
    T wc, mc;
    curl_factor<T>(d.g.csym, curl_wave<T>(c, d.g.dtab_c), wc, mc);
    struct Tri {
      cpx<T> x, y, z;
    };
    chunked<Tri>(
        nl * M,
        [&](int e) {
          const int l = e / M, k = e - l * M;
          const T g = gl[l * FL + fold_index(k, d.g.fold_line)];
          const T wl = curl_wave<T>(k, d.g.dtab_line);
          T wb, mb;
          curl_factor<T>(d.g.csym_b, curl_wave<T>(b0 + l, d.g.dtab_b), wb, mb);
          const T wx = d.g.axis_line == 0 ? wl : (d.g.axis_b == 0 ? wb : wc);
          const T wy = d.g.axis_line == 1 ? wl : (d.g.axis_b == 1 ? wb : wc);
          const T wz = d.g.axis_line == 2 ? wl : (d.g.axis_b == 2 ? wb : wc);
          cpx<T> fx = buf[(0 * nl + l) * ls + pad16(k)];
          cpx<T> fy = buf[(1 * nl + l) * ls + pad16(k)];
          cpx<T> fz = buf[(2 * nl + l) * ls + pad16(k)];
          curl_point<T>(g, wx, wy, wz, d.g.axis_c, mc, d.g.axis_b, mb, fx, fy, fz);
          return Tri{fx, fy, fz};
        },
        [&](int e, const Tri& v) {
          const int l = e / M, k = e - l * M;
          buf[(0 * nl + l) * ls + pad16(k)] = v.x;
          buf[(1 * nl + l) * ls + pad16(k)] = v.y;
          buf[(2 * nl + l) * ls + pad16(k)] = v.z;
        });
    __syncthreads();
    auto lds = [buf, ls](int line, int idx) { return buf[line * ls + pad16(idx)]; };
    if constexpr (MC > 1) {
      if (d.out_s_line == 1) {
        // contiguous output lines: component q's line l (FFT line q nl + l) is stored
        // by the last inverse stage directly
        cpx<T>* o = reinterpret_cast<cpx<T>*>(out) + c * d.out_s_c + b0 * d.out_s_b;
        const int64_t sb = d.out_s_b, sq = d.out_s_comp;
        const int on = d.out_n;
        auto sink = [o, sb, sq, on, nl](int line, int j, const cpx<T>& v) {
          const int q = line >= 2 * nl ? 2 : (line >= nl ? 1 : 0);
          cpx<T>* r = o + q * sq + (line - q * nl) * sb;
          r[j] = v;
          if (j + MC < on) r[j + MC] = v;
        };
        stages_ct<T, MC, +1, 0, 1>(buf, ls, F, tb.stw, lds, min(on, M), sink);
        return;
      }
    }
    fft_lines<T, MC, +1>(buf, ls, F, d, tb.stw, lds, min(d.out_n, M));
  }
  for (int q = 0; q < ncl; ++q) {
    const int cc = curl ? q : comp;
    const int64_t out_off = cc * d.out_s_comp + c * d.out_s_c + b0 * d.out_s_b;
    const cpx<T>* z = buf + (size_t)q * nl * ls;
    auto val = [&](int l, int j) { return z[l * ls + pad16(j < M ? j : j - M)]; };
    store_tile<false>(reinterpret_cast<cpx<T>*>(out) + out_off, d.out_s_line, d.out_s_b, d.out_s_c,
                      nl, d.out_n, d.mag_out, d.B, d.mag_B, b0, c, nofix, val);
  }
}

// ---------------------------------------------------------------------------------
// Input staging: a tile's input is read from global memory into registers (`fetch`),
// then written to the raw LDS region (`commit`).  Element e of the tile walks along
// the lines when they are contiguous, else across the B lines of the tile; the fused
// Biot-Savart pass reads the three components of the same lines (component q's lines
// follow component q-1's in LDS).
// ---------------------------------------------------------------------------------
// Values per thread held by the register stage of one tile (per component).
template <typename T, typename E, int NCL, int MC>
struct StageCount {
  static constexpr int U = stage_values((int)sizeof(T), MC, sizeof(E) != sizeof(T), NCL);
};

struct TileWalk {
  int per, n, B, nl;
  bool lc;
  uint64_t mag_n, mag_B;
  // element r of one component -> line l, index i; false when outside the tile
  __device__ __forceinline__ bool at(int r, int& l, int& i) const {
    if (r >= per) return false;
    if (lc) {
      l = (int)fdiv(r, mag_n);
      i = r - l * n;
    } else {
      i = (int)fdiv(r, mag_B);
      l = r - i * B;
      if (l >= nl) return false;
    }
    return true;
  }
};

__device__ __forceinline__ TileWalk in_walk(const PassDesc& d, const TileIdx& ti) {
  TileWalk w;
  w.lc = (d.in_s_line == 1);
  w.n = d.in_n;
  w.B = d.B;
  w.nl = ti.nl;
  w.per = w.lc ? ti.nl * d.in_n : d.B * d.in_n;
  w.mag_n = d.mag_in;
  w.mag_B = d.mag_B;
  return w;
}

// Register stage of one thread: complex values are held as two real arrays (a 16-byte
// struct array is not always promoted to registers).
template <typename T, typename E, int N>
struct RegStage {
  T a[N];
  __device__ __forceinline__ void set(int k, const T& v) { a[k] = v; }
  __device__ __forceinline__ T get(int k) const { return a[k]; }
};
template <typename T, int N>
struct RegStage<T, cpx<T>, N> {
  T x[N], y[N];
  __device__ __forceinline__ void set(int k, const cpx<T>& v) {
    x[k] = v.x;
    y[k] = v.y;
  }
  __device__ __forceinline__ cpx<T> get(int k) const { return {x[k], y[k]}; }
};

// Global -> registers.  Addresses are a uniform 64-bit base per component plus a 32-bit
// byte offset per element; the planner sends tiles that span 4 GiB or more to the
// runtime-length kernels (OFF64), which use 64-bit offsets.
template <int U, int NCL, bool OFF64, typename E, class Stage>
__device__ __forceinline__ void fetch(Stage& v, const PassDesc& d, const void* in, const TileIdx& ti) {
  const TileWalk w = in_walk(d, ti);
  const int comp0 = NCL == 3 ? 0 : ti.comp;
#pragma unroll
  for (int q = 0; q < NCL; ++q) {
    const char* base = reinterpret_cast<const char*>(in) +
                       ((int64_t)(comp0 + q) * d.in_s_comp + (int64_t)ti.c * d.in_s_c +
                        (int64_t)ti.b0 * d.in_s_b) * (int64_t)sizeof(E);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int l, i;
      if (w.at((int)threadIdx.x + u * kThreads, l, i)) {
        if constexpr (OFF64) {
          const int64_t off = ((int64_t)l * d.in_s_b + (int64_t)i * d.in_s_line) * (int64_t)sizeof(E);
          v.set(q * U + u, *reinterpret_cast<const E*>(base + off));
        } else {
          const uint32_t off = ((uint32_t)l * (uint32_t)d.in_s_b + (uint32_t)i * (uint32_t)d.in_s_line) *
                               (uint32_t)sizeof(E);
          v.set(q * U + u, *reinterpret_cast<const E*>(base + off));
        }
      }
    }
  }
}

// Registers -> raw LDS tile; component q's lines follow component q-1's.
template <int U, int NCL, typename E, class Stage>
__device__ __forceinline__ void commit(const Stage& v, const PassDesc& d, const TileIdx& ti,
                                       char* smem) {
  const TileWalk w = in_walk(d, ti);
  E* raw = reinterpret_cast<E*>(smem + d.raw_off);
  const int rs = d.in_n + 1;
#pragma unroll
  for (int q = 0; q < NCL; ++q) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int l, i;
      if (w.at((int)threadIdx.x + u * kThreads, l, i)) raw[(q * ti.nl + l) * rs + i] = v.get(q * U + u);
    }
  }
}

// The Green rows of a fused tile (nl rows of g.F_line values) travel with the tile's
// input: loaded into registers by `fetch_green`, written to LDS at g_off by
// `commit_green`.
template <typename T, int UG>
struct GreenStage {
  T a[UG];
};

template <typename T, int UG>
__device__ __forceinline__ void fetch_green(GreenStage<T, UG>& gs, const PassDesc& d,
                                            const TileIdx& ti) {
  const auto* G = gptr<T>(d.g.G);
  const int FL = d.g.F_line;
  const int per = ti.nl * FL;
  const int64_t fc = fold_index(ti.c, d.g.fold_c);
#pragma unroll
  for (int u = 0; u < UG; ++u) {
    const int r = (int)threadIdx.x + u * kThreads;
    if (r < per) {
      const int l = (int)fdiv(r, d.mag_gline);
      const int j = r - l * FL;
      gs.a[u] = G[(fc * d.g.F_b + fold_index(ti.b0 + l, d.g.fold_b)) * FL + j];
    }
  }
}

template <typename T, int UG>
__device__ __forceinline__ void commit_green(const GreenStage<T, UG>& gs, const PassDesc& d,
                                             const TileIdx& ti, char* smem) {
  T* gl = reinterpret_cast<T*>(smem + d.g_off);
  const int per = ti.nl * d.g.F_line;
#pragma unroll
  for (int u = 0; u < UG; ++u) {
    const int r = (int)threadIdx.x + u * kThreads;
    if (r < per) gl[r] = gs.a[u];
  }
}

// Values per thread of the Green stage of a kind (K_ANY: the largest).
template <typename T, int MC, int KIND>
constexpr int green_stage() {
  return fused_of(KIND) || KIND == K_ANY
             ? green_values((int)sizeof(T), MC, !(KIND == K_F_C2C || KIND == K_F_CURL))
             : 1;
}

template <typename T>
__device__ __forceinline__ Tabs<GTab<T>> global_tabs(const PassDesc& d) {
  return {gptr<cpx<T>>(d.stw), gptr<cpx<T>>(d.tw)};
}

template <typename T, int MC, int KIND, class P>
__device__ __forceinline__ void compute(const PassDesc& d, void* out, const TileIdx& ti,
                                        char* smem, const Tabs<P>& tb) {
  if constexpr (KIND == K_ANY) {
    if (d.fused) fused_compute<T, MC, K_ANY>(d, out, ti, smem, tb);
    else plain_compute<T, MC, K_ANY>(d, out, ti, smem, tb);
  } else if constexpr (fused_of(KIND)) {
    fused_compute<T, MC, KIND>(d, out, ti, smem, tb);
  } else {
    plain_compute<T, MC, KIND>(d, out, ti, smem, tb);
  }
}

// One tile, no pipelining (batched launches: the kind is read from the descriptor).
template <typename T, int MC, typename E, int NCL>
__device__ __forceinline__ void run_tile_e(const PassDesc& d, const void* in, void* out, int tile,
                                           char* smem) {
  constexpr int U = StageCount<T, E, NCL, MC>::U;
  constexpr int UG = green_stage<T, MC, K_ANY>();
  RegStage<T, E, U * NCL> v;
  GreenStage<T, UG> gs;
  const TileIdx ti = tile_index(d, tile);
  fetch<U, NCL, (MC <= 1), E>(v, d, in, ti);
  if (d.fused) fetch_green<T, UG>(gs, d, ti);
  commit<U, NCL, E>(v, d, ti, smem);
  if (d.fused) commit_green<T, UG>(gs, d, ti, smem);
  __syncthreads();
  compute<T, MC, K_ANY>(d, out, ti, smem, global_tabs<T>(d));
}

template <typename T, int MC>
__device__ __forceinline__ void run_tile(const PassDesc& d, const void* in, void* out, int tile,
                                         char* smem) {
  if (d.fused && d.g.curl) run_tile_e<T, MC, cpx<T>, 3>(d, in, out, tile, smem);
  else if (d.in_cplx) run_tile_e<T, MC, cpx<T>, 1>(d, in, out, tile, smem);
  else run_tile_e<T, MC, T, 1>(d, in, out, tile, smem);
}

// XCD-aware order of the tiles.  Workgroups are dispatched to the 8 XCDs round-robin
// (block b on XCD b mod 8), and each XCD has its own L2.  The tiles are cut into 8
// contiguous ranges, one per XCD, and the blocks of an XCD walk their range side by side:
// tiles that are neighbours along the tile axis (and share cache lines of a strided
// input or output) run at the same time on the same L2.  Tile k of block b (k = 0, 1,
// ...) is returned, or -1 past the end of the block's share.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int grid, int k, int tiles) {
  if (grid < kXcds) {  // too few blocks to give every XCD a share: plain striding
    const int t = b + k * grid;
    return t < tiles ? t : -1;
  }
  const int x = b % kXcds, j = b / kXcds;
  const int per = (tiles + kXcds - 1) / kXcds;       // tiles of one XCD
  const int nbx = (grid - x + kXcds - 1) / kXcds;    // blocks on XCD x
  const int local = j + k * nbx;
  if (local >= per) return -1;
  const int t = x * per + local;
  return t < tiles ? t : -1;
}

// Persistent loop over the tiles of a pass: while tile t is transformed in LDS, the
// input of the next tile of this workgroup (and its Green rows) is already on its way
// into registers.  The twiddle tables are copied to LDS once, so that the transform
// issues no global loads: vector-memory loads complete in order, and a global load
// inside the transform would wait for the whole prefetch.
template <typename T, int MC, int KIND>
__device__ __forceinline__ void run_pipelined(const PassDesc& d, const void* in, void* out,
                                              char* smem) {
  using E = typename std::conditional<in_cplx_of(KIND), cpx<T>, T>::type;
  constexpr int NCL = KIND == K_F_CURL ? 3 : 1;
  constexpr int U = StageCount<T, E, NCL, MC>::U;
  constexpr bool FUSED = fused_of(KIND);
  constexpr int UG = green_stage<T, MC, KIND>();
  int k = 0;
  int tile = xcd_tile(blockIdx.x, gridDim.x, k, d.tiles);
  if (tile < 0) return;
  // the first tile's input is requested before the tables are copied: the two HBM
  // latencies overlap (the copy waits for both, loads completing in order)
  RegStage<T, E, U * NCL> v;
  GreenStage<T, UG> gs;
  TileIdx ti = tile_index(d, tile);
  fetch<U, NCL, false, E>(v, d, in, ti);
  if constexpr (FUSED) fetch_green<T, UG>(gs, d, ti);
  // twiddle tables -> LDS (visible to the transform after the loop's barriers)
  cpx<T>* lt = reinterpret_cast<cpx<T>*>(smem + d.tab_off);
  {
    const auto* stw = gptr<cpx<T>>(d.stw);
    const auto* tw = gptr<cpx<T>>(d.tw);
    const int n1 = d.stw_n, n2 = d.stw_n + d.tw_n;
    for (int i = threadIdx.x; i < n2; i += kThreads) {
      const auto& w = i < n1 ? stw[i] : tw[i - n1];
      lt[i] = cpx<T>{w.x, w.y};
    }
  }
  // real-to-real kinds always have their twiddles staged (tw_n = 2M); other kinds do
  // not read tw in the compile-time kernels
  const Tabs<const cpx<T>*> tb{lt, lt + d.stw_n};
  while (true) {
    __syncthreads();  // the previous tile's LDS reads are finished
    commit<U, NCL, E>(v, d, ti, smem);
    if constexpr (FUSED) commit_green<T, UG>(gs, d, ti, smem);
    __syncthreads();
    const int next = xcd_tile(blockIdx.x, gridDim.x, ++k, d.tiles);
    TileIdx tn = ti;
    if (next >= 0) {
      tn = tile_index(d, next);
      fetch<U, NCL, false, E>(v, d, in, tn);
      if constexpr (FUSED) fetch_green<T, UG>(gs, d, tn);
    }
    compute<T, MC, KIND>(d, out, ti, smem, tb);
    if (next < 0) break;
    tile = next;
    ti = tn;
  }
}

// One tile per workgroup (runtime lengths, long FP64 lines, and compile-time lengths
// launched with one workgroup per tile): no register prefetch, tables read from global
// memory.
template <typename T, int MC, int KIND>
__device__ __forceinline__ void run_single(const PassDesc& d, const void* in, void* out,
                                           char* smem) {
  // tiles in the XCD-aware order; with a grid of one block per tile each block takes
  // one or two tiles
  using E = typename std::conditional<in_cplx_of(KIND), cpx<T>, T>::type;
  constexpr int NCL = KIND == K_F_CURL ? 3 : 1;
  constexpr int U = StageCount<T, E, NCL, MC>::U;
  constexpr int UG = green_stage<T, MC, KIND>();
  for (int k = 0;; ++k) {
    const int tile = xcd_tile(blockIdx.x, gridDim.x, k, d.tiles);
    if (tile < 0) return;
    if (k > 0) __syncthreads();  // the previous tile's LDS reads are finished
    const TileIdx ti = tile_index(d, tile);
    if constexpr (MC > 1 && (KIND == K_C2C_F || (KIND == K_R2C && MC <= 512))) {
      if (d.in_s_line == 1) {
        // contiguous input lines: the first FFT stage reads them from global memory
        // (measured slower for real-to-complex lines of 1024 and more, which keep the
        // LDS tile)
        const void* gin = reinterpret_cast<const char*>(in) +
                          ((int64_t)ti.comp * d.in_s_comp + (int64_t)ti.c * d.in_s_c +
                           (int64_t)ti.b0 * d.in_s_b) * (int64_t)sizeof(E);
        plain_compute<T, MC, KIND, true>(d, out, ti, smem, global_tabs<T>(d), gin);
        continue;
      }
    }
    RegStage<T, E, U * NCL> v;
    GreenStage<T, UG> gs;
    fetch<U, NCL, (MC <= 1), E>(v, d, in, ti);
    if constexpr (fused_of(KIND)) fetch_green<T, UG>(gs, d, ti);
    commit<U, NCL, E>(v, d, ti, smem);
    if constexpr (fused_of(KIND)) commit_green<T, UG>(gs, d, ti, smem);
    __syncthreads();
    compute<T, MC, KIND>(d, out, ti, smem, global_tabs<T>(d));
  }
}

// The descriptor lives in device memory (uniform loads); the buffers of this solve are
// kernel arguments.
// PIPE = 1: the pipelined kernel, with the twiddle tables staged in LDS (a persistent
// grid, or one tile per workgroup); PIPE = 0: one tile per workgroup with the tables read
// from global memory, which leaves LDS for more workgroups per CU.  The plain kinds of
// the latter are held to at most 168 VGPRs (three waves per SIMD), which they fit
// without spilling; the fused kinds would spill there and keep the compiler's choice.
template <int KIND, int PIPE>
constexpr int min_waves_per_simd() {
  return (PIPE == 0 && !fused_of(KIND) && KIND != K_ANY) ? 3 : 1;
}

template <typename T, int MC, int KIND, int PIPE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(min_waves_per_simd<KIND, PIPE>())))
void pass_kernel(const PassDesc* __restrict__ dp,
                                                        const void* in, void* out) {
  extern __shared__ __align__(16) char smem[];
  if constexpr (PIPE && pipelined_kernel((int)sizeof(T), MC)) run_pipelined<T, MC, KIND>(*dp, in, out, smem);
  else run_single<T, MC, KIND>(*dp, in, out, smem);
}

// Batched form: tiles of many descriptors of one length class in one launch;
// prefix[i] = first tile of descriptor i, prefix[n] = total.
template <typename T, int MC>
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
  const PassDesc& d = ds[lo];
  run_tile<T, MC>(d, d.in, d.out, tile - prefix[lo], smem);
}


}  // namespace fm
