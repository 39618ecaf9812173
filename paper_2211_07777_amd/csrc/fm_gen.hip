// FP64 generation kernels (twiddles, Green's spectrum) and the length dispatch of the
// pass launchers.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fm_device.h"
#include "fm_launch.h"
#include "fm_special.h"

namespace fm {

// ---------------------------------------------------------------------------------
// FP64 generation: twiddles, Green's spectrum samples, finalisation
// ---------------------------------------------------------------------------------
// Per-stage twiddles of a compile-time length: stage s (radix R, Ns = product of the
// earlier radices) holds W_{Ns R}^{k r} = exp(-2 pi i k r / (Ns R)) at
// offset(s) + k (R - 1) + r - 1, for k < Ns and 1 <= r < R.
template <typename T>
__global__ void stage_twiddle_kernel(cpx<T>* out, int M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int off = 0, ns = 1;
  for (int s = 0;; ++s) {
    const int R = radix_at(M, s, max_radix((int)sizeof(T)));
    if (R == 0) return;
    const int n = ns * (R - 1);
    if (j < off + n) {
      const int e = j - off;
      const int k = e / (R - 1), r = e % (R - 1) + 1;
      const long long num = 2LL * k * r;  // angle 2 pi k r / (ns R) = pi * num / (ns R)
      double sn, cs;
      sincospi((double)(num % (2LL * ns * R)) / (double)(ns * R), &sn, &cs);
      out[j] = {T(cs), T(-sn)};
      return;
    }
    off += n;
    ns *= R;
  }
}

// Stage twiddles of the per-wavefront kernels: stage s >= 1 (radix R, Ns) holds
// W_{Ns R}^{k r} at wave_tw_offset(M, s) + (r - 1) Ns + k.
template <typename T>
__global__ void wave_twiddle_kernel(cpx<T>* out, int M, int E) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  for (int s = 1; wave_radix(M, s, E) != 0; ++s) {
    const int R = wave_radix(M, s, E), Ns = wave_ns(M, s, E);
    const int off = wave_tw_offset(M, s, E);
    if (e >= off && e < off + Ns * (R - 1)) {
      const int r = (e - off) / Ns + 1, k = (e - off) % Ns;
      const long long num = 2LL * k * r;  // angle 2 pi k r / (Ns R) = pi num / (Ns R)
      double sn, cs;
      sincospi((double)(num % (2LL * Ns * R)) / (double)(Ns * R), &sn, &cs);
      out[e] = {T(cs), T(-sn)};
      return;
    }
  }
}

template <typename T>
__global__ void twiddle_kernel(cpx<T>* out, int M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 4 * M) return;
  double s, c;
  sincospi((double)j / (2.0 * (double)M), &s, &c);  // angle 2 pi j / (4 M)
  out[j] = {T(c), T(-s)};
}

// Regularised kernels (FM_GREEN_HEJ*): variant 2..6 is the order m = 2 (variant - 1),
// variant 7 the spectral truncation.  Real space (three convolution directions), with
// p = r / eps:
//   G = -(1 / 4 pi r) [erf(p / sqrt 2) + sqrt(2/pi) p exp(-p^2 / 2) Q_m(p^2)],
//   Q_2 = 0, Q_4 = 1/2, Q_6 = (7 - p^2) / 8, Q_8 = (57 - 16 p^2 + p^4) / 48,
//   Q_10 = (561 - 233 p^2 + 29 p^4 - p^6) / 384,
// which solves lap G = zeta_m for the Gaussian-Laguerre source; G(0) = -sqrt(2/pi) C_m /
// (4 pi eps) with C_m = 1, 3/2, 15/8, 35/16, 315/128 (the limit of the bracket / p).
// Truncated kernel: G = -Si(k_c r) / (2 pi^2 r), G(0) = -k_c / (2 pi^2).  Spectral form
// (no convolution direction): -zeta_hat(k) / k^2, zero at k = 0.
__device__ double hej_value(const GreenGen& g, double r, double k) {
  const double pi = 3.14159265358979323846;
  const int q = g.variant - 2;
  if (g.du == 3) {
    if (g.variant == 7)
      return r > 0.0 ? -sine_integral(g.kc * r) / (2.0 * pi * pi * r) : -g.kc / (2.0 * pi * pi);
    const double sq2pi = sqrt(2.0 / pi);
    if (r == 0.0) {
      const double cm[5] = {1.0, 1.5, 1.875, 2.1875, 2.4609375};
      return -sq2pi * cm[q] / (4.0 * pi * g.eps);
    }
    const double p = r / g.eps, p2 = p * p;
    double poly;
    switch (q) {
      case 0: poly = 0.0; break;
      case 1: poly = 0.5; break;
      case 2: poly = (7.0 - p2) / 8.0; break;
      case 3: poly = (57.0 + p2 * (-16.0 + p2)) / 48.0; break;
      default: poly = (561.0 + p2 * (-233.0 + p2 * (29.0 - p2))) / 384.0; break;
    }
    return -(erf(p / sqrt(2.0)) + sq2pi * p * exp(-0.5 * p2) * poly) / (4.0 * pi * r);
  }
  if (k == 0.0) return 0.0;
  if (g.variant == 7) return k <= g.kc * (1.0 + 1e-12) ? -1.0 / (k * k) : 0.0;
  const double s = 0.5 * (k * g.eps) * (k * g.eps);
  double term = 1.0, sum = 1.0;  // sum_{j <= q} s^j / j!
  for (int j = 1; j <= q; ++j) {
    term *= s / j;
    sum += term;
  }
  return -exp(-s) * sum / (k * k);
}

// ---------------------------------------------------------------------------------
// Lattice Green's function (FM_GREEN_LGF2): the Green's function of the second-difference
// Laplacian.  With the discrete heat kernel exp(-2t/h^2) I_n(2t/h^2) of each axis,
//   G(n) = -(1 / prod h) int_0^inf prod_a exp(-x_a) I_{n_a}(x_a) dt,   x_a = 2 t / h_a^2.
// The integral is taken with the trapezoidal rule in u = ln t after subtracting
// prod h (4 pi (t + c))^(-3/2) (the far field, integrated in closed form).  The scaled
// Bessel values of every node come from the power series (x < 1), Miller's backward
// recurrence normalised by exp(x) = I_0 + 2 sum I_k (moderate x), or the large-argument
// expansion (x >= 40 (n_max^2 + 10)).
// ---------------------------------------------------------------------------------
__global__ void lgf_bessel_kernel(double* A, LgfGen g) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 3 * g.K) return;
  const int a = id / g.K, k = id % g.K;
  const double t = exp(g.u_lo + k * g.du);
  scaled_bessel_row(2.0 * t / (g.h[a] * g.h[a]), g.nA[a], A + ((size_t)a * g.K + k) * g.stride);
}

// Node weights du t_k and far-field values prod h (4 pi (t_k + c))^(-3/2), k < K.
__global__ void lgf_weight_kernel(double* W, LgfGen g) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.K) return;
  const double pi = 3.14159265358979323846;
  const double t = exp(g.u_lo + k * g.du);
  W[k] = g.du * t;
  W[g.K + k] = g.h[0] * g.h[1] * g.h[2] * pow(4.0 * pi * (t + g.c), -1.5);
}

__global__ void lgf_sample_kernel(double* S, LgfGen g, const double* __restrict__ A,
                                  const double* __restrict__ W) {
  const int64_t total = (int64_t)g.nA[0] * g.nA[1] * g.nA[2];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int64_t r = e;
  const int i2 = (int)(r % g.nA[2]);
  r /= g.nA[2];
  const int i1 = (int)(r % g.nA[1]);
  const int i0 = (int)(r / g.nA[1]);
  const double pi = 3.14159265358979323846;
  const double ph = g.h[0] * g.h[1] * g.h[2];
  const double* a0 = A + i0;
  const double* a1 = A + (size_t)g.K * g.stride + i1;
  const double* a2 = A + (size_t)2 * g.K * g.stride + i2;
  double acc = 0.0;
  for (int k = 0; k < g.K; ++k) {
    const size_t o = (size_t)k * g.stride;
    acc += W[k] * (a0[o] * a1[o] * a2[o] - W[g.K + k]);
  }
  acc += ph * 2.0 * pow(4.0 * pi, -1.5) / sqrt(g.c);
  S[e] = -acc / ph;
}

__device__ double green_value(const GreenGen& g, double rho, double k) {
  const double pi = 3.14159265358979323846;
  if (g.variant == 8) return nan("");  // LGF2 is sampled by lgf_sample_kernel
  if (g.variant >= 2) return hej_value(g, rho, k);
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
  double r2 = 0.0, k2 = 0.0, s2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (g.unb[a]) {
      const double dd = idx[a] * g.h[a];
      r2 += dd * dd;
    } else {
      const double w = g.dw[a] * (idx[a] + g.shift[a]);
      k2 += w * w;
      const double sd = 2.0 * sin(0.5 * w * g.h[a]) / g.h[a];  // second-difference symbol
      s2 += sd * sd;
    }
  }
  if (g.variant == 8) {  // LGF2 without convolution directions: the inverse symbol
    S[e] = s2 > 0.0 ? -1.0 / s2 : 0.0;
    return;
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

bool is_fast_len(int M) {
  for (int m : kFastLens)
    if (m == M) return true;
  return false;
}

#define FM_LEN_CASES(T, CALL)       \
  case 32: return CALL(T, 32);      \
  case 48: return CALL(T, 48);      \
  case 64: return CALL(T, 64);      \
  case 96: return CALL(T, 96);      \
  case 128: return CALL(T, 128);    \
  case 192: return CALL(T, 192);    \
  case 256: return CALL(T, 256);    \
  case 384: return CALL(T, 384);    \
  case 512: return CALL(T, 512);    \
  case 768: return CALL(T, 768);    \
  case 1024: return CALL(T, 1024);  \
  case 2048: return CALL(T, 2048);  \
  case 4096: return CALL(T, 4096);

template <typename T>
hipError_t launch_pass(const PassDesc& d, const PassDesc* dev, const void* in, void* out,
                       hipStream_t st) {
  if (d.tiles <= 0) return hipSuccess;
  if (d.stw == nullptr) {
    if constexpr (sizeof(T) == 8)
      if (d.M > kMaxFastLen64 || d.long_rt) return launch_len<T, kRtLong>(d, dev, in, out, st);
    return launch_len<T, kRtShort>(d, dev, in, out, st);
  }
#define FM_CALL(TT, M) launch_len<TT, M>(d, dev, in, out, st)
  switch (d.M) {
    FM_LEN_CASES(T, FM_CALL)
    default: return launch_len<T, kRtShort>(d, dev, in, out, st);
  }
#undef FM_CALL
}

// All descriptors of one batched launch share the length class of ds_host[0].
template <typename T>
hipError_t launch_pass_batched(int len_class, const PassDesc* ds, const int* prefix, int n,
                               int total_tiles, int lds_bytes, hipStream_t st) {
  if (total_tiles <= 0) return hipSuccess;
#define FM_CALL(TT, M) launch_len_batched<TT, M>(ds, prefix, n, total_tiles, lds_bytes, st)
  switch (len_class) {
    FM_LEN_CASES(T, FM_CALL)
    case kRtLong:
      if constexpr (sizeof(T) == 8) return launch_len_batched<T, kRtLong>(ds, prefix, n, total_tiles, lds_bytes, st);
      return hipErrorInvalidValue;
    default: return launch_len_batched<T, kRtShort>(ds, prefix, n, total_tiles, lds_bytes, st);
  }
#undef FM_CALL
}

template <typename T>
hipError_t launch_twiddles(void* out, int M, hipStream_t st) {
  const int n = 4 * M;
  hipLaunchKernelGGL(twiddle_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<cpx<T>*>(out), M);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stage_twiddles(void* out, int M, hipStream_t st) {
  const int n = stage_table_size(M, max_radix((int)sizeof(T)));
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(stage_twiddle_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<cpx<T>*>(out), M);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wave_twiddles(void* out, int M, int E, hipStream_t st) {
  const int n = wave_tw_size(M, E);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(wave_twiddle_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<cpx<T>*>(out), M, E);
  return hipGetLastError();
}

// A: 3 K stride doubles (Bessel rows), W: 2 K doubles (node weights, far field).
hipError_t launch_lgf(double* S, double* A, double* W, const LgfGen& g, hipStream_t st) {
  hipLaunchKernelGGL(lgf_bessel_kernel, dim3((3 * g.K + 63) / 64), dim3(64), 0, st, A, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lgf_weight_kernel, dim3((g.K + 255) / 256), dim3(256), 0, st, W, g);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)g.nA[0] * g.nA[1] * g.nA[2];
  hipLaunchKernelGGL(lgf_sample_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, S, g, A, W);
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

// u_hat_p = G sum over (a, b) of eps_pab s_ab w_a psi_hat_b at every point of the real
// spectra (all three axes symmetric: every derivative is a real factor, Sec. V).
template <typename T>
__global__ void curl_real_kernel(CurlReal c) {
  const int64_t total = (int64_t)c.n[0] * c.n[1] * c.n[2];
  T* S = reinterpret_cast<T*>(c.S);
  const T* G = reinterpret_cast<const T*>(c.G);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i2 = i % c.n[2], r = i / c.n[2];
    const int64_t i1 = r % c.n[1], i0 = r / c.n[1];
    T w[3];  // derivative factor along physical axes x, y, z
    w[c.ax[0]] = reinterpret_cast<const T*>(c.d[0])[i0];
    w[c.ax[1]] = reinterpret_cast<const T*>(c.d[1])[i1];
    w[c.ax[2]] = reinterpret_cast<const T*>(c.d[2])[i2];
    const T f[3] = {S[i], S[i + c.comp_stride], S[i + 2 * c.comp_stride]};
    auto D = [&](int a, int b) { return T(c.sg[a][b]) * w[a] * f[b]; };  // d/dx_a of component b
    const T g = G[i];
    const T ux = D(1, 2) - D(2, 1), uy = D(2, 0) - D(0, 2), uz = D(0, 1) - D(1, 0);
    S[i] = g * ux;
    S[i + c.comp_stride] = g * uy;
    S[i + 2 * c.comp_stride] = g * uz;
  }
}

template <typename T>
hipError_t launch_curl_real(const CurlReal& c, hipStream_t st) {
  const int64_t total = (int64_t)c.n[0] * c.n[1] * c.n[2];
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(curl_real_kernel<T>, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, c);
  return hipGetLastError();
}

template hipError_t launch_curl_real<float>(const CurlReal&, hipStream_t);
template hipError_t launch_curl_real<double>(const CurlReal&, hipStream_t);
template hipError_t launch_pass<float>(const PassDesc&, const PassDesc*, const void*, void*, hipStream_t);
template hipError_t launch_pass<double>(const PassDesc&, const PassDesc*, const void*, void*, hipStream_t);
template hipError_t launch_pass_batched<float>(int, const PassDesc*, const int*, int, int, int, hipStream_t);
template hipError_t launch_pass_batched<double>(int, const PassDesc*, const int*, int, int, int, hipStream_t);
template hipError_t launch_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_wave_twiddles<float>(void*, int, int, hipStream_t);
template hipError_t launch_wave_twiddles<double>(void*, int, int, hipStream_t);
template hipError_t launch_stage_twiddles<float>(void*, int, hipStream_t);
template hipError_t launch_stage_twiddles<double>(void*, int, hipStream_t);
template hipError_t launch_green_final<float>(void*, const double*, const int*, const int*, const int*, double, hipStream_t);
template hipError_t launch_green_final<double>(void*, const double*, const int*, const int*, const int*, double, hipStream_t);

}  // namespace fm
