// Reference solver used ONLY as test infrastructure.
//
// A plain, slow, FP64 CPU implementation of the Fourier-convolution Poisson and
// Biot-Savart solve described in FLUPS (Balty, Chatelain, Gillis, arXiv 2211.07777).
// Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
// load this library.  It shares no code, header, table or constant with the GPU
// library; the two are written independently from the paper.
//
// Contents
//   * its own recursive mixed-radix Cooley-Tukey FFT (any length; a prime factor p is
//     combined with a p-point DFT written out as a sum),
//   * naive O(n^2) DFT and the eight real-to-real transforms exactly as their defining
//     sums (Sec. II-B gives the node-centred ones; the cell-centred ones are the
//     textbook DCT/DST-II, -III and -IV),
//   * the same real-to-real transforms computed as the DFT of the explicitly
//     symmetric-extended sequence (a textbook identity, used by the fast solve),
//   * the per-axis boundary-condition table (Table I, Sec. II-B, Sec. II-C),
//   * the CHAT2-family Green's functions in mixed spectral/physical space,
//   * three solve modes: "fast" (own FFT), "naive" (every transform replaced by its
//     defining sum) and "direct" (spectral directions by their defining sums,
//     unbounded directions by an explicit real-space convolution with images).
//
// Conventions (readings of the paper where it is silent are listed with each step):
//   forward transforms use exp(-i w x) and are unnormalised; backward transforms use
//   exp(+i w x); the product of the normalisation lengths is divided out once, after
//   the spectral multiplication.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cd = std::complex<double>;
const double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------------
// 1-D transforms
// ---------------------------------------------------------------------------------

// exp(sign * 2 pi i * m / n) with the integer m reduced modulo n first.
cd root_of_unity(long long m, long long n, int sign) {
  m %= n;
  if (m < 0) m += n;
  const double a = 2.0 * kPi * (double)m / (double)n;
  return cd(std::cos(a), sign * std::sin(a));
}

int smallest_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

// Table of exp(sign*2*pi*i*j/n), j = 0..n-1, built once per (n, sign).
const std::vector<cd>& roots_table(int n, int sign) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, std::vector<cd>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto key = std::make_pair(n, sign);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  std::vector<cd> t(n);
  for (int j = 0; j < n; ++j) t[j] = root_of_unity(j, n, sign);
  return cache.emplace(key, std::move(t)).first->second;
}

// Decimation in time: X[k + m q] = sum_r W_n^{r (k + m q)} S_r[k], where S_r is the
// length-m DFT of the sub-sequence x[p j + r].  `tw` holds W_n0^j for the top-level
// length n0; W_n^e = W_n0^(e * n0 / n).
void fft_rec(int n, const cd* in, long stride, cd* out, const std::vector<cd>& tw, int n0,
             cd* scratch) {
  if (n == 1) {
    out[0] = in[0];
    return;
  }
  const int p = smallest_factor(n);
  const int m = n / p;
  cd* sub = scratch;          // n values
  cd* deeper = scratch + n;   // scratch for the recursion
  for (int r = 0; r < p; ++r) fft_rec(m, in + r * stride, stride * p, sub + r * m, tw, n0, deeper);
  const long scale = n0 / n;
  for (int k = 0; k < m; ++k) {
    for (int q = 0; q < p; ++q) {
      cd acc = 0.0;
      for (int r = 0; r < p; ++r) {
        const long e = ((long)r * (long)(k + m * q)) % n;
        acc += sub[r * m + k] * tw[e * scale];
      }
      out[k + m * q] = acc;
    }
  }
}

// out[k] = sum_j in[j] exp(sign * 2 pi i j k / n)   (own FFT; sign -1 = forward)
void fft(int n, const cd* in, cd* out, int sign) {
  const std::vector<cd>& tw = roots_table(n, sign);
  std::vector<cd> scratch(4 * (size_t)n + 64);
  fft_rec(n, in, 1, out, tw, n, scratch.data());
}

// Same sum evaluated directly.
void dft_naive(int n, const cd* in, cd* out, int sign) {
  for (int k = 0; k < n; ++k) {
    cd acc = 0.0;
    for (int j = 0; j < n; ++j) acc += in[j] * root_of_unity((long long)j * k, n, sign);
    out[k] = acc;
  }
}

// Real-to-real kinds, numbered as FFTW numbers them.
enum R2R { REDFT00 = 0, REDFT01 = 1, REDFT10 = 2, REDFT11 = 3,
           RODFT00 = 4, RODFT01 = 5, RODFT10 = 6, RODFT11 = 7 };

// cos(pi * num / den) and sin(pi * num / den), num reduced modulo 2 den.
double cospi_frac(long long num, long long den) {
  num %= 2 * den;
  if (num < 0) num += 2 * den;
  return std::cos(kPi * (double)num / (double)den);
}
double sinpi_frac(long long num, long long den) {
  num %= 2 * den;
  if (num < 0) num += 2 * den;
  return std::sin(kPi * (double)num / (double)den);
}

// The defining sums (Sec. II-B for node data; textbook DCT/DST-II/III/IV for cells).
void r2r_naive(int kind, int n, const double* x, double* y) {
  for (int k = 0; k < n; ++k) {
    double acc = 0.0;
    switch (kind) {
      case REDFT00:  // y_k = x_0 + (-1)^k x_{n-1} + 2 sum_{j=1}^{n-2} x_j cos(pi j k/(n-1))
        if (n == 1) { acc = x[0]; break; }
        acc = x[0] + ((k % 2) ? -x[n - 1] : x[n - 1]);
        for (int j = 1; j <= n - 2; ++j) acc += 2.0 * x[j] * cospi_frac((long long)j * k, n - 1);
        break;
      case RODFT00:  // y_k = 2 sum_j x_j sin(pi (j+1)(k+1)/(n+1))
        for (int j = 0; j < n; ++j) acc += 2.0 * x[j] * sinpi_frac((long long)(j + 1) * (k + 1), n + 1);
        break;
      case REDFT10:  // y_k = 2 sum_j x_j cos(pi (j+1/2) k / n)
        for (int j = 0; j < n; ++j) acc += 2.0 * x[j] * cospi_frac((long long)(2 * j + 1) * k, 2LL * n);
        break;
      case REDFT01:  // y_k = x_0 + 2 sum_{j>=1} x_j cos(pi j (k+1/2) / n)
        acc = x[0];
        for (int j = 1; j < n; ++j) acc += 2.0 * x[j] * cospi_frac((long long)j * (2 * k + 1), 2LL * n);
        break;
      case REDFT11:  // y_k = 2 sum_j x_j cos(pi (j+1/2)(k+1/2) / n)
        for (int j = 0; j < n; ++j)
          acc += 2.0 * x[j] * cospi_frac((long long)(2 * j + 1) * (2 * k + 1), 4LL * n);
        break;
      case RODFT10:  // y_k = 2 sum_j x_j sin(pi (j+1/2)(k+1) / n)
        for (int j = 0; j < n; ++j) acc += 2.0 * x[j] * sinpi_frac((long long)(2 * j + 1) * (k + 1), 2LL * n);
        break;
      case RODFT01:  // y_k = (-1)^k x_{n-1} + 2 sum_{j=0}^{n-2} x_j sin(pi (j+1)(k+1/2) / n)
        acc = (k % 2) ? -x[n - 1] : x[n - 1];
        for (int j = 0; j <= n - 2; ++j)
          acc += 2.0 * x[j] * sinpi_frac((long long)(j + 1) * (2 * k + 1), 2LL * n);
        break;
      case RODFT11:  // y_k = 2 sum_j x_j sin(pi (j+1/2)(k+1/2) / n)
        for (int j = 0; j < n; ++j)
          acc += 2.0 * x[j] * sinpi_frac((long long)(2 * j + 1) * (2 * k + 1), 4LL * n);
        break;
    }
    y[k] = acc;
  }
}

// The same transforms as the DFT (own FFT) of an explicit symmetric extension.
void r2r_fft(int kind, int n, const double* x, double* y) {
  std::vector<cd> v, V;
  auto run = [&](int len) {
    V.assign(len, 0.0);
    fft(len, v.data(), V.data(), -1);
  };
  switch (kind) {
    case REDFT00: {  // even extension of period 2(n-1)
      if (n == 1) { y[0] = x[0]; return; }
      const int L = 2 * (n - 1);
      v.assign(L, 0.0);
      for (int j = 0; j < n; ++j) v[j] = x[j];
      for (int j = 1; j <= n - 2; ++j) v[L - j] = x[j];
      run(L);
      for (int k = 0; k < n; ++k) y[k] = V[k].real();
      return;
    }
    case RODFT00: {  // odd extension of period 2(n+1)
      const int L = 2 * (n + 1);
      v.assign(L, 0.0);
      for (int j = 0; j < n; ++j) { v[j + 1] = x[j]; v[L - j - 1] = -x[j]; }
      run(L);
      for (int k = 0; k < n; ++k) y[k] = -V[k + 1].imag();
      return;
    }
    case REDFT10: {  // samples at odd positions of a period-4n even sequence
      const int L = 4 * n;
      v.assign(L, 0.0);
      for (int j = 0; j < n; ++j) { v[2 * j + 1] = x[j]; v[L - 2 * j - 1] = x[j]; }
      run(L);
      for (int k = 0; k < n; ++k) y[k] = V[k].real();
      return;
    }
    case REDFT01: {  // even sequence of period 4n read at odd frequencies
      const int L = 4 * n;
      v.assign(L, 0.0);
      v[0] = x[0];
      for (int j = 1; j < n; ++j) { v[j] = x[j]; v[L - j] = x[j]; }
      run(L);
      for (int k = 0; k < n; ++k) y[k] = V[2 * k + 1].real();
      return;
    }
    case REDFT11: {  // period 8n, odd positions and odd frequencies
      const int L = 8 * n;
      v.assign(L, 0.0);
      for (int j = 0; j < n; ++j) {
        v[2 * j + 1] = x[j];
        v[L - 2 * j - 1] = x[j];
        v[4 * n + 2 * j + 1] = -x[j];
        v[4 * n - 2 * j - 1] = -x[j];
      }
      run(L);
      for (int k = 0; k < n; ++k) y[k] = 0.5 * V[2 * k + 1].real();
      return;
    }
    case RODFT10: {
      const int L = 4 * n;
      v.assign(L, 0.0);
      for (int j = 0; j < n; ++j) { v[2 * j + 1] = x[j]; v[L - 2 * j - 1] = -x[j]; }
      run(L);
      for (int k = 0; k < n; ++k) y[k] = -V[k + 1].imag();
      return;
    }
    case RODFT01: {
      const int L = 4 * n;
      v.assign(L, 0.0);
      for (int j = 0; j < n - 1; ++j) { v[j + 1] = x[j]; v[L - j - 1] = -x[j]; }
      v[n] += 0.5 * x[n - 1];          // the last sample enters with weight 1, not 2
      v[L - n] -= 0.5 * x[n - 1];
      run(L);
      for (int k = 0; k < n; ++k) y[k] = -V[2 * k + 1].imag();
      return;
    }
    case RODFT11: {
      const int L = 8 * n;
      v.assign(L, 0.0);
      for (int j = 0; j < n; ++j) {
        v[2 * j + 1] = x[j];
        v[L - 2 * j - 1] = -x[j];
        v[4 * n + 2 * j + 1] = -x[j];
        v[4 * n - 2 * j - 1] = x[j];
      }
      run(L);
      for (int k = 0; k < n; ++k) y[k] = -0.5 * V[2 * k + 1].imag();
      return;
    }
  }
}

// ---------------------------------------------------------------------------------
// Boundary conditions -> per-axis operations (Table I; Sec. II-B; Sec. II-C)
// ---------------------------------------------------------------------------------

enum BC { BC_EVEN = 0, BC_ODD = 1, BC_PER = 2, BC_UNB = 3 };
enum Cls { C_P, C_EE, C_OO, C_EO, C_OE, C_UU, C_EU, C_OU, C_UE, C_UO };
enum Mode { MODE_FAST = 0, MODE_NAIVE = 1, MODE_DIRECT = 2 };

struct Axis {
  int N = 0;        // cells (cell layout) or intervals (node layout)
  double h = 0;
  bool node = false;
  int cls = C_P;
  int nuser = 0;    // points the user holds on this axis
  bool unb = false; // convolution direction (fully or semi-unbounded)
  bool dft = false; // periodic or fully unbounded: complex DFT
  bool rev = false; // symmetric face on the right: work on the reversed line
  int fwd = 0, bwd = 0;   // real-to-real kinds (spectral and semi-unbounded axes)
  int first = 0;          // first line index fed to the transform
  int nin = 0;            // transform input length
  int nspec = 0;          // spectral length
  int kshift = 0;         // mode s pairs with frequency / kernel index s + kshift
  double half = 0.0;      // frequency offset (1/2 for the half-frequency transforms)
  double nlog = 1.0;      // normalisation length
  double L() const { return N * h; }
};

int classify(int bl, int br, int* cls) {
  if ((bl == BC_PER) != (br == BC_PER)) return -1;
  if (bl < 0 || bl > 3 || br < 0 || br > 3) return -1;
  if (bl == BC_PER) *cls = C_P;
  else if (bl == BC_UNB && br == BC_UNB) *cls = C_UU;
  else if (bl == BC_EVEN && br == BC_EVEN) *cls = C_EE;
  else if (bl == BC_ODD && br == BC_ODD) *cls = C_OO;
  else if (bl == BC_EVEN && br == BC_ODD) *cls = C_EO;
  else if (bl == BC_ODD && br == BC_EVEN) *cls = C_OE;
  else if (bl == BC_EVEN && br == BC_UNB) *cls = C_EU;
  else if (bl == BC_ODD && br == BC_UNB) *cls = C_OU;
  else if (bl == BC_UNB && br == BC_EVEN) *cls = C_UE;
  else *cls = C_UO;
  return 0;
}

int make_axis(int N, double h, int node, int bl, int br, Axis* a) {
  if (N < 2 || !(h > 0)) return -2;
  a->N = N;
  a->h = h;
  a->node = node != 0;
  if (classify(bl, br, &a->cls)) return -1;
  a->nuser = a->node ? N + 1 : N;
  const int c = a->cls;
  a->unb = (c >= C_UU);
  a->dft = (c == C_P || c == C_UU);
  a->rev = (c == C_UE || c == C_UO);
  switch (c) {
    case C_P:  // Eq. of the DFT in Sec. II-B; the node f_N is not used
      a->first = 0; a->nin = N; a->nspec = N; a->nlog = N; break;
    case C_UU:  // domain doubling: N (+1 for nodes) data, zeros up to 2N
      a->first = 0; a->nin = 2 * N; a->nspec = 2 * N; a->nlog = 2 * N; break;
    case C_EE:
      if (a->node) { a->fwd = a->bwd = REDFT00; a->first = 0; a->nin = N + 1; }
      else { a->fwd = REDFT10; a->bwd = REDFT01; a->first = 0; a->nin = N; }
      a->nspec = a->nin; a->nlog = 2 * N; break;
    case C_OO:
      if (a->node) { a->fwd = a->bwd = RODFT00; a->first = 1; a->nin = N - 1; a->kshift = 1; }
      else { a->fwd = RODFT10; a->bwd = RODFT01; a->first = 0; a->nin = N; a->kshift = 1; }
      a->nspec = a->nin; a->nlog = 2 * N; break;
    case C_EO:
      if (a->node) { a->fwd = REDFT01; a->bwd = REDFT10; a->first = 0; }
      else { a->fwd = a->bwd = REDFT11; a->first = 0; }
      a->nin = N; a->nspec = N; a->half = 0.5; a->nlog = 2 * N; break;
    case C_OE:
      if (a->node) { a->fwd = RODFT01; a->bwd = RODFT10; a->first = 1; }
      else { a->fwd = a->bwd = RODFT11; a->first = 0; }
      a->nin = N; a->nspec = N; a->half = 0.5; a->nlog = 2 * N; break;
    default: {  // semi-unbounded: pad the unbounded side to 2L, then DCT/DST (Sec. II-C)
      const bool even = (c == C_EU || c == C_UE);
      if (a->node) {
        if (even) { a->fwd = a->bwd = REDFT00; a->first = 0; a->nin = 2 * N + 1; a->kshift = 0; }
        else { a->fwd = a->bwd = RODFT00; a->first = 1; a->nin = 2 * N - 1; a->kshift = 1; }
      } else {
        if (even) { a->fwd = REDFT10; a->bwd = REDFT01; a->kshift = 0; }
        else { a->fwd = RODFT10; a->bwd = RODFT01; a->kshift = 1; }
        a->first = 0; a->nin = 2 * N;
      }
      a->nspec = a->nin; a->nlog = 4 * N; break;
    }
  }
  return 0;
}

// Wavenumber of spectral mode s on a spectral axis (periodic or symmetric), of the
// doubled-domain DFT mode s on a fully unbounded axis, or of the DCT / DST mode s on the
// 2L extension of a semi-unbounded axis (the last two used by the curl).  The Nyquist
// mode of an even-length DFT gets 0 when `nyquist_zero` is set.
double omega(const Axis& a, int s, bool nyquist_zero) {
  if (a.dft) {
    const int n = a.nspec;
    const double period = (a.cls == C_P) ? a.L() : 2.0 * a.L();
    if (2 * s == n && nyquist_zero) return 0.0;
    const int k = (2 * s > n) ? s - n : s;
    return 2.0 * kPi * k / period;
  }
  return kPi * (s + a.kshift + a.half) / (a.unb ? 2.0 * a.L() : a.L());
}

// Forward operation along one axis: user line (nuser) -> spectral line (nspec).
void axis_forward(const Axis& a, const cd* in, cd* out, int mode) {
  std::vector<cd> line(a.nuser);
  for (int j = 0; j < a.nuser; ++j) line[j] = in[a.rev ? a.nuser - 1 - j : j];
  if (a.dft) {
    std::vector<cd> v(a.nin, 0.0);
    const int ndata = (a.cls == C_P) ? a.N : a.nuser;
    for (int j = 0; j < ndata; ++j) v[j] = line[j];
    if (mode == MODE_FAST) fft(a.nin, v.data(), out, -1);
    else dft_naive(a.nin, v.data(), out, -1);
    return;
  }
  std::vector<double> xr(a.nin, 0.0), xi(a.nin, 0.0), yr(a.nin), yi(a.nin);
  for (int t = 0; t < a.nin; ++t) {
    const int j = a.first + t;
    if (j < a.nuser) { xr[t] = line[j].real(); xi[t] = line[j].imag(); }
  }
  if (mode == MODE_FAST) { r2r_fft(a.fwd, a.nin, xr.data(), yr.data()); r2r_fft(a.fwd, a.nin, xi.data(), yi.data()); }
  else { r2r_naive(a.fwd, a.nin, xr.data(), yr.data()); r2r_naive(a.fwd, a.nin, xi.data(), yi.data()); }
  for (int t = 0; t < a.nspec; ++t) out[t] = cd(yr[t], yi[t]);
}

// Backward operation (unnormalised): spectral line -> user line, with the crop and the
// fix-ups of Sec. II-A/II-B (odd-face nodes are zero, the periodic node f_N = f_0).
void axis_backward(const Axis& a, const cd* in, cd* out, int mode) {
  std::vector<cd> line(a.nuser, 0.0);
  if (a.dft) {
    std::vector<cd> v(a.nin);
    if (mode == MODE_FAST) fft(a.nin, in, v.data(), +1);
    else dft_naive(a.nin, in, v.data(), +1);
    if (a.cls == C_P) {
      for (int j = 0; j < a.N; ++j) line[j] = v[j];
      if (a.node) line[a.N] = v[0];
    } else {
      for (int j = 0; j < a.nuser; ++j) line[j] = v[j];
    }
  } else {
    std::vector<double> xr(a.nspec), xi(a.nspec), yr(a.nin), yi(a.nin);
    for (int t = 0; t < a.nspec; ++t) { xr[t] = in[t].real(); xi[t] = in[t].imag(); }
    if (mode == MODE_FAST) { r2r_fft(a.bwd, a.nin, xr.data(), yr.data()); r2r_fft(a.bwd, a.nin, xi.data(), yi.data()); }
    else { r2r_naive(a.bwd, a.nin, xr.data(), yr.data()); r2r_naive(a.bwd, a.nin, xi.data(), yi.data()); }
    for (int t = 0; t < a.nin; ++t) {
      const int j = a.first + t;
      if (j < a.nuser) line[j] = cd(yr[t], yi[t]);
    }
    // the face nodes that an odd condition pins to zero
    if (a.node) {
      const int c = a.cls;
      if (c == C_OO) { line[0] = 0.0; line[a.N] = 0.0; }
      if (c == C_EO) line[a.N] = 0.0;
      if (c == C_OE || c == C_OU || c == C_UO) line[0] = 0.0;
    }
  }
  for (int j = 0; j < a.nuser; ++j) out[a.rev ? a.nuser - 1 - j : j] = line[j];
}

// ---------------------------------------------------------------------------------
// Green's functions (CHAT2 family), mixed spectral / physical space
// ---------------------------------------------------------------------------------
// d_u = number of convolution (unbounded or semi-unbounded) directions, rho = distance
// in those directions, k = magnitude of the wavevector over the spectral directions.
//   d_u = 3: -1/(4 pi r)
//   d_u = 2: -K0(k rho)/(2 pi)   (k > 0);    ln(rho)/(2 pi)   (k = 0)
//   d_u = 1: -exp(-k|z|)/(2k)     (k > 0);    |z|/2            (k = 0)
//   d_u = 0: -1/k^2 in spectral space, 0 at k = 0
// The singular value at the origin (the "regularisation at the origin", Sec. II):
//   d_u = 3, green 0: equal-volume-sphere mean of -1/(4 pi r), multiplied by the cell
//            volume (this reading reproduces the printed CHAT2 errors of Sec. IV),
//   d_u = 3, green 1: the equal-volume-sphere mean itself, -3/(8 pi r_eq),
//   d_u = 2, k = 0:  (pi - 6 + 2 ln(pi r_eq^2 / 2)) / (8 pi), the corrected expression
//            of the footnote in Sec. V (the square-cell mean of ln(rho)/(2 pi)),
//   d_u = 2, k > 0:  the mean of -K0(k rho)/(2 pi) over the disc of area hx*hy.
// Regularised kernels (Sec. IV names them HEJ2 ... HEJ10 and HEJ0 after Hejlesen et al.;
// their formulas are in that work, not in the paper).  Order m = 2 q + 2 smooths the
// point source with the Gaussian-Laguerre function
//   zeta_m(x) = (2 pi eps^2)^(-3/2) exp(-rho^2 / 2) L_q^(3/2)(rho^2 / 2),  rho = |x| / eps,
// whose moments vanish up to order m; its Fourier transform is
//   exp(-s) sum_{j < m/2} s^j / j!,  s = (k eps)^2 / 2.
// The kernel -(1/4 pi r) * [erf(rho / sqrt 2) + sqrt(2/pi) rho exp(-rho^2/2) P_m(rho^2)]
// solves lap G = zeta_m (P_m below follows from integrating the radial equation
// twice); its origin value is -sqrt(2/pi) c_m / (4 pi eps).  HEJ0 cuts the spectrum off
// at the sphere |k| <= pi / h: G = -Si(pi r / h) / (2 pi^2 r), G(0) = -1 / (2 pi h).
// With eps = 2 h these reproduce the printed convergence of every HEJ kernel.
const double kHejPoly[5][4] = {{0, 0, 0, 0},
                               {0.5, 0, 0, 0},
                               {7.0 / 8.0, -1.0 / 8.0, 0, 0},
                               {19.0 / 16.0, -1.0 / 3.0, 1.0 / 48.0, 0},
                               {187.0 / 128.0, -233.0 / 384.0, 29.0 / 384.0, -1.0 / 384.0}};
const double kHejOrigin[5] = {1.0, 1.5, 15.0 / 8.0, 35.0 / 16.0, 315.0 / 128.0};

// Gauss-Legendre nodes and weights on [-1, 1] (Newton's method on P_n).
void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
  x->resize(n);
  w->resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    (*x)[i] = z;
    (*w)[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Si(x) = int_0^x sin(t)/t dt, x >= 0, by 24-point Gauss-Legendre on panels [j pi,
// (j+1) pi] (whole panels summed once and cached) plus the last partial panel.
double sine_integral(double x) {
  static std::mutex mu;
  static std::vector<double> gx, gw, prefix{0.0};
  auto panel = [&](double a, double b) {
    double acc = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) {
      const double t = 0.5 * (a + b) + 0.5 * (b - a) * gx[i];
      acc += gw[i] * std::sin(t) / t;
    }
    return 0.5 * (b - a) * acc;
  };
  std::lock_guard<std::mutex> lock(mu);
  if (gx.empty()) gauss_legendre(24, &gx, &gw);
  const long j = (long)(x / kPi);
  while ((long)prefix.size() <= j) {
    const long m = (long)prefix.size() - 1;
    prefix.push_back(prefix.back() + panel(m * kPi, (m + 1) * kPi));
  }
  return prefix[j] + (x > j * kPi ? panel(j * kPi, x) : 0.0);
}

struct Green {
  int du = 0;
  int variant = 0;
  double cellvol = 1.0;  // product of h over the convolution directions
  double r_eq = 0.0;
  double eps = 0.0;      // HEJ2..10: regularisation length 2 h
  double kc = 0.0;       // HEJ0: spectral cut-off pi / h
  // LGF2 (variant 8): the lattice Green's function at integer offsets 0 .. lgf_n[a] - 1
  // along each axis (x fastest), supplied by the caller (oracle/lgf.py)
  const double* lgf = nullptr;
  long lgf_n[3] = {0, 0, 0};
  double lattice(long m0, long m1, long m2) const {
    m0 = std::labs(m0);
    m1 = std::labs(m1);
    m2 = std::labs(m2);
    if (!lgf || m0 >= lgf_n[0] || m1 >= lgf_n[1] || m2 >= lgf_n[2]) return std::nan("");
    return lgf[m0 + lgf_n[0] * (m1 + lgf_n[1] * m2)];
  }
  double value(double rho, double k) const {
    if (variant == 8) return std::nan("");  // LGF2: sampled by offset (lattice) or symbol
    if (variant >= 2) return hej(rho, k);
    if (du == 3) {
      if (rho > 0) return -1.0 / (4.0 * kPi * rho);
      const double s = -3.0 / (8.0 * kPi * r_eq);
      return variant == 0 ? s * cellvol : s;
    }
    if (du == 2) {
      if (k == 0.0) {
        if (rho > 0) return std::log(rho) / (2.0 * kPi);
        return (kPi - 6.0 + 2.0 * std::log(kPi * r_eq * r_eq / 2.0)) / (8.0 * kPi);
      }
      if (rho > 0) return -std::cyl_bessel_k(0.0, k * rho) / (2.0 * kPi);
      const double x = k * r_eq;
      return -(1.0 - x * std::cyl_bessel_k(1.0, x)) / (kPi * x * x);
    }
    if (du == 1) {
      if (k == 0.0) return 0.5 * rho;
      return -std::exp(-k * rho) / (2.0 * k);
    }
    return (k == 0.0) ? 0.0 : -1.0 / (k * k);
  }
  // variant 2..6: HEJ2..HEJ10; variant 7: HEJ0.  Three convolution directions (mixed
  // space = real space) or none (spectral); the mixed forms are not built.
  double hej(double r, double k) const {
    const int q = variant - 2;  // 0..4 for HEJ2..HEJ10
    if (du == 3) {
      if (variant == 7) {
        if (r > 0) return -sine_integral(kc * r) / (2.0 * kPi * kPi * r);
        return -kc / (2.0 * kPi * kPi);
      }
      const double c = std::sqrt(2.0 / kPi);
      if (r == 0.0) return -c * kHejOrigin[q] / (4.0 * kPi * eps);
      const double p = r / eps, p2 = p * p;
      double poly = 0.0;
      for (int i = 3; i >= 0; --i) poly = poly * p2 + kHejPoly[q][i];
      return -(std::erf(p / std::sqrt(2.0)) + c * p * std::exp(-0.5 * p2) * poly) / (4.0 * kPi * r);
    }
    // spectral: -zeta_hat(k) / k^2
    if (k == 0.0) return 0.0;
    // modes on the cut-off sphere (the Nyquist modes of an even periodic grid lie on it)
    // are kept: a relative margin keeps the rounding of |k| from deciding
    if (variant == 7) return k <= kc * (1.0 + 1e-12) ? -1.0 / (k * k) : 0.0;
    const double sv = 0.5 * (k * eps) * (k * eps);
    double term = 1.0, sum = 1.0;
    for (int j = 1; j <= q; ++j) {
      term *= sv / j;
      sum += term;
    }
    return -std::exp(-sv) * sum / (k * k);
  }
};

// ---------------------------------------------------------------------------------
// 3-D helpers: arrays are [z][y][x], x fastest.
// ---------------------------------------------------------------------------------
struct Dims { long n[3]; long size() const { return n[0] * n[1] * n[2]; } };

// Apply `fn(in_line, out_line)` along axis `ax` for every line.
template <class F>
void along_axis(int ax, const Dims& din, const std::vector<cd>& in, const Dims& dout,
                std::vector<cd>& out, F fn) {
  const long sin_[3] = {1, din.n[0], din.n[0] * din.n[1]};
  const long sout[3] = {1, dout.n[0], dout.n[0] * dout.n[1]};
  const int o1 = (ax == 0) ? 1 : 0, o2 = (ax == 2) ? 1 : 2;
  const long n1 = din.n[o1], n2 = din.n[o2];
  const long lin = din.n[ax], lout = dout.n[ax];
#pragma omp parallel
  {
    std::vector<cd> a(lin), b(lout);
#pragma omp for collapse(2) schedule(static)
    for (long i2 = 0; i2 < n2; ++i2)
      for (long i1 = 0; i1 < n1; ++i1) {
        const long bi = i1 * sin_[o1] + i2 * sin_[o2];
        const long bo = i1 * sout[o1] + i2 * sout[o2];
        for (long t = 0; t < lin; ++t) a[t] = in[bi + t * sin_[ax]];
        fn(a.data(), b.data());
        for (long t = 0; t < lout; ++t) out[bo + t * sout[ax]] = b[t];
      }
  }
}

// x (axis 0), y (axis 1), z (axis 2) descriptors.
struct Problem {
  Axis ax[3];
  int du = 0;
  Green g;
  int kind = 0;  // 0 Poisson, 1 Biot-Savart with spectral curl, 2 / 3 / 4 Biot-Savart with
                 // the finite-difference derivative of order 2 / 4 / 6 (Sec. V)
};

// The lattice Green's function table of the next solves (oracle_set_lgf).
const double* g_lgf = nullptr;
long g_lgf_n[3] = {0, 0, 0};

int make_problem(const int* n, const double* h, const int* bc, int layout, int green, int kind,
                 Problem* P) {
  for (int a = 0; a < 3; ++a) {
    const int rc = make_axis(n[a], h[a], layout, bc[2 * a], bc[2 * a + 1], &P->ax[a]);
    if (rc) return rc;
  }
  if (green < 0 || green > 8) return -3;
  if (kind < 0 || kind > 4) return -3;
  P->kind = kind;
  if (kind >= 1)
    for (int a = 0; a < 3; ++a)
      if (!P->ax[a].dft) return -3;  // spectral curl on periodic / fully unbounded axes only
  P->du = 0;
  double vol = 1.0;
  for (int a = 0; a < 3; ++a)
    if (P->ax[a].unb) { P->du++; vol *= P->ax[a].h; }
  P->g.du = P->du;
  P->g.variant = green;
  P->g.cellvol = vol;
  if (P->du == 3) P->g.r_eq = std::cbrt(3.0 * vol / (4.0 * kPi));
  if (P->du == 2) P->g.r_eq = std::sqrt(vol / kPi);
  if (green == 8) {
    // lattice Green's function: three convolution directions (the table covers offsets
    // up to 2N along each) or none (the inverse of the second-difference symbol)
    if (P->du == 1 || P->du == 2) return -3;
    if (P->du == 3) {
      if (!g_lgf) return -6;
      for (int a = 0; a < 3; ++a)
        if (g_lgf_n[a] < 2L * P->ax[a].N + 1) return -6;
      P->g.lgf = g_lgf;
      for (int a = 0; a < 3; ++a) P->g.lgf_n[a] = g_lgf_n[a];
    }
    return 0;
  }
  if (green >= 2) {
    // regularised kernels: three convolution directions or none; the grid spacing is
    // the cube root of the cell volume (the spacing itself on isotropic grids)
    if (P->du == 1 || P->du == 2) return -3;
    const double hc = std::cbrt(P->ax[0].h * P->ax[1].h * P->ax[2].h);
    P->g.eps = 2.0 * hc;
    P->g.kc = kPi / hc;
  }
  return 0;
}

// Green's spectrum on the spectral grid (nspec per axis): sample the kernel on the
// extended physical grid of every convolution direction, then transform those
// directions (Sec. II-C: the fully unbounded kernel is symmetrised about L and DFT'ed
// on 2L; the semi-unbounded kernel is evaluated on [0, 2L] and DCT'ed).  Includes the
// quadrature weight (cell volume) and 1 / prod(nlog).
std::vector<cd> green_spectrum(const Problem& P, int mode) {
  Dims ds;
  long ext[3];
  for (int a = 0; a < 3; ++a) {
    const Axis& A = P.ax[a];
    if (!A.unb) ext[a] = A.nspec;
    else if (A.cls == C_UU) ext[a] = 2 * A.N;
    else ext[a] = 2 * A.N + 1;
    ds.n[a] = ext[a];
  }
  std::vector<cd> G(ds.size());
#pragma omp parallel for collapse(2) schedule(static)
  for (long z = 0; z < ext[2]; ++z)
    for (long y = 0; y < ext[1]; ++y)
      for (long x = 0; x < ext[0]; ++x) {
        const long idx[3] = {x, y, z};
        double k2 = 0.0, r2 = 0.0, s2 = 0.0;
        long off[3] = {0, 0, 0};
        for (int a = 0; a < 3; ++a) {
          const Axis& A = P.ax[a];
          if (!A.unb) {
            const double w = omega(A, (int)idx[a], false);
            k2 += w * w;
            const double d = 2.0 * std::sin(0.5 * w * A.h) / A.h;  // second-difference symbol
            s2 += d * d;
          } else {
            long m = idx[a];
            if (A.cls == C_UU && m > A.N) m = 2 * A.N - m;  // symmetrised about L
            off[a] = m;
            const double d = m * A.h;
            r2 += d * d;
          }
        }
        double gv;
        if (P.g.variant == 8) gv = P.du == 3 ? P.g.lattice(off[0], off[1], off[2]) : (s2 > 0.0 ? -1.0 / s2 : 0.0);
        else gv = P.g.value(std::sqrt(r2), std::sqrt(k2));
        G[x + ext[0] * (y + ext[1] * z)] = gv;
      }
  // transform the convolution directions
  Dims cur = ds;
  for (int a = 0; a < 3; ++a) {
    const Axis& A = P.ax[a];
    if (!A.unb) continue;
    Dims nd = cur;
    nd.n[a] = A.nspec;
    std::vector<cd> out(nd.size());
    if (A.cls == C_UU) {
      along_axis(a, cur, G, nd, out, [&](const cd* i, cd* o) {
        if (mode == MODE_FAST) fft(2 * A.N, i, o, -1);
        else dft_naive(2 * A.N, i, o, -1);
        for (int t = 0; t < 2 * A.N; ++t) o[t] = o[t].real();  // even kernel: real spectrum
      });
    } else {
      along_axis(a, cur, G, nd, out, [&](const cd* i, cd* o) {
        const int n = 2 * A.N + 1;
        std::vector<double> xr(n), yr(n), xi(n), yi(n);
        for (int t = 0; t < n; ++t) { xr[t] = i[t].real(); xi[t] = i[t].imag(); }
        if (mode == MODE_FAST) { r2r_fft(REDFT00, n, xr.data(), yr.data()); r2r_fft(REDFT00, n, xi.data(), yi.data()); }
        else { r2r_naive(REDFT00, n, xr.data(), yr.data()); r2r_naive(REDFT00, n, xi.data(), yi.data()); }
        // "common indexing": spectral mode s of the data pairs with kernel index s+kshift
        for (int s = 0; s < A.nspec; ++s) o[s] = cd(yr[s + A.kshift], yi[s + A.kshift]);
      });
    }
    G.swap(out);
    cur = nd;
  }
  double scale = 1.0;
  for (int a = 0; a < 3; ++a) {
    scale /= P.ax[a].nlog;
    if (P.ax[a].unb) scale *= P.ax[a].h;
  }
  for (auto& v : G) v *= scale;
  return G;
}

Dims user_dims(const Problem& P) { return Dims{{P.ax[0].nuser, P.ax[1].nuser, P.ax[2].nuser}}; }

std::vector<cd> forward3(const Problem& P, const std::vector<cd>& f, int mode) {
  Dims cur = user_dims(P);
  std::vector<cd> a = f;
  for (int ax = 0; ax < 3; ++ax) {
    Dims nd = cur;
    nd.n[ax] = P.ax[ax].nspec;
    std::vector<cd> b(nd.size());
    along_axis(ax, cur, a, nd, b, [&](const cd* i, cd* o) { axis_forward(P.ax[ax], i, o, mode); });
    a.swap(b);
    cur = nd;
  }
  return a;
}

std::vector<cd> backward3(const Problem& P, const std::vector<cd>& fh, int mode) {
  Dims cur{{P.ax[0].nspec, P.ax[1].nspec, P.ax[2].nspec}};
  std::vector<cd> a = fh;
  for (int ax = 2; ax >= 0; --ax) {
    Dims nd = cur;
    nd.n[ax] = P.ax[ax].nuser;
    std::vector<cd> b(nd.size());
    along_axis(ax, cur, a, nd, b, [&](const cd* i, cd* o) { axis_backward(P.ax[ax], i, o, mode); });
    a.swap(b);
    cur = nd;
  }
  return a;
}

// Transform-based solve (fast: own FFT; naive: defining sums).
int solve_spectral(const Problem& P, const double* rhs, double* out, int mode) {
  const Dims du = user_dims(P);
  const long V = du.size();
  const std::vector<cd> G = green_spectrum(P, mode);
  const int ncomp = (P.kind >= 1) ? 3 : 1;
  std::vector<std::vector<cd>> fh(ncomp);
  for (int c = 0; c < ncomp; ++c) {
    std::vector<cd> f(V);
    for (long i = 0; i < V; ++i) f[i] = rhs[c * V + i];
    fh[c] = forward3(P, f, mode);
  }
  const long nx = P.ax[0].nspec, ny = P.ax[1].nspec, nz = P.ax[2].nspec;
  if (P.kind == 0) {
    for (long i = 0; i < nx * ny * nz; ++i) fh[0][i] *= G[i];
  } else {
    // u_hat = G_hat * (i w x f_hat)   (Sec. V); the finite-difference forms replace the
    // wavenumber w of each axis by its central-difference symbol
    const cd I(0.0, 1.0);
    auto deriv = [&](const Axis& A, int s) {
      const double w = omega(A, s, true);
      if (P.kind == 1) return w;
      const double wh = omega(A, s, false) * A.h;  // the symbols vanish at the Nyquist mode
      if (P.kind == 2) return std::sin(wh) / A.h;
      if (P.kind == 3) return (4.0 / 3.0 * std::sin(wh) - 1.0 / 6.0 * std::sin(2.0 * wh)) / A.h;
      return (1.5 * std::sin(wh) - 0.3 * std::sin(2.0 * wh) + std::sin(3.0 * wh) / 30.0) / A.h;
    };
#pragma omp parallel for collapse(2) schedule(static)
    for (long z = 0; z < nz; ++z)
      for (long y = 0; y < ny; ++y)
        for (long x = 0; x < nx; ++x) {
          const long i = x + nx * (y + ny * z);
          const double wx = deriv(P.ax[0], (int)x);
          const double wy = deriv(P.ax[1], (int)y);
          const double wz = deriv(P.ax[2], (int)z);
          const cd fx = fh[0][i], fy = fh[1][i], fz = fh[2][i];
          fh[0][i] = G[i] * I * (wy * fz - wz * fy);
          fh[1][i] = G[i] * I * (wz * fx - wx * fz);
          fh[2][i] = G[i] * I * (wx * fy - wy * fx);
        }
  }
  for (int c = 0; c < ncomp; ++c) {
    const std::vector<cd> u = backward3(P, fh[c], mode);
    for (long i = 0; i < V; ++i) out[c * V + i] = u[i].real();
  }
  return 0;
}

// Biot-Savart with boundary conditions per component (Sec. V).  A derivative along a
// symmetric direction turns an even field odd and an odd one even, so component p of the
// velocity takes, face by face, the opposite symmetry of component p of the source, and
// its backward transform is the swapped DCT / DST.  Periodic and unbounded faces are
// shared by the three components; on a symmetric face of axis a the component along a
// has one symmetry and the two others the opposite one (the faces of a mirror-symmetric
// vector field), otherwise the problem is rejected (-1).
// bcv[18] = per component q (x, y, z), per axis a, (left, right): bcv[6 q + 2 a + f].
int swap_face(int b) { return b == BC_EVEN ? BC_ODD : (b == BC_ODD ? BC_EVEN : b); }

int vector_faces_ok(const int* bcv) {
  for (int a = 0; a < 3; ++a)
    for (int f = 0; f < 2; ++f) {
      const int t[3] = {bcv[2 * a + f], bcv[6 + 2 * a + f], bcv[12 + 2 * a + f]};
      const bool sym = t[0] <= BC_ODD || t[1] <= BC_ODD || t[2] <= BC_ODD;
      if (!sym) {
        if (t[0] != t[1] || t[0] != t[2]) return -1;
        continue;
      }
      const int b = (a + 1) % 3, c = (a + 2) % 3;  // the two tangential components
      if (t[a] > BC_ODD || t[b] > BC_ODD || t[c] > BC_ODD) return -1;
      if (t[b] != t[c] || t[a] == t[b]) return -1;
    }
  return 0;
}

// Each component is transformed with its own conditions and multiplied by the Green's
// spectrum in its own indexing (psi_hat_b = G_hat f_hat_b).  Coefficients of one frequency
// index K sit at index K - kshift of every spectrum, so that u_hat_p at the index of
// frequency K gathers the psi_hat_b of the same K.  The derivative along a periodic or
// unbounded direction is i w (Sec. V); along a symmetric or semi-unbounded one the
// coefficient of a sine transform stands for the complex value -i times it, so the
// derivative is +w times it, and a cosine coefficient's derivative is -w times it (that
// value, with the sign changed for the backward sine transform); on a reversed axis (a
// semi-unbounded one symmetric on the right) both signs flip.  The finite-difference
// kinds replace w by their symbols.
int solve_vector(const Problem Pin[3], const Problem Pout[3], int kind, const double* rhs,
                 double* out, int mode) {
  const Dims du = user_dims(Pin[0]);
  const long V = du.size();
  std::vector<std::vector<cd>> psi(3);
  for (int b = 0; b < 3; ++b) {
    std::vector<cd> f(V);
    for (long i = 0; i < V; ++i) f[i] = rhs[b * V + i];
    psi[b] = forward3(Pin[b], f, mode);
    const std::vector<cd> G = green_spectrum(Pin[b], mode);
    for (size_t i = 0; i < psi[b].size(); ++i) psi[b][i] *= G[i];
  }
  auto deriv = [&](const Axis& A, int s) {
    const double w = omega(A, s, true);
    if (kind == 1) return w;
    const double wh = omega(A, s, false) * A.h;
    if (kind == 2) return std::sin(wh) / A.h;
    if (kind == 3) return (4.0 / 3.0 * std::sin(wh) - 1.0 / 6.0 * std::sin(2.0 * wh)) / A.h;
    return (1.5 * std::sin(wh) - 0.3 * std::sin(2.0 * wh) + std::sin(3.0 * wh) / 30.0) / A.h;
  };
  auto is_sine = [](int k) { return k >= RODFT00; };
  const cd I(0.0, 1.0);
  for (int p = 0; p < 3; ++p) {
    const Problem& Q = Pout[p];
    const long nx = Q.ax[0].nspec, ny = Q.ax[1].nspec, nz = Q.ax[2].nspec;
    std::vector<cd> uh(nx * ny * nz);
    // u_p = D_a psi_b - D_b psi_a with (p, a, b) cyclic
    const int a = (p + 1) % 3, b = (p + 2) % 3;
    // D_e psi_c at output index s[3]
    auto term = [&](int e, int c, const long* s) -> cd {
      long t[3];
      for (int x = 0; x < 3; ++x) {
        const Axis& Ao = Q.ax[x];
        const Axis& Ai = Pin[c].ax[x];
        t[x] = Ao.dft ? s[x] : s[x] + Ao.kshift - Ai.kshift;
        if (t[x] < 0 || t[x] >= Ai.nspec) return cd(0.0, 0.0);
      }
      const long ni0 = Pin[c].ax[0].nspec, ni1 = Pin[c].ax[1].nspec;
      const cd v = psi[c][t[0] + ni0 * (t[1] + ni1 * t[2])];
      const double w = deriv(Q.ax[e], (int)s[e]);
      if (Q.ax[e].dft) return I * w * v;
      // a symmetric face on the right: the transforms see the reversed line x' = L - x,
      // and d/dx = -d/dx'
      const double sg = (is_sine(Pin[c].ax[e].fwd) ? 1.0 : -1.0) * (Q.ax[e].rev ? -1.0 : 1.0);
      return sg * w * v;
    };
#pragma omp parallel for collapse(2) schedule(static)
    for (long z = 0; z < nz; ++z)
      for (long y = 0; y < ny; ++y)
        for (long x = 0; x < nx; ++x) {
          const long s[3] = {x, y, z};
          uh[x + nx * (y + ny * z)] = term(a, b, s) - term(b, a, s);
        }
    const std::vector<cd> u = backward3(Q, uh, mode);
    for (long i = 0; i < V; ++i) out[p * V + i] = u[i].real();
  }
  return 0;
}

// Direct form: spectral directions by their defining sums, convolution directions as an
// explicit sum over the user's points and their images (even image: same sign, odd
// image: opposite sign; a node on the symmetric face is its own image and counts once).
int solve_direct(const Problem& P, const double* rhs, double* out) {
  if (P.kind != 0) return -3;
  const Dims du = user_dims(P);
  const long V = du.size();
  // 1) forward defining sums along spectral directions only
  std::vector<cd> a(V);
  for (long i = 0; i < V; ++i) a[i] = rhs[i];
  Dims cur = du;
  for (int ax = 0; ax < 3; ++ax) {
    if (P.ax[ax].unb) continue;
    Dims nd = cur;
    nd.n[ax] = P.ax[ax].nspec;
    std::vector<cd> b(nd.size());
    along_axis(ax, cur, a, nd, b, [&](const cd* i, cd* o) { axis_forward(P.ax[ax], i, o, MODE_NAIVE); });
    a.swap(b);
    cur = nd;
  }
  // 2) source points of each convolution direction, with their images
  struct Src { int j; double x; double sign; };
  std::vector<Src> src[3];
  for (int ax = 0; ax < 3; ++ax) {
    const Axis& A = P.ax[ax];
    if (!A.unb) continue;
    const double off = A.node ? 0.0 : 0.5;
    if (A.cls == C_UU) {
      for (int j = 0; j < A.nuser; ++j) src[ax].push_back({j, (j + off) * A.h, 1.0});
      continue;
    }
    const double sgn = (A.cls == C_EU || A.cls == C_UE) ? 1.0 : -1.0;
    const double face = A.rev ? A.L() : 0.0;  // position of the symmetric face
    for (int j = 0; j < A.nuser; ++j) {
      const double x = (j + off) * A.h;
      const double xi = 2.0 * face - x;
      if (A.node && std::fabs(xi - x) < 0.25 * A.h) {
        // a node on the symmetric face is its own image: counted once (even face), or
        // pinned to zero (odd face)
        if (sgn > 0) src[ax].push_back({j, x, 1.0});
        continue;
      }
      src[ax].push_back({j, x, 1.0});
      src[ax].push_back({j, xi, sgn});
    }
  }
  double cellvol = 1.0;
  for (int ax = 0; ax < 3; ++ax)
    if (P.ax[ax].unb) cellvol *= P.ax[ax].h;
  // 3) convolution per spectral mode
  std::vector<cd> b(cur.size(), 0.0);
  const long n0 = cur.n[0], n1 = cur.n[1], n2 = cur.n[2];
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (long z = 0; z < n2; ++z)
    for (long y = 0; y < n1; ++y)
      for (long x = 0; x < n0; ++x) {
        const long idx[3] = {x, y, z};
        double k2 = 0.0, s2 = 0.0;
        for (int ax = 0; ax < 3; ++ax)
          if (!P.ax[ax].unb) {
            const double w = omega(P.ax[ax], (int)idx[ax], false);
            k2 += w * w;
            const double d = 2.0 * std::sin(0.5 * w * P.ax[ax].h) / P.ax[ax].h;
            s2 += d * d;
          }
        const double k = std::sqrt(k2);
        if (P.du == 0) {
          const double gv = P.g.variant == 8 ? (s2 > 0.0 ? -1.0 / s2 : 0.0) : P.g.value(0.0, k);
          b[x + n0 * (y + n1 * z)] = a[x + n0 * (y + n1 * z)] * gv;
          continue;
        }
        // target position in the convolution directions
        double xt[3] = {0, 0, 0};
        for (int ax = 0; ax < 3; ++ax)
          if (P.ax[ax].unb) xt[ax] = (idx[ax] + (P.ax[ax].node ? 0.0 : 0.5)) * P.ax[ax].h;
        // iterate over sources: for non-convolution axes the "source list" is the single
        // mode itself
        const int sz0 = P.ax[0].unb ? (int)src[0].size() : 1;
        const int sz1 = P.ax[1].unb ? (int)src[1].size() : 1;
        const int sz2 = P.ax[2].unb ? (int)src[2].size() : 1;
        cd acc = 0.0;
        for (int s2 = 0; s2 < sz2; ++s2)
          for (int s1 = 0; s1 < sz1; ++s1)
            for (int s0 = 0; s0 < sz0; ++s0) {
              const int ss[3] = {s0, s1, s2};
              long jj[3], off[3] = {0, 0, 0};
              double r2 = 0.0, sign = 1.0;
              for (int ax = 0; ax < 3; ++ax) {
                if (!P.ax[ax].unb) { jj[ax] = idx[ax]; continue; }
                const Src& S = src[ax][ss[ax]];
                jj[ax] = S.j;
                const double d = xt[ax] - S.x;
                off[ax] = std::lround(d / P.ax[ax].h);
                r2 += d * d;
                sign *= S.sign;
              }
              const double gv = P.g.variant == 8 ? P.g.lattice(off[0], off[1], off[2])
                                                 : P.g.value(std::sqrt(r2), k);
              acc += sign * gv * a[jj[0] + n0 * (jj[1] + n1 * jj[2])];
            }
        b[x + n0 * (y + n1 * z)] = acc * cellvol;
      }
  // 4) backward defining sums along spectral directions, normalised
  double scale = 1.0;
  for (int ax = 2; ax >= 0; --ax) {
    if (P.ax[ax].unb) continue;
    scale /= P.ax[ax].nlog;
    Dims nd = cur;
    nd.n[ax] = P.ax[ax].nuser;
    std::vector<cd> c(nd.size());
    along_axis(ax, cur, b, nd, c, [&](const cd* i, cd* o) { axis_backward(P.ax[ax], i, o, MODE_NAIVE); });
    b.swap(c);
    cur = nd;
  }
  // odd-face nodes of semi-unbounded axes are exactly zero
  for (long z = 0; z < du.n[2]; ++z)
    for (long y = 0; y < du.n[1]; ++y)
      for (long x = 0; x < du.n[0]; ++x) {
        const long idx[3] = {x, y, z};
        double v = b[x + du.n[0] * (y + du.n[1] * z)].real() * scale;
        for (int ax = 0; ax < 3; ++ax) {
          const Axis& A = P.ax[ax];
          if (!A.node || !A.unb) continue;
          if (A.cls == C_OU && idx[ax] == 0) v = 0.0;
          if (A.cls == C_UO && idx[ax] == A.N) v = 0.0;
        }
        out[x + du.n[0] * (y + du.n[1] * z)] = v;
      }
  return 0;
}

// The plain definition at chosen points, for problems whose three axes are all
// convolution directions (fully or semi-unbounded, Sec. II-C): the discrete convolution
// of the image-extended right-hand side with the sampled kernel, times the cell volume.
// pts holds (x, y, z) user indices.  Costs one sum over the whole grid per point.
int direct_points(const Problem& P, const double* rhs, int npts, const int* pts, double* out) {
  if (P.kind != 0) return -3;
  for (int ax = 0; ax < 3; ++ax)
    if (!P.ax[ax].unb) return -3;
  const Dims du = user_dims(P);
  struct Src { int j; double x; double sign; };
  std::vector<Src> src[3];
  double cellvol = 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    const Axis& A = P.ax[ax];
    cellvol *= A.h;
    const double off = A.node ? 0.0 : 0.5;
    if (A.cls == C_UU) {
      for (int j = 0; j < A.nuser; ++j) src[ax].push_back({j, (j + off) * A.h, 1.0});
      continue;
    }
    const double sgn = (A.cls == C_EU || A.cls == C_UE) ? 1.0 : -1.0;
    const double face = A.rev ? A.L() : 0.0;
    for (int j = 0; j < A.nuser; ++j) {
      const double x = (j + off) * A.h;
      const double xi = 2.0 * face - x;
      if (A.node && std::fabs(xi - x) < 0.25 * A.h) {
        if (sgn > 0) src[ax].push_back({j, x, 1.0});
        continue;
      }
      src[ax].push_back({j, x, 1.0});
      src[ax].push_back({j, xi, sgn});
    }
  }
  const long nx = du.n[0], ny = du.n[1];
  for (int q = 0; q < npts; ++q) {
    const int* ip = pts + 3 * q;
    double xt[3];
    bool zero = false;
    for (int ax = 0; ax < 3; ++ax) {
      const Axis& A = P.ax[ax];
      if (ip[ax] < 0 || ip[ax] >= A.nuser) return -2;
      xt[ax] = (ip[ax] + (A.node ? 0.0 : 0.5)) * A.h;
      if (A.node && ((A.cls == C_OU && ip[ax] == 0) || (A.cls == C_UO && ip[ax] == A.N))) zero = true;
    }
    double acc = 0.0;
    const long s2n = (long)src[2].size();
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (long s2 = 0; s2 < s2n; ++s2) {
      const Src& Z = src[2][s2];
      const double dz = xt[2] - Z.x;
      double part = 0.0;
      for (const Src& Y : src[1]) {
        const double dy = xt[1] - Y.x;
        const double* row = rhs + nx * (Y.j + ny * (long)Z.j);
        const double syz = Y.sign * Z.sign;
        for (const Src& X : src[0]) {
          const double dx = xt[0] - X.x;
          const double gv = P.g.variant == 8
                                ? P.g.lattice(std::lround(dx / P.ax[0].h), std::lround(dy / P.ax[1].h),
                                              std::lround(dz / P.ax[2].h))
                                : P.g.value(std::sqrt(dx * dx + dy * dy + dz * dz), 0.0);
          part += syz * X.sign * gv * row[X.j];
        }
      }
      acc += part;
    }
    out[q] = zero ? 0.0 : acc * cellvol;
  }
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------------
// C interface (ctypes)
// ---------------------------------------------------------------------------------
extern "C" {

// LGF2: the lattice Green's function at integer offsets [n2][n1][n0] (x fastest) used by
// the following solves with three convolution directions; the caller keeps it alive.
void oracle_set_lgf(const double* table, long n0, long n1, long n2) {
  g_lgf = table;
  g_lgf_n[0] = n0;
  g_lgf_n[1] = n1;
  g_lgf_n[2] = n2;
}

int oracle_fft(int n, const double* in, double* out, int sign) {
  if (n < 1) return -2;
  fft(n, reinterpret_cast<const cd*>(in), reinterpret_cast<cd*>(out), sign < 0 ? -1 : 1);
  return 0;
}

int oracle_dft_naive(int n, const double* in, double* out, int sign) {
  if (n < 1) return -2;
  dft_naive(n, reinterpret_cast<const cd*>(in), reinterpret_cast<cd*>(out), sign < 0 ? -1 : 1);
  return 0;
}

int oracle_r2r(int kind, int n, const double* in, double* out, int naive) {
  if (kind < 0 || kind > 7 || n < 1) return -2;
  if ((kind == REDFT00 && n < 2)) return -2;
  if (naive) r2r_naive(kind, n, in, out);
  else r2r_fft(kind, n, in, out);
  return 0;
}

// Per-axis table as the oracle understands it (for tests):
// info[0]=class, [1]=nuser, [2]=nspec, [3]=nlog, [4]=fwd kind, [5]=bwd kind,
// [6]=first, [7]=kshift, [8]=unbounded, [9]=dft, [10]=reversed, [11]=2*half
int oracle_axis_info(int N, double h, int node, int bl, int br, int* info) {
  Axis a;
  const int rc = make_axis(N, h, node, bl, br, &a);
  if (rc) return rc;
  info[0] = a.cls; info[1] = a.nuser; info[2] = a.nspec; info[3] = (int)a.nlog;
  info[4] = a.fwd; info[5] = a.bwd; info[6] = a.first; info[7] = a.kshift;
  info[8] = a.unb; info[9] = a.dft; info[10] = a.rev; info[11] = (int)(2 * a.half);
  return 0;
}

// Kernel value (for tests): du, variant, cell volume via h[3] of the convolution axes.
double oracle_green_value(int du, int variant, double cellvol, double rho, double k) {
  Green g;
  g.du = du;
  g.variant = variant;
  g.cellvol = cellvol;
  if (du == 3) g.r_eq = std::cbrt(3.0 * cellvol / (4.0 * kPi));
  if (du == 2) g.r_eq = std::sqrt(cellvol / kPi);
  if (variant >= 2) {  // HEJ: h = cellvol^(1/3)
    g.eps = 2.0 * std::cbrt(cellvol);
    g.kc = kPi / std::cbrt(cellvol);
  }
  return g.value(rho, k);
}

// Solve.  n[3] = cells / intervals per axis (x, y, z); h[3]; bc[6] = (x-left, x-right,
// y-left, y-right, z-left, z-right) with 0 even, 1 odd, 2 periodic, 3 unbounded;
// layout 0 cell / 1 node; green 0 (CHAT2 as printed) / 1 (sphere-mean self-term);
// kind 0 Poisson / 1 Biot-Savart with the spectral curl / 2, 3, 4 Biot-Savart with the
// finite-difference derivative of order 2, 4, 6 (3 components); mode 0 fast / 1 naive /
// 2 direct (Poisson only).
// rhs, out: [ncomp][nz][ny][nx] doubles with the user's point counts.
int oracle_solve(const int* n, const double* h, const int* bc, int layout, int green, int kind,
                 int mode, const double* rhs, double* out) {
  Problem P;
  const int rc = make_problem(n, h, bc, layout, green, kind, &P);
  if (rc) return rc;
  if (mode == MODE_DIRECT) return solve_direct(P, rhs, out);
  return solve_spectral(P, rhs, out, mode == MODE_NAIVE ? MODE_NAIVE : MODE_FAST);
}

// Biot-Savart with boundary conditions per component: bcv[18] = (component q, axis a,
// face f) at 6 q + 2 a + f, codes as for oracle_solve; kind 1 spectral curl, 2 / 3 / 4
// finite differences of order 2 / 4 / 6; mode 0 fast / 1 naive.  rhs, out: [3][nz][ny][nx].
// Component p of the result satisfies the swapped symmetry of component p of bcv.
int oracle_solve_vector(const int* n, const double* h, const int* bcv, int layout, int green,
                        int kind, int mode, const double* rhs, double* out) {
  if (kind < 1 || kind > 4) return -3;
  if (vector_faces_ok(bcv)) return -1;
  Problem Pin[3], Pout[3];
  for (int q = 0; q < 3; ++q) {
    int swapped[6];
    for (int i = 0; i < 6; ++i) swapped[i] = swap_face(bcv[6 * q + i]);
    int rc = make_problem(n, h, bcv + 6 * q, layout, green, 0, &Pin[q]);
    if (rc) return rc;
    rc = make_problem(n, h, swapped, layout, green, 0, &Pout[q]);
    if (rc) return rc;
  }
  return solve_vector(Pin, Pout, kind, rhs, out, mode == MODE_NAIVE ? MODE_NAIVE : MODE_FAST);
}

// The solution at npts user points (x, y, z indices in pts[3 * npts]) by the direct
// convolution sum; every axis must be fully or semi-unbounded; Poisson only.
int oracle_direct_points(const int* n, const double* h, const int* bc, int layout, int green,
                         const double* rhs, int npts, const int* pts, double* out) {
  Problem P;
  const int rc = make_problem(n, h, bc, layout, green, 0, &P);
  if (rc) return rc;
  return direct_points(P, rhs, npts, pts, out);
}

// The plain transforms of a plan without the spectral multiplication (Sec. II-B, II-C:
// the forward operation of every axis, or the backward operation with its crop and
// fix-ups), unnormalised.  dir -1: in = real user field [nz][ny][nx], out = complex
// spectrum [sz][sy][sx] (interleaved, full length along every axis); dir +1: in =
// complex spectrum, out = real part of the backward transform on the user grid.
int oracle_transform(const int* n, const double* h, const int* bc, int layout, int dir,
                     const double* in, double* out) {
  Problem P;
  const int rc = make_problem(n, h, bc, layout, 0, 0, &P);
  if (rc) return rc;
  if (dir < 0) {
    const long V = user_dims(P).size();
    std::vector<cd> f(V);
    for (long i = 0; i < V; ++i) f[i] = in[i];
    const std::vector<cd> F = forward3(P, f, MODE_FAST);
    std::memcpy(out, F.data(), F.size() * sizeof(cd));
    return 0;
  }
  const long S = (long)P.ax[0].nspec * P.ax[1].nspec * P.ax[2].nspec;
  std::vector<cd> F(S);
  std::memcpy(F.data(), in, S * sizeof(cd));
  const std::vector<cd> u = backward3(P, F, MODE_FAST);
  for (size_t i = 0; i < u.size(); ++i) out[i] = u[i].real();
  return 0;
}

// Green's spectrum on the (unfolded) spectral grid, complex interleaved, [z][y][x].
int oracle_green_spectrum(const int* n, const double* h, const int* bc, int layout, int green,
                          int mode, double* out) {
  Problem P;
  const int rc = make_problem(n, h, bc, layout, green, 0, &P);
  if (rc) return rc;
  const std::vector<cd> G = green_spectrum(P, mode);
  std::memcpy(out, G.data(), G.size() * sizeof(cd));
  return 0;
}

int oracle_spectral_dims(const int* n, const double* h, const int* bc, int layout, int* dims) {
  Problem P;
  const int rc = make_problem(n, h, bc, layout, 0, 0, &P);
  if (rc) return rc;
  for (int a = 0; a < 3; ++a) dims[a] = P.ax[a].nspec;
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Threads used by later calls (the CPU-baseline timing on one core and on all cores).
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
