// Descriptor of one "line pass": a batch of 1-D transforms along one axis of a 3-D
// array, read from one layout and written (transposed) into another.  Shared by the
// host planner and the device kernels of the GPU library.
#pragma once
#include <stdint.h>

namespace fm {

constexpr int kThreads = 256;    // threads per workgroup of every pass kernel
// Kernel length classes: a compile-time FFT length (> 1), or one of the two
// runtime-length kernels.  FP64 lines longer than kMaxFastLen64 take the long class.
constexpr int kRtShort = 0;
constexpr int kRtLong = 1;
constexpr int kMaxFastLen64 = 2048;
// Values per thread held across a radix stage for lines of length M (or kernel length
// class M).  FP64 holds 8 (radices up to 8), so that a stage, its butterfly temporaries
// and the persistent kernels' prefetch of the next tile stay in VGPRs; FP64 lines
// longer than kMaxFastLen64 need 16 and run one tile per workgroup without prefetch.
constexpr int elems_per_thread(int real_bytes, int M) {
  return (real_bytes == 4 || M == kRtLong || M > kMaxFastLen64) ? 16 : 8;
}
constexpr int max_radix(int real_bytes) { return real_bytes == 8 ? 8 : 16; }
// Green's-spectrum values per thread staged with a fused tile (its nl rows of F_line
// values): complex tiles (one line per FFT, F_line <= M/2 + 1) need at most E/2 + 1,
// tiles of two real lines per FFT at most E + 1.
constexpr int green_values(int real_bytes, int M, bool packed) {
  return packed ? elems_per_thread(real_bytes, M) + 1 : elems_per_thread(real_bytes, M) / 2 + 1;
}
// Persistent kernels with register prefetch: compile-time lengths with 8 FP64 values per
// thread, every compile-time length in FP32.
constexpr bool pipelined_kernel(int real_bytes, int MC) {
  return MC > 1 && (real_bytes == 4 || MC <= kMaxFastLen64);
}
// Input values per thread held by the register stage of one tile, per component: complex
// tiles hold kThreads * elems_per_thread values, real tiles (two lines per FFT) twice
// that, and the fused Biot-Savart tile (three components) a third per component.  A
// tile must not hold more input than kThreads times this.
constexpr int stage_values(int real_bytes, int M, bool in_cplx, int ncl) {
  return ncl == 3 ? (elems_per_thread(real_bytes, M) + 2) / 3
                  : (in_cplx ? 1 : 2) * elems_per_thread(real_bytes, M);
}
constexpr int kMaxLen = 4096;    // longest FFT
constexpr int kMaxStages = 16;
constexpr int kMaxLds = 163840;  // LDS a gfx950 workgroup may allocate
constexpr int kSoftLds = 65536;  // preferred tile LDS (keeps >= 2 workgroups per CU)

// How the FFT input z[0..M) of one FFT line is built from the loaded tile.
enum Gather : int32_t {
  G_CPLX = 0,   // z[m] = x[m] for m < n_data, else 0                      (complex lines)
  G_REAL2 = 1,  // z[m] = x1[m] + i x2[m] for m < n_data, else 0          (2 real lines)
  G_HERM2 = 2,  // z[m] = X1[m] + i X2[m] from two Hermitian half-spectra (inverse R2C)
  G_R2R = 3,    // symmetric extension of 2 real lines, pre-twiddle        (DCT / DST)
};

// How the FFT output Z[0..M) becomes the written line(s).
enum Scatter : int32_t {
  S_CPLX = 0,   // y[j] = Z[j mod M]                                      (complex lines)
  S_R2C2 = 1,   // two half-spectra X1[k], X2[k], k = 0..M/2                (forward R2C)
  S_REAL2 = 2,  // y1[j] = Re Z[j mod M], y2[j] = Im Z[j mod M]             (inverse R2C)
  S_R2R = 3,    // post-twiddle, real or imaginary part                    (DCT / DST)
};

// The pass kinds, each compiled as its own kernel (K_ANY: one kernel that reads the
// kind from the descriptor; used by batched launches).
enum PassKind : int32_t {
  K_ANY = 0,
  K_C2C_F = 1,   // complex forward along a DFT axis (zero padded)
  K_C2C_I = 2,   // complex inverse (crop / periodic duplicate)
  K_R2C = 3,     // first DFT axis, forward: two real lines per FFT
  K_C2R = 4,     // first DFT axis, inverse
  K_R2R = 5,     // DCT / DST, either direction
  K_F_C2C = 6,   // fused last axis, complex, Poisson
  K_F_CURL = 7,  // fused last axis, complex, three components with the spectral curl
  K_F_R2C = 8,   // fused last axis, the only DFT axis (two real lines per FFT)
  K_F_R2R = 9,   // fused last axis, all axes real-to-real
};
constexpr int kNumKinds = 10;

// Real-to-real transform in the form  y_q = sum_p w_p x_p cs(pi (p+a)(q+b) / nh),
// evaluated as a length-2nh DFT of a symmetric extension with pre- and post-twiddles.
struct R2R {
  int32_t nh;        // half period (FFT length M = 2 nh)
  int32_t a2, b2;    // 2a, 2b (0 or 1)
  int32_t sin;       // 0: cosine transform, 1: sine transform
  int32_t plo, phi;  // input index range (inclusive)
  int32_t wlo, whi;  // weights of the end points (2 elsewhere)
  int32_t in_rev, in_base;   // line index j of input p: rev ? base - p : p - base
  int32_t qlo, qhi;  // output index range (inclusive); others write 0
  int32_t out_rev, out_base; // output index q of line index j: rev ? base - j : j + base
};

// Green's spectrum lookup (pass 3).  Table index along an axis: DFT axes fold the
// mode index k to min(k, M - k); real-to-real axes use the spectral index itself.
struct GreenRef {
  const void* G;       // table [F_c][F_b][F_line] in the working precision
  int32_t F_b, F_line; // table extents along the tile axis and the line axis
  int32_t fold_c, fold_b, fold_line;  // 0: identity, else the DFT length M to fold with
  // spectral curl (Biot-Savart): wavenumber of mode k on DFT axis = 2 pi k' / period
  int32_t curl;
  int32_t axis_line, axis_b, axis_c;  // physical axis (0 x, 1 y, 2 z) of each direction
  double dw_line, dw_b, dw_c;         // 2 pi / period
  int32_t M_line, M_b, M_c;           // DFT lengths for the signed-mode map
  // derivative of the curl: 0 spectral (i w), 2 / 4 / 6 the central-difference symbol of
  // that order, i/h sum_j c_j sin(j w h) with w h = 2 pi k / M (Sec. V); the kernels read
  // the factor of every mode of the three directions from tables in the working precision
  // (generated in FP64)
  int32_t deriv;
  const void* dtab_line;
  const void* dtab_b;
  const void* dtab_c;
  // a symmetric or semi-unbounded c direction (conditions per component, Sec. V): the
  // derivative of a component along it is s w times its real-to-real coefficient, s = +1
  // after a sine transform and -1 after a cosine one (both flipped on a reversed axis).
  // The kernels form u_hat = G i (w x f_hat); only the two components tangential to c
  // (which share their faces, hence s) enter its c-direction terms, so the c factor
  // becomes the complex -i s w.  csym = s, or 0 when c is a DFT direction; csym_b the
  // same for the b direction (a second symmetric axis).
  int32_t csym, csym_b;
};


// Output conventions applied by the last pass along its two batch axes (Sec. II-A,
// II-B): node-centred periodic duplicate f_N := f_0, nodes on odd faces := 0.
struct Fixup {
  int32_t b_dup, b_zero_lo, b_zero_hi, b_last;
  int32_t c_dup, c_zero_lo, c_zero_hi, c_last;
};

// Radix schedule of an FFT length: radix-16 stages first (when rmax allows), then one
// of 8 / 4 / 2, then 3, 5 and 7.  Shared by the host (table generation) and the device (compile-time
// stage sequence); returns 0 past the last stage.
constexpr int radix_at(int M, int s, int rmax) {
  int m = M;
  for (int i = 0;; ++i) {
    int r = 0;
    if (m > 1) {
      if (rmax >= 16 && m % 16 == 0) r = 16;
      else if (m % 8 == 0) r = 8;
      else if (m % 4 == 0) r = 4;
      else if (m % 2 == 0) r = 2;
      else if (m % 3 == 0) r = 3;
      else if (m % 5 == 0) r = 5;
      else if (m % 7 == 0) r = 7;
    }
    if (i == s || r == 0) return r;
    m /= r;
  }
}

// LDS layout of an FFT line: slot i sits at i + i / 16 (one unused slot after every
// 16), so that the power-of-two strides of the radix passes' writes fall on different
// LDS banks; lines are fft_line_stride(M) slots apart.
constexpr int fft_line_stride(int M) { return M + (M >> 4) + 1; }

// Per-wavefront fused kernels (complex lines of a power-of-two length M): each lane holds
// E points of a line (E = 16, or 8 for lines of at most 512 points), so a line spans
// P = M / E <= 64 lanes.  Radix schedule: E first, then min(E, rest) until the product is
// M.  Stage s >= 1 reads its twiddles W_{Ns R}^{k r} (Ns = product of the earlier radices,
// 1 <= r < R, k < Ns) from a table at wave_tw_offset(M, s, E) + (r-1) Ns + k.
constexpr int kWaveValues = 16;
constexpr bool wave_length(int M, int E = kWaveValues) {
  return (E == 8 || E == 16 || E == 32) && M >= 2 * E && M <= 64 * E && (M & (M - 1)) == 0;
}
constexpr int wave_radix(int M, int s, int E = kWaveValues) {
  int rest = M / E;
  if (s == 0) return E;
  for (int i = 1; i < s; ++i) rest /= (rest < E ? rest : E);
  return rest <= 1 ? 0 : (rest < E ? rest : E);
}
constexpr int wave_ns(int M, int s, int E = kWaveValues) {
  int n = 1;
  for (int i = 0; i < s; ++i) n *= wave_radix(M, i, E);
  return n;
}
constexpr int wave_tw_offset(int M, int s, int E = kWaveValues) {
  int off = 0;
  for (int i = 1; i < s; ++i) off += wave_ns(M, i, E) * (wave_radix(M, i, E) - 1);
  return off;
}
constexpr int wave_stage_count(int M, int E = kWaveValues) {
  int s = 0;
  while (wave_radix(M, s, E) != 0) ++s;
  return s;
}
constexpr int wave_tw_size(int M, int E = kWaveValues) {
  return wave_tw_offset(M, wave_stage_count(M, E), E);
}
// lines one wavefront holds (0 for lengths the per-wavefront kernels do not serve)
constexpr int wave_lines(int M, int E = kWaveValues) { return wave_length(M, E) ? 64 / (M / E) : 0; }

// Lengths with compile-time kernels (other lengths use the runtime-length kernel).
constexpr int kFastLens[] = {32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048, 4096};

// Offset of stage s in the per-length stage twiddle table: stage s holds
// W_{Ns R}^{k r} for k < Ns (product of the earlier radices), 1 <= r < R.
constexpr int stage_table_offset(int M, int s, int rmax) {
  int off = 0, ns = 1;
  for (int i = 0; i < s; ++i) {
    const int r = radix_at(M, i, rmax);
    off += ns * (r - 1);
    ns *= r;
  }
  return off;
}
constexpr int stage_table_size(int M, int rmax) {
  int s = 0;
  while (radix_at(M, s, rmax) != 0) ++s;
  return stage_table_offset(M, s, rmax);
}

struct PassDesc {
  // tile geometry: lines along `line`, B consecutive lines along `b`, index c, comp
  const void* in;
  void* out;
  int64_t in_s_line, in_s_b, in_s_c, in_s_comp;    // element strides of the input
  int64_t out_s_line, out_s_b, out_s_c, out_s_comp; // element strides of the output
  int32_t nb, nc, ncomp;    // extents of b, c and the component count
  int32_t in_n, out_n;      // values read / written per line
  int32_t in_cplx, out_cplx;
  int32_t B;                // lines per tile
  int32_t tiles;            // tiles of this pass = ceil(nb / B) * nc * (ncomp or 1)
  // transform
  int32_t M;
  int32_t nstages;
  int32_t radix[kMaxStages];
  const void* tw;           // 4M table: tw[j] = exp(-2 pi i j / (4M))
  int32_t gather, scatter;
  int32_t n_data;           // G_CPLX / G_REAL2: values taken before the zero padding
  R2R r2r;
  // fused pass 3: forward (gather/scatter above with sign -1), spectral multiply,
  // inverse (gather2/scatter2 with sign +1)
  int32_t fused;            // 0: plain pass, 1: fused pass
  int32_t sign;             // plain pass: -1 forward, +1 inverse
  int32_t gather2, scatter2;
  int32_t spec_n;           // fused R2R: spectral values per line held in LDS
  R2R r2r2;
  GreenRef g;
  Fixup fix;                // last pass only
  int32_t has_fix;
  int32_t lds_bytes;        // dynamic LDS the tile needs
  // host-precomputed multipliers for division by in_n, out_n, B, spec_n:
  // n / d = (n * mag) >> 32 for n * d < 2^32
  uint64_t mag_in, mag_out, mag_B, mag_spec;
  const void* stw;          // stage twiddle table of a compile-time length (or null)
  int32_t persist;          // with lds_tabs: 1 = as many workgroups as fit on the device,
                            // each looping over tiles; 0 = one tile each
  int32_t kind;             // PassKind
  int32_t raw_off;          // byte offset of the raw input tile in LDS (0: aliases the
                            // FFT buffer; real-to-real tiles keep it apart)
  // LDS staging.  Persistent kernels copy the stage twiddle table (stw_n entries) and,
  // for real-to-real kinds, the first tw_n entries of the 4M table to LDS at tab_off
  // once per workgroup; fused passes load the tile's Green rows (nl x g.F_line values)
  // with the tile's input and keep them in LDS at g_off.  The transform itself then
  // reads no global memory, so the prefetch of the next tile overlaps it.
  int32_t tab_off, stw_n, tw_n;
  int32_t long_rt;          // FP64: run in the runtime-length class with 16 values per
                            // thread (a tile that does not fit 8, e.g. a 3-component curl)
  int32_t g_off;
  uint64_t mag_gline;       // division by g.F_line
  int32_t lds_tabs;         // compile-time-length kernels that allow it: 1 = twiddle tables
                            // staged in LDS (persistent loop, or one tile per workgroup);
                            // 0 = one tile per workgroup reading them from global memory
  int32_t wave;             // pass in a per-wavefront kernel (fm_wave.h): its values per
                            // lane E (16 or 8; 0: not that kernel).  Fused complex passes:
                            // B = lines per workgroup, a multiple of wave_lines(M, E).
                            // Plain passes: four wavefronts, B = 4 wave_lines(M, E) FFT
                            // lines (times 2 real lines per FFT for the packed kinds)
  int32_t wave_rs;          // plain passes: raw tile line stride, in input elements
  const void* wtw;          // its stage twiddle tables: E = 16 (wave_tw_size(M, 16) entries)
  const void* wtw8;         // and E = 8
  const void* wtw32;        // and E = 32 (FP32 Poisson fused passes)
};

// Sampling description of the Green's function for the spectrum generation (FP64).
struct GreenGen {
  int32_t du, variant;       // convolution directions, self-term variant
  double cellvol, r_eq;      // product of h over convolution directions, r_eq
  int32_t unb[3];            // per table axis: 1 convolution direction, 0 spectral
  double h[3];               // spacing (convolution directions)
  double dw[3], shift[3];    // spectral: omega = dw * (index + shift)
  int32_t n[3];              // sample extents
  double eps, kc;            // regularised kernels: smoothing length, spectral cut-off
};

// Biot-Savart with three symmetric axes (conditions per component): the curl times the
// Green's spectrum on the real three-axis spectra of the components, in place.  Spectra
// [comp][n0][n1][n2] (table axes a0 slowest .. a2 fastest, frequency-indexed), Green's
// table of the same extents; d[t] the derivative factor of each frequency of table axis t;
// ax[t] its physical axis; sg[a][b] the sign of the derivative of component b along
// physical axis a (+1 after a sine transform, -1 after a cosine one, flipped on a
// reversed axis).
struct CurlReal {
  void* S;                   // spectra, working precision
  int64_t comp_stride;       // elements between components
  const void* G;             // Green's table
  const void* d[3];          // derivative factors per table axis
  int32_t n[3];              // extents per table axis
  int32_t ax[3];             // physical axis of each table axis
  int32_t sg[3][3];          // [physical axis][component]
};

// Lattice Green's function (LGF2) quadrature: nodes t_k = exp(u_lo + k du), k < K, and
// per table axis the scaled Bessel values exp(-x) I_n(x), x = 2 t_k / h^2, n < nA.
struct LgfGen {
  int32_t K, stride;         // nodes, row stride of the Bessel table (>= max nA)
  int32_t nA[3];             // offsets per table axis
  double u_lo, du, c;        // log-t grid; far-field subtraction constant
  double h[3];               // spacing per table axis
};

}  // namespace fm
