// Host side of the GPU library: planning (boundary conditions -> per-axis transforms,
// transform order, padded sizes, data layouts, tile shapes), generation of twiddles and
// of the Green's spectrum on the device, and the C entry points of include/fluxmi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "../../include/fluxmi.h"
#include "fm_internal.h"
#include "fm_pass.h"

namespace fm {
template <typename T>
hipError_t launch_pass(const PassDesc& d, const PassDesc* dev, const void* in, void* out,
                       hipStream_t st);
template <typename T>
hipError_t launch_pass_batched(int len_class, const PassDesc* ds, const int* prefix, int n,
                               int total_tiles, int lds_bytes, hipStream_t st);
template <typename T> hipError_t launch_twiddles(void* out, int M, hipStream_t st);
template <typename T> hipError_t launch_stage_twiddles(void* out, int M, hipStream_t st);
template <typename T> hipError_t launch_wave_twiddles(void* out, int M, int E, hipStream_t st);
bool is_fast_len(int M);

hipError_t launch_green_sample(double* S, const GreenGen& g, hipStream_t st);
hipError_t launch_lgf(double* S, double* A, double* W, const LgfGen& g, hipStream_t st);
template <typename T>
hipError_t launch_curl_real(const CurlReal& c, hipStream_t st);
template <typename T>
hipError_t launch_green_final(void* G, const double* S, const int F[3], const int n[3],
                              const int off[3], double scale, hipStream_t st);
}  // namespace fm

namespace {

thread_local int g_last_hip = 0;

#define FM_HIP(call)                       \
  do {                                     \
    hipError_t e_ = (call);                \
    if (e_ != hipSuccess) {                \
      g_last_hip = (int)e_;                \
      return FM_E_HIP;                     \
    }                                      \
  } while (0)

// per-axis class (left/right faces)
enum Cls { C_P, C_EE, C_OO, C_EO, C_OE, C_UU, C_EU, C_OU, C_UE, C_UO };

// Real-to-real transform families (FFTW's numbering of the kinds).
enum Kind { REDFT00, REDFT01, REDFT10, REDFT11, RODFT00, RODFT01, RODFT10, RODFT11 };

// y_q = sum_p w_p x_p cs(pi (p + a)(q + b) / nh): parameters of each kind for n points
// (input index t = p - pin, output index k = q - qout).
struct KindForm {
  int nh_add, a2, b2, sin, pin, wlo, whi, qout;
};
KindForm kind_form(int k) {
  switch (k) {
    case REDFT00: return {-1, 0, 0, 0, 0, 1, 1, 0};
    case RODFT00: return {+1, 0, 0, 1, 1, 2, 2, 1};
    case REDFT10: return {0, 1, 0, 0, 0, 2, 2, 0};
    case REDFT01: return {0, 0, 1, 0, 0, 1, 2, 0};
    case REDFT11: return {0, 1, 1, 0, 0, 2, 2, 0};
    case RODFT10: return {0, 1, 0, 1, 0, 2, 2, 1};
    case RODFT01: return {0, 0, 1, 1, 1, 2, 1, 0};
    default: return {0, 1, 1, 1, 0, 2, 2, 0};  // RODFT11
  }
}

struct AxisPlan {
  int N = 0, nuser = 0, cls = C_P;
  double h = 0, L = 0;
  bool node = false, unb = false, dft = false, rev = false;
  // DFT axes
  int M = 0, n_data = 0;
  bool first_dft = false;
  // real-to-real axes
  int fwd = 0, bwd = 0, first = 0, nin = 0;
  int nspec = 0;          // spectral extent along this axis after its forward pass
  double nlog = 1;        // normalisation length
  // Green table
  int F = 0, Fs = 0, off = 0;
  double dw = 0, shift = 0;
};

int classify(int bl, int br, int* cls) {
  if (bl < 0 || bl > 3 || br < 0 || br > 3) return FM_E_BC;
  if ((bl == FM_BC_PER) != (br == FM_BC_PER)) return FM_E_BC;
  static const int table[4][4] = {
      // right: EVEN  ODD   PER  UNB        left:
      {C_EE, C_EO, -1, C_EU},  // EVEN
      {C_OE, C_OO, -1, C_OU},  // ODD
      {-1, -1, C_P, -1},       // PER
      {C_UE, C_UO, -1, C_UU},  // UNB
  };
  *cls = table[bl][br];
  return FM_OK;
}

// Table I (symmetric classes), Sec. II-B (periodic), Sec. II-C (unbounded and
// semi-unbounded): forward / backward transforms, used input points, sizes.
int plan_axis(int N, double h, bool node, int bl, int br, AxisPlan* a) {
  if (N < 2 || !(h > 0)) return FM_E_SIZE;
  int rc = classify(bl, br, &a->cls);
  if (rc) return rc;
  a->N = N;
  a->h = h;
  a->L = N * h;
  a->node = node;
  a->nuser = node ? N + 1 : N;
  const int c = a->cls;
  a->unb = c >= C_UU;
  a->dft = (c == C_P || c == C_UU);
  a->rev = (c == C_UE || c == C_UO);
  if (c == C_P) {
    a->M = N;
    a->n_data = N;  // the node f_N duplicates f_0 and is not used
    a->nlog = N;
  } else if (c == C_UU) {
    a->M = 2 * N;
    a->n_data = a->nuser;  // zero padding up to 2N
    a->nlog = 2 * N;
  } else if (c <= C_OE) {
    // spectral symmetric classes
    if (node) {
      switch (c) {
        case C_EE: a->fwd = a->bwd = REDFT00; a->first = 0; a->nin = N + 1; break;
        case C_OO: a->fwd = a->bwd = RODFT00; a->first = 1; a->nin = N - 1; break;
        case C_OE: a->fwd = RODFT01; a->bwd = RODFT10; a->first = 1; a->nin = N; break;
        default: a->fwd = REDFT01; a->bwd = REDFT10; a->first = 0; a->nin = N; break;  // EO
      }
    } else {
      a->first = 0;
      a->nin = N;
      switch (c) {
        case C_EE: a->fwd = REDFT10; a->bwd = REDFT01; break;
        case C_OO: a->fwd = RODFT10; a->bwd = RODFT01; break;
        case C_OE: a->fwd = a->bwd = RODFT11; break;
        default: a->fwd = a->bwd = REDFT11; break;  // EO
      }
    }
    a->nlog = 2 * N;
  } else {
    // semi-unbounded: padded to 2L on the unbounded side, DCT / DST on the extension
    const bool even = (c == C_EU || c == C_UE);
    if (node) {
      if (even) { a->fwd = a->bwd = REDFT00; a->first = 0; a->nin = 2 * N + 1; }
      else { a->fwd = a->bwd = RODFT00; a->first = 1; a->nin = 2 * N - 1; }
    } else {
      a->first = 0;
      a->nin = 2 * N;
      if (even) { a->fwd = REDFT10; a->bwd = REDFT01; }
      else { a->fwd = RODFT10; a->bwd = RODFT01; }
    }
    a->nlog = 4 * N;
  }
  if (!a->dft) {
    const KindForm f = kind_form(a->fwd);
    a->M = 2 * (a->nin + f.nh_add);
    a->nspec = a->nin;
  }
  return FM_OK;
}

// R2R descriptor of kind `k` with n points, mapped onto the line arrays.
//  forward (dir = +1): input = user line (nuser, `first`, reversal), output = spectrum
//  backward (dir = -1): input = spectrum, output = user line
// common: spectral index = frequency index (the spectra of several components, of
// different kinds, share one indexing; the slots outside a kind's range hold 0).
fm::R2R make_r2r(const AxisPlan& a, int kind, bool forward, bool common = false) {
  const KindForm f = kind_form(kind);
  const int n = a.nin;
  fm::R2R r{};
  r.nh = n + f.nh_add;
  r.a2 = f.a2;
  r.b2 = f.b2;
  r.sin = f.sin;
  r.plo = f.pin;
  r.phi = f.pin + n - 1;
  r.wlo = f.wlo;
  r.whi = f.whi;
  r.qlo = f.qout;
  r.qhi = f.qout + n - 1;
  if (forward) {
    // p = (rev ? nuser-1-j : j) - first + pin
    if (a.rev) { r.in_rev = 1; r.in_base = a.nuser - 1 - a.first + f.pin; }
    else { r.in_rev = 0; r.in_base = f.pin - a.first; }
    r.out_rev = 0;
    r.out_base = common ? 0 : f.qout;  // q = s + qout
  } else {
    r.in_rev = 0;
    r.in_base = common ? 0 : f.pin;    // p = s + pin
    // q = (rev ? nuser-1-j : j) - first + qout
    if (a.rev) { r.out_rev = 1; r.out_base = a.nuser - 1 - a.first + f.qout; }
    else { r.out_rev = 0; r.out_base = f.qout - a.first; }
  }
  return r;
}

int radix_plan(int M, fm::PassDesc* d) {
  if (M < 2 || M > fm::kMaxLen) return FM_E_SIZE;
  int m = M, ns = 0;
  const int rs[] = {8, 4, 2, 3, 5, 7};  // at most radix 8 (fits both precisions)
  for (int r : rs) {
    while (m % r == 0) {
      if (ns >= fm::kMaxStages) return FM_E_SIZE;
      d->radix[ns++] = r;
      m /= r;
    }
  }
  if (m != 1) return FM_E_SIZE;
  d->M = M;
  d->nstages = ns;
  return FM_OK;
}

// strides (elements) of a layout given its axis order (slow -> fast) and extents
void layout_strides(const int order[3], const int ext[3], int64_t stride[3], int64_t* size) {
  int64_t s = 1;
  for (int i = 2; i >= 0; --i) {
    stride[order[i]] = s;
    s *= ext[order[i]];
  }
  *size = s;
}

}  // namespace

struct fm_plan_s {
  int n[3];
  double h[3];
  int bc[3][2];
  int layout, green, prec, kind, ncomp;
  AxisPlan ax[3];
  int order[3];     // transform order
  int tb1;          // tile axis of passes 1 and 5
  int L1[3], L2[3]; // layouts (slow -> fast)
  int ext_user[3], ext1[3], ext2[3];
  int64_t Vu, V1, V2;
  bool cplx1, cplx2;
  size_t elem;      // sizeof(real)
  size_t bytesA, bytesB;  // per component
  size_t ws_bytes;
  // the five passes of a solve, then the last axis's plain forward (B -> spectrum) and
  // backward (spectrum -> B) transforms of fm_fft_forward / fm_fft_backward
  static constexpr int kPasses = 7;
  fm::PassDesc pass[kPasses];
  bool long_rt[kPasses] = {};  // the pass needs the runtime-length class in the LDS-tile kernel
  const void* stw_plan[kPasses] = {};  // stage table of the planned kernel (null: runtime-length class)
  int ext_spec[3];
  int64_t Vspec;
  bool cplx_spec;
  void* G = nullptr;
  fm::PassDesc* dpass = nullptr;  // the descriptors in device memory
  int GF[3];
  std::map<int, void*> tw;
  std::map<int, void*> stw;
  std::map<int, void*> tw64;
  int tuned_from_cache = 0;  // the last fm_plan_tune applied a FLUXMI_TUNE_CACHE entry
  std::map<int, void*> wtw;  // stage twiddles of the per-wavefront kernels, by (M << 6) | E
  void* dtab = nullptr;      // central-difference symbols of the curl (line, b, c tables)
  void* ws_internal = nullptr;
  std::mutex ws_mu;  // guards the lazy allocation of ws_internal
  // Deferred creation (serving loop): the generation kernels may still run when the
  // plan is returned.  `ready` completes with them; the FP64 temporaries in gen_free
  // and the host copies of the generation descriptors are released after it.
  hipEvent_t ready = nullptr;
  std::vector<void*> gen_free;
  std::vector<fm::PassDesc> gen_desc;
  int device = 0;
  size_t table_bytes = 0;  // device memory of the plan's tables (Green, twiddles, descriptors)
  // fm_plan_create_vector: faces per component (bc above holds component 0's).  The
  // symmetric or semi-unbounded axis is the first transformed (a0); passes 1 and 5 run
  // once per component, each with its own real-to-real transform (the input's kind
  // forward, the swapped kind of the output backward), on a spectrum indexed by
  // frequency shared by the three components.  Device descriptors of components 1 and 2
  // follow the kPasses at dpass[kPasses + vec_slot(pass, comp)].
  bool vec = false;
  // a second symmetric axis (transformed by passes 2 and 4, also once per component): the
  // DFT axis is then transformed as a full complex DFT, pass 2 writes complex values with
  // a zero imaginary part and pass 4 reads their real parts
  bool vec2 = false;
  // three symmetric axes: pass 3 is replaced by the plain transforms along the last axis
  // (descriptors 6 and 7, once per component) around the real curl on the spectra in a
  // workspace region after B (curl_real_kernel)
  bool vec3 = false;
  fm::CurlReal vcurl{};
  int bcv[3][3][2] = {};
  // [component][0: pass 1 forward, 1: pass 5 backward, 2: pass 2 forward, 3: pass 4
  // backward, 4: last-axis forward, 5: last-axis backward]
  fm::R2R vr2r[3][6] = {};
  fm::Fixup vfix[3] = {};  // pass 5's output conventions per component (its faces)
  int vhas_fix[3] = {};
  static constexpr int kVecDesc = 12;
  fm::PassDesc vdesc[kVecDesc];  // host copies of the device slots (vec_slot)
};

namespace {

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

// Device allocations of plan creation and tuning.  Test hook: with FLUXMI_FAIL_ALLOC=k the
// k-th of them (counted from 1 since the variable last changed) reports out-of-memory, so
// that every failure path of plan creation can be driven from the host.
hipError_t plan_malloc_raw(void** ptr, size_t bytes) {
  static std::mutex mu;
  static std::string last;
  static long count = 0;
  const char* e = std::getenv("FLUXMI_FAIL_ALLOC");
  if (e && *e) {
    std::lock_guard<std::mutex> lock(mu);
    if (last != e) {
      last = e;
      count = 0;
    }
    if (++count == std::atol(e)) {
      *ptr = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(ptr, bytes);
}

template <typename P>
hipError_t plan_malloc(P** ptr, size_t bytes) {
  return plan_malloc_raw(reinterpret_cast<void**>(ptr), bytes);
}

// multiplier m = ceil(2^32 / d): n / d == (n * m) >> 32 whenever n * d < 2^32
uint64_t magic(int d) {
  const uint64_t dd = (uint64_t)std::max(d, 1);
  return ((uint64_t(1) << 32) + dd - 1) / dd;
}

void set_magics(fm::PassDesc* d) {
  d->mag_in = magic(d->in_n);
  d->mag_out = magic(d->out_n);
  d->mag_B = magic(d->B);
  d->mag_spec = magic(d->spec_n);
  d->mag_gline = magic(d->g.F_line);
}

bool pass_in_bounds(const fm::PassDesc& d, int64_t in_size, int64_t out_size, size_t elem);
int64_t tile_in_span_bytes(const fm::PassDesc& d, size_t elem);

// LDS layout of one tile: the FFT buffer and the raw input tile (the raw tile aliases the
// buffer, except for fused real-to-real tiles, which keep it and their real spectrum
// after the buffer), then the fused tile's Green rows at g_off, then the twiddle tables
// of the persistent kernels at tab_off.  Returns the total bytes.
struct TileLds {
  size_t raw_off, g_off, tab_off, total;
};
TileLds tile_lds(const fm::PassDesc& d, int B, size_t elem, int comps, bool fused_r2r) {
  const int packs = (d.gather == fm::G_CPLX) ? 1 : 2;
  const size_t cplx = 2 * elem;
  const size_t in_elem = d.in_cplx ? cplx : elem;
  const int F = comps * ((B + packs - 1) / packs);
  const size_t fft = (size_t)F * fm::fft_line_stride(d.M) * cplx;
  const size_t raw = (size_t)comps * B * (d.in_n + 1) * in_elem;
  TileLds t{};
  size_t end;
  if (d.gather == fm::G_R2R && fused_r2r) {
    t.raw_off = round256(fft);
    end = t.raw_off + std::max(raw, (size_t)B * (d.spec_n + 1) * elem);
  } else {
    end = std::max(fft, raw);
  }
  if (d.fused) {
    t.g_off = round256(end);
    end = t.g_off + (size_t)B * d.g.F_line * elem;
  }
  if (d.stw_n + d.tw_n > 0) {
    t.tab_off = round256(end);
    end = t.tab_off + (size_t)(d.stw_n + d.tw_n) * cplx;
  }
  t.total = round256(end);
  return t;
}

// FP32 one-launch batches and the FP32 fused real-to-real kernel of length 32 are off
// in the library (an FP32 batched test faulted the GPU with no cause shown).  The CPU
// emulation build of the device code (tests/emu) defines FM_FP32_ONE_LAUNCH to replay
// those paths under the sanitizers.
#ifdef FM_FP32_ONE_LAUNCH
constexpr bool kFp32OneLaunch = true;
#else
constexpr bool kFp32OneLaunch = false;
#endif

// Kernel length class that fixes the values per thread of a pass.
int pass_class(const fm::PassDesc& d) { return d.long_rt ? fm::kRtLong : d.M; }

// Whether a pass runs in the compile-time-length kernel of its FFT length (else in the
// runtime-length kernel).  FP32 fused real-to-real passes of length 32 are kept on the
// runtime-length kernel: the compile-time one ran only in a test that faulted the GPU,
// and nothing has shown it free of that fault.
bool compile_time_kernel(const fm::PassDesc& d, size_t elem) {
  if (d.long_rt || !fm::is_fast_len(d.M)) return false;
  if (!kFp32OneLaunch && elem == 4 && d.fused && d.gather == fm::G_R2R && d.M == 32) return false;
  return true;
}

// Twiddle entries the persistent kernel of this pass copies to LDS: the stage table,
// and for real-to-real gathers the first 2M entries of the 4M table (pre- and
// post-twiddles).  Descriptors with lds_tabs = 0 read them from global memory.
void set_lds_tables(fm::PassDesc* d, size_t elem) {
  d->stw_n = d->tw_n = 0;
  if (!d->lds_tabs || !compile_time_kernel(*d, elem) || !fm::pipelined_kernel((int)elem, d->M))
    return;
  d->stw_n = fm::stage_table_size(d->M, fm::max_radix((int)elem));
  if (d->gather == fm::G_R2R) d->tw_n = 2 * d->M;
}

// Largest tile (lines per workgroup) that fits the register budget and, if possible,
// the preferred LDS size; otherwise the largest that fits the device's LDS.
int choose_tile(fm::PassDesc* d, size_t elem, int comps, bool fused_r2r, int nb, int bmax = 64) {
  const int packs = (d->gather == fm::G_CPLX) ? 1 : 2;
  set_lds_tables(d, elem);
  for (const int cap : {fm::kSoftLds, fm::kMaxLds}) {
    int best = 0;
    TileLds best_lds{};
    for (int B = 1; B <= bmax; ++B) {
      const int F = comps * ((B + packs - 1) / packs);
      const int cls = pass_class(*d);
      if ((int64_t)F * d->M > (int64_t)fm::kThreads * fm::elems_per_thread((int)elem, cls)) break;
      // the register stage must hold the whole input tile (a Hermitian half-spectrum
      // pair has M + 2 values per FFT line), and a fused tile's Green rows
      if ((int64_t)B * d->in_n > (int64_t)fm::kThreads * fm::stage_values((int)elem, cls, d->in_cplx != 0, comps))
        break;
      if (d->fused && (int64_t)B * d->g.F_line >
                          (int64_t)fm::kThreads * fm::green_values((int)elem, cls, packs == 2))
        break;
      const TileLds t = tile_lds(*d, B, elem, comps, fused_r2r);
      if (t.total > (size_t)cap) break;
      best = B;
      best_lds = t;
      if (B >= nb) break;
    }
    if (best > 0) {
      d->B = best;
      d->lds_bytes = (int)best_lds.total;
      d->raw_off = (int)best_lds.raw_off;
      d->g_off = (int)best_lds.g_off;
      d->tab_off = (int)best_lds.tab_off;
      return FM_OK;
    }
  }
  return FM_E_SIZE;
}

// The per-wavefront fused kernel (fm_wave.h) with E values per lane: complex fused
// passes of a power-of-two length whose lines are contiguous in memory (every fused
// complex pass: the last axis is the fastest of its layout); three-component lines of 16
// values per lane in FP64 only at 1024 points (one line per wavefront) and without a
// second symmetric axis.
int wave_plain_rs(const fm::PassDesc& d, int E);

bool wave_capable(const fm::PassDesc& d, size_t elem, int E) {
  // the kernels are compiled with the compile-time-length classes (fm_inst.hip)
  if (d.long_rt || !fm::wave_length(d.M, E) || !fm::is_fast_len(d.M)) return false;
  if (E == 32 && (!d.fused || d.g.curl || elem != 4)) return false;  // FP32 Poisson lines only
  if (!d.fused && d.gather == fm::G_R2R && d.out_cplx) return false;  // LDS-tile kernel only
  if (!d.fused) return wave_plain_rs(d, E) > 0;
  if (d.gather != fm::G_CPLX) return false;
  if (d.g.curl && elem != 4 && E == 16 && (d.M != 1024 || d.g.csym_b != 0)) return false;
  return d.in_s_line == 1 && d.out_s_line == 1;
}

// The per-wavefront plain kernel (fm_wave.h, wave_plain_tile): any unfused pass of a
// power-of-two length.  Its tile is four wavefronts of L = wave_lines(M, E) FFT lines,
// pk tile lines per FFT line (2 for the packed real kinds).  The raw lines of a
// wavefront share the LDS region of its FFT lines (L line strides of complex values):
// returns their stride in input elements (odd when there is room, against LDS bank
// conflicts between consecutive lines), or 0 when the lines do not fit.
int wave_plain_pk(const fm::PassDesc& d) { return d.gather == fm::G_CPLX ? 1 : 2; }

int wave_plain_rs(const fm::PassDesc& d, int E) {
  if (d.fused || !fm::wave_length(d.M, E) || d.in_n < 1) return 0;
  const int pk = wave_plain_pk(d);
  const int cap = fm::fft_line_stride(d.M) * (d.in_cplx ? 1 : 2) / pk;  // per raw line
  const int rs = d.in_n | 1;
  if (rs <= cap) return rs;
  return d.in_n <= cap ? d.in_n : 0;
}

// LDS tables of the plain per-wavefront kernel after its FFT lines: stage twiddles; for
// real-to-real passes the post-twiddles (2M entries of the 4M table) and M gather slots
// (weight and source index, R2RSlot).
size_t wave_plain_tab_bytes(const fm::PassDesc& d, int E, size_t elem) {
  const bool r2r = d.gather == fm::G_R2R;
  return (size_t)(fm::wave_tw_size(d.M, E) + (r2r ? 2 * d.M : 0)) * 2 * elem +
         (r2r ? (size_t)d.M * (2 * elem + 8) : 0);
}

// Input values per thread of the plain per-wavefront kernel's register stage.
int wave_plain_u(const fm::PassDesc& d, int E) { return d.gather == fm::G_REAL2 ? 2 * E + 1 : E + 1; }

bool wave_capable(const fm::PassDesc& d, size_t elem) {
  return wave_capable(d, elem, 16) || wave_capable(d, elem, 8);
}

// Values per lane the planner gives a fused pass in the per-wavefront kernel: 8 for
// three-component lines when their length allows it (three 8-value FP32 lines fit the
// registers of three waves per SIMD, three 16-value lines need the 256 of two), else
// 16.  FP64 three-component lines stay on the LDS-tile kernel unless the tuner picks
// otherwise.
int default_wave_values(const fm::PassDesc& d, size_t elem) {
  if (d.g.curl && wave_capable(d, elem, 8)) return 8;
  return wave_capable(d, elem, 16) ? 16 : 8;
}

size_t wave_lds(int B, int M, size_t elem) {
  return round256((size_t)B * fm::fft_line_stride(M) * 2 * elem);
}

// Pass d in the per-wavefront kernel with E values per lane and W (1, 2 or 4) wavefronts
// per workgroup; false if it cannot run there.  comp_tiles: tiles per (b, c) tile
// position (ncomp, or 1 for the three-component curl).
bool set_wave(fm::PassDesc* d, size_t elem, int W, int comp_tiles, int E) {
  if (!wave_capable(*d, elem, E) || (W != 1 && W != 2 && W != 4)) return false;
  // plain passes: four wavefronts (the tile's loads and stores use every thread)
  if (!d->fused && W != 4) return false;
  const int F = W * fm::wave_lines(d->M, E);  // FFT lines per workgroup
  const int B = d->fused ? F : F * wave_plain_pk(*d);
  const size_t lds = wave_lds(F, d->M, elem);
  if (lds > (size_t)fm::kMaxLds) return false;
  if (!d->fused && (int64_t)B * d->in_n > (int64_t)fm::kThreads * wave_plain_u(*d, E)) return false;
  size_t total = lds;
  if (!d->fused) {
    // the plain kernel's tables follow the FFT lines: stage twiddles, then the
    // real-to-real post-twiddles (2M entries of the 4M table)
    total = round256(lds + wave_plain_tab_bytes(*d, E, elem));
    if (total > (size_t)fm::kMaxLds) return false;
  }
  d->wave = E;
  d->wave_rs = d->fused ? 0 : wave_plain_rs(*d, E);
  d->B = B;
  d->lds_bytes = (int)total;
  d->raw_off = d->g_off = d->tab_off = 0;
  if (!d->fused) d->tab_off = (int)lds;
  d->stw_n = d->tw_n = 0;
  d->persist = 0;
  d->lds_tabs = 0;
  d->tiles = ((d->nb + B - 1) / B) * d->nc * comp_tiles;
  set_magics(d);
  return true;
}

// Fill the geometry of a pass: lines along `la`, tiles along `lb`, index `lc`.
void set_geometry(fm::PassDesc* d, int la, int lb, int lc, const int64_t sin_[3], int64_t in_size,
                  const int64_t sout[3], int64_t out_size, const int ext_b[3]) {
  d->in_s_line = sin_[la];
  d->in_s_b = sin_[lb];
  d->in_s_c = sin_[lc];
  d->in_s_comp = in_size;
  d->out_s_line = sout[la];
  d->out_s_b = sout[lb];
  d->out_s_c = sout[lc];
  d->out_s_comp = out_size;
  d->nb = ext_b[lb];
  d->nc = ext_b[lc];
}

void set_transform(fm::PassDesc* d, const AxisPlan& a, bool forward, bool fused_half) {
  (void)fused_half;
  if (!a.dft) {
    d->gather = fm::G_R2R;
    d->scatter = fm::S_R2R;
    d->sign = -1;
    d->r2r = make_r2r(a, forward ? a.fwd : a.bwd, forward);
    d->in_cplx = d->out_cplx = 0;
    return;
  }
  if (a.first_dft) {
    if (forward) {
      d->gather = fm::G_REAL2;
      d->scatter = fm::S_R2C2;
      d->sign = -1;
      d->n_data = a.n_data;
      d->in_cplx = 0;
      d->out_cplx = 1;
    } else {
      d->gather = fm::G_HERM2;
      d->scatter = fm::S_REAL2;
      d->sign = +1;
      d->in_cplx = 1;
      d->out_cplx = 0;
    }
  } else {
    d->gather = fm::G_CPLX;
    d->scatter = fm::S_CPLX;
    d->sign = forward ? -1 : +1;
    d->n_data = forward ? a.n_data : a.M;
    d->in_cplx = d->out_cplx = 1;
  }
}

// Release the generation temporaries of a plan (its generation work has completed).
void release_generation(fm_plan_s* p) {
  for (void* ptr : p->gen_free) (void)hipFree(ptr);
  p->gen_free.clear();
  p->gen_desc.clear();
  for (auto& kv : p->tw64) (void)hipFree(kv.second);
  p->tw64.clear();
}

// Whether pass i of a plan runs once per component (vector plans: passes 1 and 5, and 2
// and 4 with a second symmetric axis).
bool vec_pass(const fm_plan_s* p, int i) {
  return p->vec && (i == 0 || i == 4 || ((p->vec2 || p->vec3) && (i == 1 || i == 3)) ||
                    (p->vec3 && (i == 5 || i == 6)));
}
// Per-component transform of pass i (vr2r's second index).
int vec_r2r(int i) { return i == 0 ? 0 : i == 4 ? 1 : i == 1 ? 2 : i == 3 ? 3 : i == 5 ? 4 : 5; }
// Device slot, after the kPasses, of component q (1 or 2) of pass i of a vector plan.
int vec_slot(int i, int q) { return 2 * vec_r2r(i) + (q - 1); }

// The descriptors of components 1 and 2 of the per-component passes of a vector plan,
// rebuilt from the plan's (component 0) descriptors with their own transforms, and
// uploaded.
hipError_t upload_vec_descs(fm_plan_s* p, hipStream_t st) {
  for (const int i : {0, 1, 3, 4, 5, 6}) {
    if (!vec_pass(p, i)) continue;
    for (int q = 1; q < 3; ++q) {
      fm::PassDesc& d = p->vdesc[vec_slot(i, q)];
      d = p->pass[i];
      d.r2r = p->vr2r[q][vec_r2r(i)];
      if (i == 4) {
        d.fix = p->vfix[q];
        d.has_fix = p->vhas_fix[q];
      }
    }
  }
  const hipError_t e = hipMemcpyAsync(p->dpass + fm_plan_s::kPasses, p->vdesc, sizeof(p->vdesc),
                                      hipMemcpyHostToDevice, st);
  return e == hipSuccess ? hipStreamSynchronize(st) : e;
}

// Twiddle tables and the Green's spectrum of a plan, generated on stream st.  With
// deferred = false the call waits for the generation and releases its temporaries; with
// deferred = true it records p->ready after the generation instead and leaves the
// release to finish_generation.
template <typename T>
int make_tables_and_green(fm_plan_s* p, hipStream_t st, bool deferred) {
  // twiddle tables for every FFT length of the passes
  for (int i = 0; i < fm_plan_s::kPasses; ++i) {
    const int M = p->pass[i].M;
    if (p->tw.count(M)) continue;
    void* ptr = nullptr;
    if (plan_malloc(&ptr, sizeof(T) * 2 * 4 * (size_t)M) != hipSuccess) return FM_E_NOMEM;
    p->tw[M] = ptr;
    p->table_bytes += sizeof(T) * 2 * 4 * (size_t)M;
    FM_HIP(fm::launch_twiddles<T>(ptr, M, st));
  }
  for (int i = 0; i < fm_plan_s::kPasses; ++i) p->pass[i].tw = p->tw[p->pass[i].M];
  // per-stage tables of the lengths with compile-time kernels; also of a pass planned in
  // the runtime-length class that the tuner may move to the per-wavefront kernel (the
  // table selects the compile-time class at launch, fm_plan_s::stw_plan keeps the planned
  // choice)
  for (int i = 0; i < fm_plan_s::kPasses; ++i) {
    const int M = p->pass[i].M;
    fm::PassDesc c = p->pass[i];
    c.long_rt = 0;
    const bool planned = compile_time_kernel(p->pass[i], p->elem);
    if (!planned && !(p->long_rt[i] && wave_capable(c, p->elem))) continue;
    if (tile_in_span_bytes(p->pass[i], p->elem) >= (int64_t(1) << 32)) continue;
    if (!p->stw.count(M)) {
      void* ptr = nullptr;
      const size_t n = (size_t)std::max(1, fm::stage_table_size(M, fm::max_radix((int)sizeof(T))));
      if (plan_malloc(&ptr, sizeof(T) * 2 * n) != hipSuccess) return FM_E_NOMEM;
      p->stw[M] = ptr;
      p->table_bytes += sizeof(T) * 2 * n;
      FM_HIP(fm::launch_stage_twiddles<T>(ptr, M, st));
    }
    if (planned) p->pass[i].stw = p->stw[M];
  }
  for (int i = 0; i < fm_plan_s::kPasses; ++i) p->stw_plan[i] = p->pass[i].stw;

  // stage twiddles of the per-wavefront kernels (a pass may run there, now or after
  // tuning), one table per length and values per lane
  for (int i = 0; i < 5; ++i) {
    fm::PassDesc w = p->pass[i];
    w.long_rt = 0;  // the per-wavefront kernels take the compile-time length class
    for (const int E : {16, 8, 32}) {
      if (!wave_capable(w, p->elem, E)) continue;
      const int M = p->pass[i].M;
      const int key = (M << 6) | E;
      if (!p->wtw.count(key)) {
        void* ptr = nullptr;
        const size_t n = (size_t)std::max(1, fm::wave_tw_size(M, E));
        if (plan_malloc(&ptr, sizeof(T) * 2 * n) != hipSuccess) return FM_E_NOMEM;
        p->wtw[key] = ptr;
        p->table_bytes += sizeof(T) * 2 * n;
        FM_HIP(fm::launch_wave_twiddles<T>(ptr, M, E, st));
      }
      (E == 16 ? p->pass[i].wtw : (E == 8 ? p->pass[i].wtw8 : p->pass[i].wtw32)) = p->wtw[key];
    }
  }

  // the curl's derivative factor of every DFT mode k (signed k_s) of the three directions
  // of the fused pass, in FP64, rounded once: the wavenumber 2 pi k_s / period (0 at the
  // Nyquist mode), or the central-difference symbol (1/h) sum_j c_j sin(2 pi j k_s / M)
  if (p->pass[2].g.curl || p->vec3) {
    fm::GreenRef& g = p->pass[2].g;
    const int order = g.deriv;
    const int axes[3] = {g.axis_line, g.axis_b, g.axis_c};
    const int Ms[3] = {g.M_line, g.M_b, g.M_c};
    const double dws[3] = {g.dw_line, g.dw_b, g.dw_c};
    std::vector<T> host;
    size_t offs[3];
    for (int t = 0; t < 3; ++t) {
      offs[t] = host.size();
      const double ih = 1.0 / p->ax[axes[t]].h;
      const int M = Ms[t];
      const AxisPlan& A = p->ax[axes[t]];
      if (!A.dft) {
        // the swap axis of a vector plan (direction c): frequency index s (+ 1/2 for the
        // half-frequency kinds) on the period 2 nh of its transform (nh = N, or 2N on the
        // 2L extension of a semi-unbounded axis): w = pi (2 s + b2) / (2 nh h)
        const int b2 = kind_form(A.fwd).b2;
        const long long nh = A.unb ? 2LL * A.N : (long long)A.N;
        for (int k = 0; k < A.nspec; ++k) {
          auto sn = [&](int j) {  // sin(j w h), the angle reduced exactly
            const long long num = ((long long)j * (2LL * k + b2)) % (4LL * nh);
            return std::sin(M_PI * (double)num / (2.0 * (double)nh));
          };
          double v;
          if (order == 0) v = M_PI * (2.0 * k + b2) / (2.0 * (double)nh * A.h);
          else if (order == 2) v = ih * sn(1);
          else if (order == 4) v = ih * (4.0 / 3.0 * sn(1) - 1.0 / 6.0 * sn(2));
          else v = ih * (1.5 * sn(1) - 0.3 * sn(2) + sn(3) / 30.0);
          host.push_back(T(v));
        }
        continue;
      }
      for (int k = 0; k < M; ++k) {
        const long long ks = (2 * k > M) ? k - M : k;
        auto sn = [&](int j) {  // sin(2 pi j ks / M), the angle reduced exactly
          long long num = (2LL * j * ks) % (2LL * M);
          if (num < 0) num += 2LL * M;
          return std::sin(M_PI * (double)num / (double)M);
        };
        double v;
        if (order == 0) v = (2 * k == M) ? 0.0 : dws[t] * (double)ks;
        else if (order == 2) v = ih * sn(1);
        else if (order == 4) v = ih * (4.0 / 3.0 * sn(1) - 1.0 / 6.0 * sn(2));
        else v = ih * (1.5 * sn(1) - 0.3 * sn(2) + sn(3) / 30.0);
        host.push_back(T(v));
      }
    }
    void* ptr = nullptr;
    if (plan_malloc(&ptr, sizeof(T) * host.size()) != hipSuccess) return FM_E_NOMEM;
    p->dtab = ptr;
    p->table_bytes += sizeof(T) * host.size();
    FM_HIP(hipMemcpy(ptr, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
    T* base = reinterpret_cast<T*>(ptr);
    g.dtab_line = base + offs[0];
    g.dtab_b = base + offs[1];
    g.dtab_c = base + offs[2];
  }

  // Green's spectrum: sample (FP64) -> DCT-I along convolution directions -> scale
  const int* o = p->order;  // table axes = (a0, a1, a2), slow -> fast
  fm::GreenGen g{};
  int du = 0;
  double vol = 1.0, scale = 1.0;
  int Fs[3], F[3], off[3];
  for (int i = 0; i < 3; ++i) {
    const AxisPlan& a = p->ax[o[i]];
    Fs[i] = a.Fs;
    F[i] = a.F;
    off[i] = a.off;
    g.n[i] = a.Fs;
    g.unb[i] = a.unb ? 1 : 0;
    g.h[i] = a.h;
    g.dw[i] = a.dw;
    g.shift[i] = a.shift;
    if (a.unb) {
      du++;
      vol *= a.h;
      scale *= a.h;
    }
    scale /= a.nlog;
  }
  g.du = du;
  g.variant = p->green;
  g.cellvol = vol;
  if (du == 3) g.r_eq = std::cbrt(3.0 * vol / (4.0 * M_PI));
  if (du == 2) g.r_eq = std::sqrt(vol / M_PI);
  if (p->green >= FM_GREEN_HEJ2) {
    const double hc = std::cbrt(p->h[0] * p->h[1] * p->h[2]);
    g.eps = 2.0 * hc;
    g.kc = M_PI / hc;
  }
  const int64_t ns = (int64_t)Fs[0] * Fs[1] * Fs[2];
  double* S = nullptr;
  if (plan_malloc(&S, sizeof(double) * ns) != hipSuccess) return FM_E_NOMEM;
  p->gen_free.push_back(S);
  int rc = FM_OK;
  if (p->green == FM_GREEN_LGF2 && du == 3) {
    // lattice Green's function: Bessel rows of the quadrature nodes, then the samples
    fm::LgfGen lg{};
    int nmax = 1;
    double hmin = 1e300, hmax = 0.0;
    for (int i = 0; i < 3; ++i) {
      lg.nA[i] = Fs[i];
      lg.h[i] = g.h[i];
      nmax = std::max(nmax, Fs[i]);
      hmin = std::min(hmin, g.h[i]);
      hmax = std::max(hmax, g.h[i]);
    }
    lg.stride = nmax;
    lg.du = 0.125;
    lg.c = 2.0 * hmax * hmax;
    lg.u_lo = std::log(hmin * hmin) - 38.0;
    const double u_hi = std::log(hmax * hmax * (1.0 + (double)nmax * nmax)) + 28.0;
    lg.K = (int)std::ceil((u_hi - lg.u_lo) / lg.du) + 1;
    double* A = nullptr;
    double* W = nullptr;
    if (plan_malloc(&A, sizeof(double) * 3 * (size_t)lg.K * lg.stride) != hipSuccess) return FM_E_NOMEM;
    p->gen_free.push_back(A);
    if (plan_malloc(&W, sizeof(double) * 2 * (size_t)lg.K) != hipSuccess) return FM_E_NOMEM;
    p->gen_free.push_back(W);
    FM_HIP(fm::launch_lgf(S, A, W, lg, st));
  } else {
    FM_HIP(fm::launch_green_sample(S, g, st));
  }
  int64_t sstr[3] = {(int64_t)Fs[1] * Fs[2], Fs[2], 1};
  p->gen_desc.assign(3, fm::PassDesc{});  // host copies stay alive until the copies ran
  fm::PassDesc* gdesc = p->gen_desc.data();
  fm::PassDesc* gdev = nullptr;
  if (plan_malloc(&gdev, sizeof(fm::PassDesc) * 3) != hipSuccess) return FM_E_NOMEM;
  p->gen_free.push_back(gdev);
  for (int i = 0; i < 3 && rc == FM_OK; ++i) {
    if (!g.unb[i]) continue;
    // DCT-I (REDFT00) of Fs[i] samples, in place along table axis i
    fm::PassDesc d{};
    const int n = Fs[i];
    const KindForm f = kind_form(REDFT00);
    fm::R2R r{};
    r.nh = n - 1; r.a2 = 0; r.b2 = 0; r.sin = 0;
    r.plo = 0; r.phi = n - 1; r.wlo = f.wlo; r.whi = f.whi;
    r.in_rev = 0; r.in_base = 0; r.qlo = 0; r.qhi = n - 1; r.out_rev = 0; r.out_base = 0;
    d.r2r = r;
    d.gather = fm::G_R2R;
    d.scatter = fm::S_R2R;
    d.sign = -1;
    if ((rc = radix_plan(2 * (n - 1), &d))) break;
    const int lb = (i == 2) ? 1 : 2;  // tile along the fastest other axis
    const int lc = 3 - i - lb;
    d.in = S;
    d.out = S;
    d.in_s_line = d.out_s_line = sstr[i];
    d.in_s_b = d.out_s_b = sstr[lb];
    d.in_s_c = d.out_s_c = sstr[lc];
    d.in_s_comp = d.out_s_comp = 0;
    d.nb = Fs[lb];
    d.nc = Fs[lc];
    d.ncomp = 1;
    d.in_n = d.out_n = n;
    if ((rc = choose_tile(&d, sizeof(double), 1, false, d.nb))) break;
    d.tiles = ((d.nb + d.B - 1) / d.B) * d.nc;
    set_magics(&d);
    if (!pass_in_bounds(d, ns, ns, sizeof(double))) { rc = FM_E_SIZE; break; }
    void* t64 = nullptr;
    auto it = p->tw64.find(d.M);
    if (it == p->tw64.end()) {
      if (plan_malloc(&t64, sizeof(double) * 2 * 4 * (size_t)d.M) != hipSuccess) { rc = FM_E_NOMEM; break; }
      p->tw64[d.M] = t64;
      FM_HIP(fm::launch_twiddles<double>(t64, d.M, st));
    } else {
      t64 = it->second;
    }
    d.tw = t64;
    d.kind = fm::K_R2R;
    gdesc[i] = d;
    FM_HIP(hipMemcpyAsync(gdev + i, &gdesc[i], sizeof(fm::PassDesc), hipMemcpyHostToDevice, st));
    FM_HIP(fm::launch_pass<double>(gdesc[i], gdev + i, S, S, st));
  }
  if (rc == FM_OK) {
    const int64_t nG = (int64_t)F[0] * F[1] * F[2];
    if (plan_malloc(&p->G, sizeof(T) * nG) != hipSuccess) {
      rc = FM_E_NOMEM;
    } else {
      p->table_bytes += sizeof(T) * nG;
      FM_HIP(fm::launch_green_final<T>(p->G, S, F, Fs, off, scale, st));
    }
  }
  // the pass descriptors, now complete, go to device memory
  for (int i = 0; i < fm_plan_s::kPasses; ++i) p->pass[i].g.G = p->G;
  if (p->vec3) {  // the real curl reads the same Green's table and derivative tables
    const fm::GreenRef& g = p->pass[2].g;
    p->vcurl.G = p->G;
    p->vcurl.d[0] = g.dtab_c;     // table axis a0 = direction c of pass 3
    p->vcurl.d[1] = g.dtab_b;
    p->vcurl.d[2] = g.dtab_line;
  }
  if (rc == FM_OK) {
    const size_t nb = sizeof(fm::PassDesc) * fm_plan_s::kPasses;
    const size_t nv = p->vec ? sizeof(fm::PassDesc) * fm_plan_s::kVecDesc : 0;
    if (plan_malloc(&p->dpass, nb + nv) != hipSuccess) rc = FM_E_NOMEM;
    else p->table_bytes += nb + nv;
    if (rc == FM_OK) FM_HIP(hipMemcpyAsync(p->dpass, p->pass, nb, hipMemcpyHostToDevice, st));
    if (rc == FM_OK && p->vec) FM_HIP(upload_vec_descs(p, st));
  }
  for (int i = 0; i < 3; ++i) p->GF[i] = F[i];
  if (deferred && rc == FM_OK) {
    FM_HIP(hipEventCreateWithFlags(&p->ready, hipEventDisableTiming));
    FM_HIP(hipEventRecord(p->ready, st));
    return FM_OK;
  }
  hipError_t e = hipStreamSynchronize(st);
  release_generation(p);
  if (rc) return rc;
  if (e != hipSuccess) { g_last_hip = (int)e; return FM_E_HIP; }
  return FM_OK;
}

void free_plan(fm_plan_s* p) {
  if (!p) return;
  if (p->ready) {
    (void)hipEventSynchronize(p->ready);
    (void)hipEventDestroy(p->ready);
  } else if (!p->gen_free.empty()) {
    (void)hipDeviceSynchronize();  // a failed creation: its generation work may be queued
  }
  release_generation(p);
  for (auto& kv : p->tw) (void)hipFree(kv.second);
  for (auto& kv : p->stw) (void)hipFree(kv.second);
  for (auto& kv : p->wtw) (void)hipFree(kv.second);
  if (p->dtab) (void)hipFree(p->dtab);
  if (p->G) (void)hipFree(p->G);
  if (p->dpass) (void)hipFree(p->dpass);
  if (p->ws_internal) (void)hipFree(p->ws_internal);
  delete p;
}

// The plan's own workspace, allocated on first use (under the plan's lock, so that two
// host threads solving with one plan allocate it once); nullptr if allocation fails.
char* own_workspace(fm_plan_s* p) {
  std::lock_guard<std::mutex> lock(p->ws_mu);
  if (!p->ws_internal && plan_malloc(&p->ws_internal, p->ws_bytes) != hipSuccess) {
    p->ws_internal = nullptr;
    return nullptr;
  }
  return reinterpret_cast<char*>(p->ws_internal);
}

int pass_kind(const fm::PassDesc& d) {
  if (d.fused) {
    if (d.gather == fm::G_R2R) return fm::K_F_R2R;
    if (d.gather == fm::G_REAL2) return fm::K_F_R2C;
    return d.g.curl ? fm::K_F_CURL : fm::K_F_C2C;
  }
  switch (d.gather) {
    case fm::G_CPLX: return d.sign < 0 ? fm::K_C2C_F : fm::K_C2C_I;
    case fm::G_REAL2: return fm::K_R2C;
    case fm::G_HERM2: return fm::K_C2R;
    default: return fm::K_R2R;
  }
}

// Input span of one tile in bytes (the fast kernels address it with 32-bit offsets).
int64_t tile_in_span_bytes(const fm::PassDesc& d, size_t elem) {
  const int64_t es = (int64_t)elem * (d.in_cplx ? 2 : 1);
  return ((int64_t)(d.B - 1) * d.in_s_b + (int64_t)(d.in_n - 1) * d.in_s_line + 1) * es;
}

// Host-side check of a pass in the per-wavefront kernel: what wave_tile touches.
bool wave_in_bounds(const fm::PassDesc& d, int64_t in_size, int64_t out_size, size_t elem) {
  auto span = [](int nc, int64_t sc, int nb, int64_t sb, int n, int64_t sl) {
    return (int64_t)(nc - 1) * sc + (int64_t)(nb - 1) * sb + (int64_t)(n - 1) * sl;
  };
  const int E = d.wave;
  if (!wave_capable(d, elem, E) || d.has_fix) return false;
  const int L = fm::wave_lines(d.M, E);
  if (L < 1) return false;
  const int W = d.B / L;
  if (d.B % L || (W != 1 && W != 2 && W != 4)) return false;
  if (d.nb < 1 || d.nc < 1 || d.in_n < 1 || d.out_n < 1) return false;
  if (d.n_data < 0 || d.n_data > d.in_n || d.n_data > d.M || d.out_n > d.M) return false;
  int prodR = 1;
  for (int i = 0; i < d.nstages; ++i) prodR *= d.radix[i];
  if (prodR != d.M) return false;
  if (span(d.nc, d.in_s_c, d.nb, d.in_s_b, d.in_n, d.in_s_line) >= in_size) return false;
  if (span(d.nc, d.out_s_c, d.nb, d.out_s_b, d.out_n, d.out_s_line) >= out_size) return false;
  const int comps = d.g.curl ? 3 : d.ncomp;
  if (d.g.curl && d.ncomp != 3) return false;
  if (comps > 1 && (d.in_s_comp < in_size || d.out_s_comp < out_size)) return false;
  if (d.g.fold_line != d.M || d.g.F_line < d.M / 2 + 1) return false;
  if ((size_t)d.lds_bytes < wave_lds(d.B, d.M, elem) || d.lds_bytes > fm::kMaxLds) return false;
  const int nbt = (d.nb + d.B - 1) / d.B;
  return d.tiles == nbt * d.nc * (d.g.curl ? 1 : d.ncomp);
}

// Host-side check of one pass against the buffers and the LDS / register budgets; the
// index ranges mirror what the tile kernels touch.
bool pass_in_bounds(const fm::PassDesc& d, int64_t in_size, int64_t out_size, size_t elem) {
  if (d.wave && d.fused) return wave_in_bounds(d, in_size, out_size, elem);
  auto span = [](int nc, int64_t sc, int nb, int64_t sb, int n, int64_t sl) {
    return (int64_t)(nc - 1) * sc + (int64_t)(nb - 1) * sb + (int64_t)(n - 1) * sl;
  };
  if (d.nb < 1 || d.nc < 1 || d.in_n < 1 || d.out_n < 1 || d.B < 1) return false;
  if (span(d.nc, d.in_s_c, d.nb, d.in_s_b, d.in_n, d.in_s_line) >= in_size) return false;
  if (span(d.nc, d.out_s_c, d.nb, d.out_s_b, d.out_n, d.out_s_line) >= out_size) return false;
  if (d.has_fix) {
    const int bl = d.fix.b_dup ? std::max(d.nb, d.fix.b_last + 1) : d.nb;
    const int cl = d.fix.c_dup ? std::max(d.nc, d.fix.c_last + 1) : d.nc;
    if (span(cl, d.out_s_c, bl, d.out_s_b, d.out_n, d.out_s_line) >= out_size) return false;
    if (d.fused || d.out_cplx) return false;  // applied by the real-output last pass only
  }
  if (d.in_s_comp < in_size && d.ncomp > 1 && !(d.fused && d.g.curl && d.ncomp == 3)) return false;
  const int M = d.M;
  int prodR = 1;
  for (int i = 0; i < d.nstages; ++i) prodR *= d.radix[i];
  if (prodR != M || M < 2 || M > fm::kMaxLen) return false;
  auto r2r_ok = [&](const fm::R2R& r) { return 2 * r.nh == M && r.qhi < M && r.qlo >= 0 && r.plo >= 0 && r.phi <= r.nh; };
  switch (d.gather) {
    case fm::G_CPLX: case fm::G_REAL2: if (d.n_data > d.in_n || d.n_data > M) return false; break;
    case fm::G_HERM2: if (d.in_n < M / 2 + 1) return false; break;
    case fm::G_R2R: if (!r2r_ok(d.r2r)) return false; break;
    default: return false;
  }
  if (!d.fused) {
    switch (d.scatter) {
      case fm::S_CPLX: case fm::S_REAL2: if (d.out_n > 2 * M) return false; break;
      case fm::S_R2C2: if (d.out_n > M / 2 + 1) return false; break;
      case fm::S_R2R: if (!r2r_ok(d.r2r)) return false; break;
      default: return false;
    }
  } else {
    if (d.gather == fm::G_R2R && (!r2r_ok(d.r2r2) || d.spec_n < 1)) return false;
    if (d.gather != fm::G_R2R && d.out_n > 2 * M) return false;
    if (d.g.curl && d.gather != fm::G_CPLX) return false;
  }
  const int comps = (d.fused && d.g.curl) ? 3 : 1;
  const int packs = (d.gather == fm::G_CPLX) ? 1 : 2;
  const int F = comps * ((d.B + packs - 1) / packs);
  if (d.wave) {
    // plain pass in the per-wavefront kernel: four wavefronts of wave_lines FFT lines, the
    // raw lines of each inside its LDS region, the register stage holds the tile
    const int E = d.wave;
    if (d.fused || !wave_capable(d, elem, E) || d.wave_rs != wave_plain_rs(d, E)) return false;
    const int L = fm::wave_lines(M, E);
    if (d.B != 4 * L * packs || (int64_t)d.B * d.in_n > (int64_t)fm::kThreads * wave_plain_u(d, E))
      return false;
    if (d.wave_rs < d.in_n || (int64_t)L * packs * d.wave_rs >
                                  (int64_t)L * fm::fft_line_stride(M) * (d.in_cplx ? 1 : 2))
      return false;
    const size_t tabs = wave_plain_tab_bytes(d, E, elem);
    if ((size_t)d.tab_off < wave_lds(4 * L, M, elem) || d.tab_off % 16 ||
        (size_t)d.tab_off + tabs > (size_t)d.lds_bytes || d.lds_bytes > fm::kMaxLds)
      return false;
    if (d.raw_off != 0 || d.stw_n + d.tw_n != 0) return false;
    if (tile_in_span_bytes(d, elem) >= (int64_t(1) << 32)) return false;
    // the output of a tile is addressed with 32-bit element offsets
    const int64_t out_span = (int64_t)(d.B - 1) * d.out_s_b + (int64_t)(d.out_n - 1) * d.out_s_line + 1;
    if (out_span >= (int64_t(1) << 31)) return false;
    const int nbt = (d.nb + d.B - 1) / d.B;
    return d.tiles == nbt * d.nc * d.ncomp;
  }
  const int cls = pass_class(d);
  if (d.long_rt && elem != 8) return false;
  if ((int64_t)F * M > (int64_t)fm::kThreads * fm::elems_per_thread((int)elem, cls)) return false;
  if ((int64_t)d.B * d.in_n > (int64_t)fm::kThreads * fm::stage_values((int)elem, cls, d.in_cplx != 0, comps))
    return false;
  const size_t fft = (size_t)F * fm::fft_line_stride(M) * 2 * elem;
  const size_t raw = (size_t)comps * d.B * (d.in_n + 1) * (d.in_cplx ? 2 : 1) * elem;
  size_t need = std::max(fft, raw);
  if (d.gather == fm::G_R2R && d.fused) {
    if ((size_t)d.raw_off < fft) return false;
    need = std::max(d.raw_off + raw, d.raw_off + (size_t)d.B * (d.spec_n + 1) * elem);
  } else if (d.raw_off != 0) {
    return false;
  }
  // the staged regions follow the tile, in order, inside lds_bytes
  size_t end = need;
  if (d.fused) {
    if ((int64_t)d.B * d.g.F_line > (int64_t)fm::kThreads * fm::green_values((int)elem, cls, packs == 2))
      return false;
    if ((size_t)d.g_off < end || d.g_off % 16) return false;
    end = d.g_off + (size_t)d.B * d.g.F_line * elem;
  }
  if (d.stw_n + d.tw_n > 0) {
    if (d.stw_n != fm::stage_table_size(M, fm::max_radix((int)elem))) return false;
    if (d.tw_n != 0 && (d.gather != fm::G_R2R || d.tw_n != 2 * M)) return false;
    if ((size_t)d.tab_off < end || d.tab_off % 16) return false;
    end = d.tab_off + (size_t)(d.stw_n + d.tw_n) * 2 * elem;
  }
  if (end > (size_t)d.lds_bytes || d.lds_bytes > fm::kMaxLds) return false;
  const int nbt = (d.nb + d.B - 1) / d.B;
  if (d.tiles != nbt * d.nc * (comps == 3 ? 1 : d.ncomp)) return false;
  return true;
}

int build_plan(fm_plan_s* p) {
  const bool node = p->layout == FM_NODE;
  for (int a = 0; a < 3; ++a) {
    const int rc = plan_axis(p->n[a], p->h[a], node, p->bc[a][0], p->bc[a][1], &p->ax[a]);
    if (rc) return rc;
  }
  if (p->green >= FM_GREEN_HEJ2) {  // regularised kernels: all directions unbounded or none
    const int nu = (int)p->ax[0].unb + (int)p->ax[1].unb + (int)p->ax[2].unb;
    if (nu != 0 && nu != 3) return FM_E_KIND;
  }
  // conditions per component (fm_plan_create_vector): the transforms of every component,
  // of the source (vin) and of the velocity (vout, even and odd faces swapped)
  AxisPlan vin[3][3], vout[3][3];
  bool swap[3] = {false, false, false};
  if (p->vec) {
    auto sw = [](int b) { return b == FM_BC_EVEN ? FM_BC_ODD : (b == FM_BC_ODD ? FM_BC_EVEN : b); };
    for (int q = 0; q < 3; ++q)
      for (int a = 0; a < 3; ++a) {
        int rc = plan_axis(p->n[a], p->h[a], node, p->bcv[q][a][0], p->bcv[q][a][1], &vin[q][a]);
        if (rc) return rc;
        rc = plan_axis(p->n[a], p->h[a], node, sw(p->bcv[q][a][0]), sw(p->bcv[q][a][1]), &vout[q][a]);
        if (rc) return rc;
      }
    // one or two symmetric or semi-unbounded axes; at least one periodic or unbounded
    int nswap = 0;
    for (int a = 0; a < 3; ++a)
      if (!p->ax[a].dft) {
        swap[a] = true;
        ++nswap;
      }
    if (nswap == 0) return FM_E_KIND;
    p->vec2 = nswap == 2;
    p->vec3 = nswap == 3;
    // spectral extent along each: every frequency index of the components' kinds
    for (int a = 0; a < 3; ++a) {
      if (!swap[a]) continue;
      int ns = 0;
      for (int q = 0; q < 3; ++q) {
        const AxisPlan& ai = vin[q][a];
        const AxisPlan& ao = vout[q][a];
        ns = std::max(ns, kind_form(ai.fwd).qout + ai.nin);
        ns = std::max(ns, kind_form(ao.bwd).pin + ao.nin);
      }
      p->ax[a].nspec = ns;
    }
  }
  if (p->kind != FM_POISSON) {
    if (p->ncomp != 3) return FM_E_KIND;
    for (int a = 0; a < 3; ++a)
      if (!p->ax[a].dft && !swap[a]) return FM_E_KIND;
  }
  // transform order: symmetric < semi-unbounded < periodic < unbounded (cost)
  auto cost = [](int c) {
    if (c >= C_EE && c <= C_OE) return 0;
    if (c >= C_EU) return 1;
    if (c == C_P) return 2;
    return 3;
  };
  int ord[3] = {0, 1, 2};
  std::stable_sort(ord, ord + 3, [&](int x, int y) { return cost(p->ax[x].cls) < cost(p->ax[y].cls); });
  for (int i = 0; i < 3; ++i) p->order[i] = ord[i];
  bool seen_dft = false;
  for (int i = 0; i < 3; ++i) {
    AxisPlan& a = p->ax[ord[i]];
    // with two symmetric axes of a vector plan the DFT axis is a full complex DFT (the
    // curl mixes the components line by line, which two real lines packed in one complex
    // FFT would not allow)
    if (a.dft && !seen_dft && !p->vec2) a.first_dft = true;
    if (a.dft) seen_dft = true;
    if (a.dft) a.nspec = a.first_dft ? a.M / 2 + 1 : a.M;
  }
  // Green table geometry per axis
  for (int i = 0; i < 3; ++i) {
    AxisPlan& a = p->ax[i];
    if (a.dft) {
      a.F = a.M / 2 + 1;
      if (a.cls == C_UU) { a.Fs = a.F; a.off = 0; }  // offsets 0..N -> modes 0..N
      else { a.Fs = a.F; a.off = 0; a.dw = 2.0 * M_PI / a.L; a.shift = 0; }
    } else if (!a.unb) {
      const KindForm f = kind_form(a.fwd);
      a.F = a.nspec;
      a.Fs = a.F;
      a.off = 0;
      a.dw = M_PI / a.L;
      a.shift = f.qout + 0.5 * f.b2;
    } else {
      const KindForm f = kind_form(a.fwd);
      a.F = a.nspec;
      a.Fs = 2 * a.N + 1;  // kernel on [0, 2L]
      a.off = f.qout;      // spectral index s pairs with kernel mode s + qout
    }
  }
  for (int sa = 0; sa < 3; ++sa) {  // frequency-indexed spectra along the swap axes
    if (!swap[sa]) continue;
    AxisPlan& a = p->ax[sa];
    if (a.unb) a.off = 0;
    else a.shift = 0.5 * kind_form(a.fwd).b2;
  }
  const int a0 = ord[0], a1 = ord[1], a2 = ord[2];
  // tile axis of passes 1/5: the user's fastest axis x when the first transform does
  // not run along x, else the next transform axis
  if (a0 == 0 || a1 == 0) p->tb1 = a1;
  else p->tb1 = 0;  // x == a2
  if (p->tb1 == a1) { p->L1[0] = a2; p->L1[1] = a0; p->L1[2] = a1; }
  else { p->L1[0] = a1; p->L1[1] = a0; p->L1[2] = a2; }
  p->L2[0] = a0; p->L2[1] = a1; p->L2[2] = a2;
  const int Lu[3] = {2, 1, 0};
  // work extent of an untransformed axis: the node-centred periodic duplicate f_N is
  // never used, so intermediates hold N points; the last pass writes f_N := f_0
  int wext[3];
  for (int a = 0; a < 3; ++a) {
    const AxisPlan& A = p->ax[a];
    wext[a] = (A.cls == C_P && A.node) ? A.N : A.nuser;
    p->ext_user[a] = A.nuser;
    p->ext1[a] = wext[a];
    p->ext2[a] = wext[a];
  }
  p->ext1[a0] = p->ax[a0].nspec;
  p->ext2[a0] = p->ax[a0].nspec;
  p->ext2[a1] = p->ax[a1].nspec;
  int64_t su[3], s1[3], s2[3];
  layout_strides(Lu, p->ext_user, su, &p->Vu);
  layout_strides(p->L1, p->ext1, s1, &p->V1);
  layout_strides(p->L2, p->ext2, s2, &p->V2);
  p->cplx1 = p->ax[a0].dft;
  p->cplx2 = p->ax[a0].dft || p->ax[a1].dft || p->vec2;
  p->elem = (p->prec == FM_F64) ? 8 : 4;
  p->bytesA = round256(p->V1 * p->elem * (p->cplx1 ? 2 : 1));
  p->bytesB = round256(p->V2 * p->elem * (p->cplx2 ? 2 : 1));
  p->ws_bytes = (size_t)p->ncomp * (p->bytesA + p->bytesB);

  const int o1 = 3 - a0 - p->tb1;  // the other axis of passes 1 / 5
  const bool curl = p->kind != FM_POISSON;
  // pass 1: user -> L1 along a0
  {
    fm::PassDesc& d = p->pass[0];
    d = fm::PassDesc{};
    set_geometry(&d, a0, p->tb1, o1, su, p->Vu, s1, p->V1, wext);
    set_transform(&d, p->ax[a0], true, false);
    d.in_cplx = 0;
    d.in_n = p->ax[a0].nuser;
    d.out_n = p->ax[a0].nspec;
    if (p->vec) {
      for (int q = 0; q < 3; ++q) {
        p->vr2r[q][0] = make_r2r(vin[q][a0], vin[q][a0].fwd, true, true);
        p->vr2r[q][1] = make_r2r(vout[q][a0], vout[q][a0].bwd, false, true);
      }
      d.r2r = p->vr2r[0][0];
    }
  }
  // pass 2: L1 -> L2 along a1, tiles along a2
  {
    fm::PassDesc& d = p->pass[1];
    d = fm::PassDesc{};
    set_geometry(&d, a1, a2, a0, s1, p->V1, s2, p->V2, p->ext1);
    set_transform(&d, p->ax[a1], true, false);
    d.in_cplx = p->cplx1;
    d.out_cplx = p->cplx2;  // a second symmetric axis: complex values, zero imaginary part
    d.in_n = wext[a1];
    d.out_n = p->ax[a1].nspec;
    if (p->vec2 || p->vec3) {
      for (int q = 0; q < 3; ++q) {
        p->vr2r[q][2] = make_r2r(vin[q][a1], vin[q][a1].fwd, true, true);
        p->vr2r[q][3] = make_r2r(vout[q][a1], vout[q][a1].bwd, false, true);
      }
      d.r2r = p->vr2r[0][2];
    }
  }
  // pass 3: fused along a2 in L2, tiles along a1
  {
    fm::PassDesc& d = p->pass[2];
    d = fm::PassDesc{};
    set_geometry(&d, a2, a1, a0, s2, p->V2, s2, p->V2, p->ext2);
    const AxisPlan& A = p->ax[a2];
    d.fused = 1;
    if (!A.dft) {
      d.gather = fm::G_R2R;
      d.scatter = fm::S_R2R;
      d.r2r = make_r2r(A, A.fwd, true);
      d.r2r2 = make_r2r(A, A.bwd, false);
      d.spec_n = A.nspec;
      d.in_cplx = d.out_cplx = 0;
    } else if (A.first_dft) {
      d.gather = fm::G_REAL2;
      d.n_data = A.n_data;
      d.in_cplx = d.out_cplx = 0;
    } else {
      d.gather = fm::G_CPLX;
      d.n_data = A.n_data;
      d.in_cplx = d.out_cplx = 1;
    }
    d.in_n = d.out_n = wext[a2];
    fm::GreenRef& g = d.g;
    g.F_b = p->ax[a1].F;
    g.F_line = A.F;
    g.fold_c = p->ax[a0].dft ? p->ax[a0].M : 0;
    g.fold_b = p->ax[a1].dft ? p->ax[a1].M : 0;
    g.fold_line = A.dft ? A.M : 0;
    g.curl = (curl && !p->vec3) ? 1 : 0;  // three symmetric axes: not launched (curl_real_kernel)
    g.axis_line = a2;
    g.axis_b = a1;
    g.axis_c = a0;
    auto dw = [&](const AxisPlan& x) { return 2.0 * M_PI / (x.cls == C_P ? x.L : 2.0 * x.L); };
    g.dw_line = A.dft ? dw(A) : 0;
    g.dw_b = p->ax[a1].dft ? dw(p->ax[a1]) : 0;
    g.dw_c = p->ax[a0].dft ? dw(p->ax[a0]) : 0;
    g.M_line = A.M;
    g.M_b = p->ax[a1].M;
    g.M_c = p->ax[a0].M;
    g.deriv = p->kind == FM_BIOT_SAVART_FD2 ? 2 : p->kind == FM_BIOT_SAVART_FD4 ? 4
            : p->kind == FM_BIOT_SAVART_FD6 ? 6 : 0;
    if (p->vec) {
      // the derivative along the swap axis (a0, direction c) of a component tangential to
      // it: +w after a sine transform, -w after a cosine one, both flipped on a reversed
      // axis (Sec. V)
      const AxisPlan& ai = vin[(a0 + 1) % 3][a0];
      g.csym = ((ai.fwd >= RODFT00) != ai.rev) ? 1 : -1;
      if (p->vec2) {  // the same along the second symmetric axis (a1, direction b)
        const AxisPlan& bi = vin[(a1 + 1) % 3][a1];
        g.csym_b = ((bi.fwd >= RODFT00) != bi.rev) ? 1 : -1;
      }
    }
  }
  // pass 4: L2 -> L1 along a1 (inverse of pass 2)
  {
    fm::PassDesc& d = p->pass[3];
    d = fm::PassDesc{};
    set_geometry(&d, a1, a2, a0, s2, p->V2, s1, p->V1, p->ext2);
    set_transform(&d, p->ax[a1], false, false);
    d.in_cplx = p->cplx2;
    d.out_cplx = p->cplx1;
    d.in_n = p->ax[a1].nspec;
    d.out_n = wext[a1];
    if (p->vec3) d.r2r = p->vr2r[0][3];
    if (p->vec2) {
      // the real parts of the complex values of the fused pass (their imaginary parts
      // are the rounding of a real result): real elements at twice the complex strides
      d.in_cplx = 0;
      d.in_s_line *= 2;
      d.in_s_b *= 2;
      d.in_s_c *= 2;
      d.r2r = p->vr2r[0][3];
    }
  }
  // pass 5: L1 -> user along a0 (inverse of pass 1)
  {
    fm::PassDesc& d = p->pass[4];
    d = fm::PassDesc{};
    set_geometry(&d, a0, p->tb1, o1, s1, p->V1, su, p->Vu, p->ext1);
    set_transform(&d, p->ax[a0], false, false);
    d.out_cplx = 0;
    d.in_n = p->ax[a0].nspec;
    d.out_n = p->ax[a0].nuser;
    if (p->vec) d.r2r = p->vr2r[0][1];
    // output conventions along the two batch axes
    auto fix_axis = [](const AxisPlan& A, int32_t* dup, int32_t* zlo, int32_t* zhi, int32_t* last) {
      *last = A.N;
      *dup = (A.node && A.cls == C_P) ? 1 : 0;
      *zlo = (A.node && (A.cls == C_OO || A.cls == C_OE || A.cls == C_OU)) ? 1 : 0;
      *zhi = (A.node && (A.cls == C_OO || A.cls == C_EO || A.cls == C_UO)) ? 1 : 0;
    };
    fix_axis(p->ax[p->tb1], &d.fix.b_dup, &d.fix.b_zero_lo, &d.fix.b_zero_hi, &d.fix.b_last);
    fix_axis(p->ax[o1], &d.fix.c_dup, &d.fix.c_zero_lo, &d.fix.c_zero_hi, &d.fix.c_last);
    d.has_fix = d.fix.b_dup | d.fix.b_zero_lo | d.fix.b_zero_hi | d.fix.c_dup | d.fix.c_zero_lo |
                d.fix.c_zero_hi;
    if (p->vec) {
      // each component's own faces (its velocity faces on a second symmetric axis, which
      // is a batch axis of this pass): packed real lines leave rounding on a zero line, so
      // the odd-face nodes are zeroed here
      for (int q = 0; q < 3; ++q) {
        fm::Fixup& fx = p->vfix[q];
        fix_axis(vout[q][p->tb1], &fx.b_dup, &fx.b_zero_lo, &fx.b_zero_hi, &fx.b_last);
        fix_axis(vout[q][o1], &fx.c_dup, &fx.c_zero_lo, &fx.c_zero_hi, &fx.c_last);
        p->vhas_fix[q] = fx.b_dup | fx.b_zero_lo | fx.b_zero_hi | fx.c_dup | fx.c_zero_lo | fx.c_zero_hi;
      }
      d.fix = p->vfix[0];
      d.has_fix = p->vhas_fix[0];
    }
  }
  // component strides of the work buffers (elements), fixed by the plan
  {
    const int64_t compA = (int64_t)(p->bytesA / (p->elem * (p->cplx1 ? 2 : 1)));
    const int64_t compB = (int64_t)(p->bytesB / (p->elem * (p->cplx2 ? 2 : 1)));
    p->pass[0].out_s_comp = compA;
    p->pass[1].in_s_comp = compA;
    p->pass[1].out_s_comp = compB;
    p->pass[2].in_s_comp = compB;
    p->pass[2].out_s_comp = compB;
    p->pass[3].in_s_comp = p->vec2 ? 2 * compB : compB;
    p->pass[3].out_s_comp = compA;
    p->pass[4].in_s_comp = compA;
  }
  // plain transforms along the last axis: B (L2, a2 extent wext) <-> spectrum buffer
  // (L2 order, a2 extent nspec), one per component
  {
    const AxisPlan& A = p->ax[a2];
    for (int a = 0; a < 3; ++a) p->ext_spec[a] = p->ext2[a];
    p->ext_spec[a2] = A.nspec;
    int64_t ss[3];
    layout_strides(p->L2, p->ext_spec, ss, &p->Vspec);
    p->cplx_spec = p->cplx2 || A.dft;
    fm::PassDesc& f = p->pass[5];
    f = fm::PassDesc{};
    set_geometry(&f, a2, a1, a0, s2, p->V2, ss, p->Vspec, p->ext2);
    set_transform(&f, A, true, false);
    f.in_cplx = p->cplx2;
    f.out_cplx = p->cplx_spec;
    f.in_n = wext[a2];
    f.out_n = A.nspec;
    fm::PassDesc& g = p->pass[6];
    g = fm::PassDesc{};
    set_geometry(&g, a2, a1, a0, ss, p->Vspec, s2, p->V2, p->ext2);
    set_transform(&g, A, false, false);
    g.in_cplx = p->cplx_spec;
    g.out_cplx = p->cplx2;
    g.in_n = A.nspec;
    g.out_n = wext[a2];
    const int64_t compB = (int64_t)(p->bytesB / (p->elem * (p->cplx2 ? 2 : 1)));
    f.in_s_comp = compB;
    f.out_s_comp = p->Vspec;
    g.in_s_comp = p->Vspec;
    g.out_s_comp = compB;
    if (p->vec3) {
      for (int q = 0; q < 3; ++q) {
        p->vr2r[q][4] = make_r2r(vin[q][a2], vin[q][a2].fwd, true, true);
        p->vr2r[q][5] = make_r2r(vout[q][a2], vout[q][a2].bwd, false, true);
      }
      f.r2r = p->vr2r[0][4];
      g.r2r = p->vr2r[0][5];
      // the spectra after B; the real curl's geometry (tables are set with the Green's
      // spectrum)
      p->ws_bytes += round256((size_t)3 * p->Vspec * p->elem);
      fm::CurlReal& c = p->vcurl;
      c.comp_stride = p->Vspec;
      const int ta[3] = {a0, a1, a2};
      for (int t = 0; t < 3; ++t) {
        c.n[t] = p->ext_spec[ta[t]];
        c.ax[t] = ta[t];
      }
      for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 3; ++q) {
          const AxisPlan& ai = vin[q][a];
          c.sg[a][q] = ((ai.fwd >= RODFT00) != ai.rev) ? 1 : -1;
        }
    }
  }
  const int line_axis[fm_plan_s::kPasses] = {a0, a1, a2, a1, a0, a2, a2};
  for (int i = 0; i < fm_plan_s::kPasses; ++i) {
    fm::PassDesc& d = p->pass[i];
    const int rc = radix_plan(p->ax[line_axis[i]].M, &d);
    if (rc) return rc;
    const bool fused_curl = (i == 2) && curl && !p->vec3;
    d.ncomp = vec_pass(p, i) ? 1 : p->ncomp;  // launched per component
    d.long_rt = 0;
    d.persist = 1;
    d.lds_tabs = 1;
    int rc2 = choose_tile(&d, p->elem, fused_curl ? 3 : 1, (i == 2) && d.gather == fm::G_R2R, d.nb);
    if (rc2 && p->prec == FM_F64) {
      // no tile fits 8 FP64 values per thread: the runtime-length class with 16
      d.long_rt = 1;
      p->long_rt[i] = true;
      rc2 = choose_tile(&d, p->elem, fused_curl ? 3 : 1, (i == 2) && d.gather == fm::G_R2R, d.nb);
    }
    if (rc2) return rc2;
    d.tiles = ((d.nb + d.B - 1) / d.B) * d.nc * (fused_curl ? 1 : d.ncomp);
    set_magics(&d);
    if (i == 2 && wave_capable(d, p->elem) && !(fused_curl && p->elem == 8)) {
      // the per-wavefront kernel, with the most wavefronts per workgroup whose LDS stays
      // within the preferred size
      const int E = default_wave_values(d, p->elem);
      for (const int W : {4, 2, 1}) {
        fm::PassDesc w = d;
        if (set_wave(&w, p->elem, W, fused_curl ? 1 : d.ncomp, E) && w.lds_bytes <= fm::kSoftLds) {
          d = w;
          break;
        }
      }
    }
  }
  for (int i = 0; i < fm_plan_s::kPasses; ++i) p->pass[i].kind = pass_kind(p->pass[i]);
  const int64_t sizes_in[fm_plan_s::kPasses] = {p->Vu, p->V1, p->V2, p->vec2 ? 2 * p->V2 : p->V2, p->V1,
                                                p->V2, p->Vspec};
  const int64_t sizes_out[fm_plan_s::kPasses] = {p->V1, p->V2, p->V2, p->V1, p->Vu, p->Vspec, p->V2};
  for (int i = 0; i < fm_plan_s::kPasses; ++i)
    if (!pass_in_bounds(p->pass[i], sizes_in[i], sizes_out[i], p->elem)) return FM_E_SIZE;
  return FM_OK;
}


// Buffers of one solve: pass i reads ins[i] and writes outs[i].  Work buffer A holds
// the first-axis spectrum (layout L1), B the two-axis spectrum (layout L2).
void bind_buffers(const fm_plan_s* p, const void* rhs, void* out, char* ws, const void* ins[5],
                  void* outs[5]) {
  char* A = ws;
  char* B = ws + p->ncomp * p->bytesA;
  ins[0] = rhs; outs[0] = A;
  ins[1] = A; outs[1] = B;
  ins[2] = B; outs[2] = B;
  ins[3] = B; outs[3] = A;
  ins[4] = A; outs[4] = out;
}

// FLUXMI_SYNC_DEBUG=1: trace every pass launch on stderr and synchronise after it, so
// that a failing or stalled launch is named.
bool sync_debug() {
  static const bool v = [] {
    const char* e = std::getenv("FLUXMI_SYNC_DEBUG");
    return e != nullptr && std::atoi(e) != 0;
  }();
  return v;
}

// Launch descriptor i of the plan on buffers in -> out.
int launch_one(fm_plan_s* p, int i, const void* in, void* out, hipStream_t st) {
  const fm::PassDesc& d = p->pass[i];
  if (sync_debug()) {
    std::fprintf(stderr, "fluxmi: pass %d kind %d M %d prec %s tiles %d B %d lds %d\n", i + 1, d.kind,
                 d.M, p->prec == FM_F64 ? "f64" : "f32", d.tiles, d.B, d.lds_bytes);
    std::fflush(stderr);
  }
  if (d.wave && !(d.wave == 16 ? d.wtw : (d.wave == 8 ? d.wtw8 : d.wtw32))) return FM_E_ARG;
  if (d.fused && d.g.curl && !(d.g.dtab_line && d.g.dtab_b && d.g.dtab_c)) return FM_E_ARG;
  auto run = [&](const fm::PassDesc& dq, const fm::PassDesc* dev, const void* iq, void* oq) {
    return (p->prec == FM_F64) ? fm::launch_pass<double>(dq, dev, iq, oq, st)
                               : fm::launch_pass<float>(dq, dev, iq, oq, st);
  };
  hipError_t e = run(d, p->dpass + i, in, out);
  if (vec_pass(p, i)) {
    // the other two components, each with its own transform along the swap axis
    const size_t es_in = p->elem * (d.in_cplx ? 2 : 1), es_out = p->elem * (d.out_cplx ? 2 : 1);
    for (int q = 1; q < 3 && e == hipSuccess; ++q) {
      const int slot = vec_slot(i, q);
      e = run(p->vdesc[slot], p->dpass + fm_plan_s::kPasses + slot,
              static_cast<const char*>(in) + (size_t)q * d.in_s_comp * es_in,
              static_cast<char*>(out) + (size_t)q * d.out_s_comp * es_out);
    }
  }
  if (e == hipSuccess && sync_debug()) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return FM_E_HIP;
  }
  return FM_OK;
}

// Pass 3 of a plan with three symmetric axes: the last axis's forward transform into the
// spectra region after B, the real curl times the Green's spectrum there, the backward
// transform into B (each transform once per component).
int launch_curl3(fm_plan_s* p, void* B, hipStream_t st) {
  char* S = static_cast<char*>(B) + (size_t)p->ncomp * p->bytesB;
  int rc = launch_one(p, 5, B, S, st);
  if (rc) return rc;
  fm::CurlReal c = p->vcurl;
  c.S = S;
  const hipError_t e = (p->prec == FM_F64) ? fm::launch_curl_real<double>(c, st)
                                           : fm::launch_curl_real<float>(c, st);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return FM_E_HIP;
  }
  return launch_one(p, 6, S, B, st);
}

int launch_all(fm_plan_s* p, const void* const ins[5], void* const outs[5], hipStream_t st,
               int first = 0, int last = 4) {
  for (int i = first; i <= last; ++i) {
    const int rc = (i == 2 && p->vec3) ? launch_curl3(p, outs[2], st) : launch_one(p, i, ins[i], outs[i], st);
    if (rc) return rc;
  }
  return FM_OK;
}

// Pinned host staging for the batch descriptor tables, one per host thread.  It is
// deliberately never released: freeing it from a thread-exit destructor could run
// after the HIP runtime has been torn down.
struct BatchStaging {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
thread_local BatchStaging* g_stage_ptr = nullptr;

}  // namespace

// A prepared batch: FP64 batches hold one launch per pass and length class (descriptor
// tables in the workspace); FP32 batches hold the per-request buffers of plan-by-plan
// launches.
// Streams a prepared FP32 batch spreads its solves over.
constexpr int kBatchLanes = 8;

struct fm_batch_s {
  int prec = 0;
  std::vector<fm_plan_s*> plans;
  std::vector<const void*> ins;  // 5 per request
  std::vector<void*> outs;
  struct Group {
    int pass, len_class, first, count, tiles, lds;
    size_t off_desc, off_pref;
    int single;  // >= 0: one per-wavefront pass, launched alone (host copy singles[single])
  };
  std::vector<Group> groups;
  std::vector<fm::PassDesc> singles;
  char* dev_tables = nullptr;
  // prepared FP32 batches: the plans are spread over these streams (default priority),
  // forked from and joined back into the caller's stream with events
  std::vector<hipStream_t> lanes;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  ~fm_batch_s() {
    for (hipEvent_t e : joins)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (hipStream_t s : lanes)
      if (s) (void)hipStreamDestroy(s);
  }
};

namespace {

// Work buffers of every request and, for FP64, the grouped descriptor tables (returned
// in *host, to be copied to b->dev_tables before the first run).
int build_batch(int count, const fm_plan* plans, const void* const* rhs_dev, void* const* out_dev,
                void* workspace_dev, size_t workspace_bytes, fm_batch_s* b, std::vector<char>* host) {
  if (count < 0) return FM_E_ARG;
  if (!plans || !rhs_dev || !out_dev || !workspace_dev) return FM_E_NULL;
  size_t need = 0;
  int rc = fm_batched_workspace_bytes(count, plans, &need);
  if (rc) return rc;
  if (workspace_bytes < need) return FM_E_ARG;
  const int prec = plans[0]->prec;
  for (int i = 0; i < count; ++i) {
    if (plans[i]->prec != prec) return FM_E_ARG;
    if (plans[i]->vec) return FM_E_KIND;  // vector plans solve one by one
    if (!rhs_dev[i] || !out_dev[i]) return FM_E_NULL;
  }
  b->prec = prec;
  b->plans.assign(plans, plans + count);
  b->ins.resize(5 * (size_t)count);
  b->outs.resize(5 * (size_t)count);
  char* ws = reinterpret_cast<char*>(workspace_dev);
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    bind_buffers(plans[i], rhs_dev[i], out_dev[i], ws + off, &b->ins[5 * (size_t)i], &b->outs[5 * (size_t)i]);
    off += round256(plans[i]->ws_bytes);
  }
  host->clear();
  if (prec == FM_F32 && !kFp32OneLaunch) return FM_OK;  // plan by plan, no tables
  std::vector<fm::PassDesc> all(5 * (size_t)count);
  for (int i = 0; i < count; ++i)
    for (int ps = 0; ps < 5; ++ps) {
      fm::PassDesc& d = all[5 * (size_t)i + ps];
      d = plans[i]->pass[ps];
      d.in = b->ins[5 * (size_t)i + ps];
      d.out = b->outs[5 * (size_t)i + ps];
    }
  // group each pass's descriptors by length class: one launch per class and pass
  std::vector<int> order;
  size_t table_bytes = 0;
  for (int ps = 0; ps < 5; ++ps) {
    std::map<int, std::vector<int>> by_class;
    for (int i = 0; i < count; ++i) {
      const fm::PassDesc& d = all[5 * (size_t)i + ps];
      // passes in the per-wavefront kernel keep it (the batch equals the single solves
      // bitwise) and are launched one by one; their class key is unique and negative
      if (d.wave) {
        by_class[-1 - i].push_back(i);
        continue;
      }
      const int rt = (d.M > fm::kMaxFastLen64 || d.long_rt) ? fm::kRtLong : fm::kRtShort;
      by_class[d.stw ? d.M : rt].push_back(i);
    }
    for (auto& kv : by_class) {
      fm_batch_s::Group g{};
      g.pass = ps;
      g.len_class = kv.first;
      g.single = -1;
      if (kv.first < 0) {
        g.single = (int)b->singles.size();
        b->singles.push_back(all[5 * (size_t)kv.second[0] + ps]);
      }
      g.first = (int)order.size();
      g.count = (int)kv.second.size();
      for (int i : kv.second) order.push_back(i);
      g.off_desc = table_bytes;
      table_bytes += round256((size_t)g.count * sizeof(fm::PassDesc));
      g.off_pref = table_bytes;
      table_bytes += round256((size_t)(g.count + 1) * sizeof(int));
      b->groups.push_back(g);
    }
  }
  if (off + table_bytes > workspace_bytes) return FM_E_ARG;
  host->assign(table_bytes, 0);
  for (fm_batch_s::Group& g : b->groups) {
    fm::PassDesc* hd = reinterpret_cast<fm::PassDesc*>(host->data() + g.off_desc);
    int* hp = reinterpret_cast<int*>(host->data() + g.off_pref);
    int acc = 0, mx = 0;
    for (int j = 0; j < g.count; ++j) {
      const int i = order[g.first + j];
      hd[j] = all[5 * (size_t)i + g.pass];
      hp[j] = acc;
      acc += hd[j].tiles;
      mx = std::max(mx, hd[j].lds_bytes);
    }
    hp[g.count] = acc;
    g.tiles = acc;
    g.lds = mx;
  }
  b->dev_tables = ws + off;
  return FM_OK;
}

int run_batch(const fm_batch_s& b, hipStream_t st) {
  if (b.prec == FM_F32 && !kFp32OneLaunch) {
    const size_t K = b.lanes.size();
    if (K == 0) {
      for (size_t i = 0; i < b.plans.size(); ++i) {
        const int rc = launch_all(b.plans[i], &b.ins[5 * i], &b.outs[5 * i], st);
        if (rc) return rc;
      }
      return FM_OK;
    }
    // independent solves side by side: plan i on lane i mod K, after everything enqueued
    // on st so far; st then waits for every lane (a fork and join that a graph capture
    // of st records as parallel branches)
    FM_HIP(hipEventRecord(b.fork, st));
    for (size_t k = 0; k < K; ++k) FM_HIP(hipStreamWaitEvent(b.lanes[k], b.fork, 0));
    for (size_t i = 0; i < b.plans.size(); ++i) {
      const int rc = launch_all(b.plans[i], &b.ins[5 * i], &b.outs[5 * i], b.lanes[i % K]);
      if (rc) return rc;
    }
    for (size_t k = 0; k < K; ++k) {
      FM_HIP(hipEventRecord(b.joins[k], b.lanes[k]));
      FM_HIP(hipStreamWaitEvent(st, b.joins[k], 0));
    }
    return FM_OK;
  }
  for (const fm_batch_s::Group& g : b.groups) {
    const fm::PassDesc* dd = reinterpret_cast<const fm::PassDesc*>(b.dev_tables + g.off_desc);
    const int* dp = reinterpret_cast<const int*>(b.dev_tables + g.off_pref);
    hipError_t e;
    if (g.single >= 0) {
      const fm::PassDesc& h = b.singles[g.single];
      e = b.prec == FM_F32 ? fm::launch_pass<float>(h, dd, h.in, h.out, st)
                           : fm::launch_pass<double>(h, dd, h.in, h.out, st);
    } else {
      e = b.prec == FM_F32 ? fm::launch_pass_batched<float>(g.len_class, dd, dp, g.count, g.tiles, g.lds, st)
                           : fm::launch_pass_batched<double>(g.len_class, dd, dp, g.count, g.tiles, g.lds, st);
    }
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      return FM_E_HIP;
    }
  }
  return FM_OK;
}

}  // namespace

namespace fm {
void set_last_hip_error(int e) { g_last_hip = e; }
}  // namespace fm

namespace {

int check_enums(int layout, int green, int prec, int kind, int ncomp) {
  if (layout != FM_CELL && layout != FM_NODE) return FM_E_KIND;
  if (green < FM_GREEN_CHAT2 || green > FM_GREEN_LGF2) return FM_E_KIND;
  if (prec != FM_F64 && prec != FM_F32) return FM_E_KIND;
  if (kind < FM_POISSON || kind > FM_BIOT_SAVART_FD6) return FM_E_KIND;
  if (ncomp < 1 || ncomp > 64) return FM_E_KIND;
  return FM_OK;
}

fm_plan_s* new_plan(const int n[3], const double h[3], const int bc[3][2], int layout, int green,
                    int prec, int kind, int ncomp) {
  fm_plan_s* p = new (std::nothrow) fm_plan_s();
  if (!p) return nullptr;
  for (int a = 0; a < 3; ++a) {
    p->n[a] = n[a];
    p->h[a] = h[a];
    p->bc[a][0] = bc[a][0];
    p->bc[a][1] = bc[a][1];
  }
  p->layout = layout;
  p->green = green;
  p->prec = prec;
  p->kind = kind;
  p->ncomp = ncomp;
  return p;
}

int create_plan(fm_plan* out, const int n[3], const double h[3], const int bc[3][2], int layout,
                int green, int prec, int kind, int ncomp, hipStream_t st, bool deferred) {
  if (!out || !n || !h || !bc) return FM_E_NULL;
  *out = nullptr;
  int rc = check_enums(layout, green, prec, kind, ncomp);
  if (rc) return rc;
  fm_plan_s* p = new_plan(n, h, bc, layout, green, prec, kind, ncomp);
  if (!p) return FM_E_NOMEM;
  rc = build_plan(p);
  if (rc == FM_OK) {
    const hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      rc = FM_E_HIP;
    }
  }
  if (rc == FM_OK)
    rc = (prec == FM_F64) ? make_tables_and_green<double>(p, st, deferred)
                          : make_tables_and_green<float>(p, st, deferred);
  if (rc != FM_OK) {
    free_plan(p);
    return rc;
  }
  *out = p;
  return FM_OK;
}

// fm_plan_create_vector: the faces of a mirror-symmetric vector field (periodic and
// unbounded faces shared; on a symmetric face of axis a, the component along a with one
// symmetry and the two others with the opposite one).
int check_vector_faces(const int bc[3][3][2]) {
  for (int a = 0; a < 3; ++a)
    for (int f = 0; f < 2; ++f) {
      const int t[3] = {bc[0][a][f], bc[1][a][f], bc[2][a][f]};
      for (int q = 0; q < 3; ++q)
        if (t[q] < FM_BC_EVEN || t[q] > FM_BC_UNB) return FM_E_BC;
      const bool sym = t[0] <= FM_BC_ODD || t[1] <= FM_BC_ODD || t[2] <= FM_BC_ODD;
      if (!sym) {
        if (t[0] != t[1] || t[0] != t[2]) return FM_E_BC;
        continue;
      }
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      if (t[a] > FM_BC_ODD || t[b] > FM_BC_ODD || t[c] > FM_BC_ODD) return FM_E_BC;
      if (t[b] != t[c] || t[a] == t[b]) return FM_E_BC;
    }
  return FM_OK;
}

int create_vector_plan(fm_plan* out, const int n[3], const double h[3], const int bc[3][3][2],
                       int layout, int green, int prec, int kind, hipStream_t st) {
  if (!out || !n || !h || !bc) return FM_E_NULL;
  *out = nullptr;
  int rc = check_enums(layout, green, prec, kind, 3);
  if (rc) return rc;
  if (kind == FM_POISSON) return FM_E_KIND;
  rc = check_vector_faces(bc);
  if (rc) return rc;
  fm_plan_s* p = new_plan(n, h, bc[0], layout, green, prec, kind, 3);
  if (!p) return FM_E_NOMEM;
  // without a symmetric face the components share their faces: the plain Biot-Savart plan
  for (int a = 0; a < 3; ++a)
    for (int f = 0; f < 2; ++f) p->vec = p->vec || bc[0][a][f] <= FM_BC_ODD;
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a)
      for (int f = 0; f < 2; ++f) p->bcv[q][a][f] = bc[q][a][f];
  rc = build_plan(p);
  if (rc == FM_OK) {
    const hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      rc = FM_E_HIP;
    }
  }
  if (rc == FM_OK)
    rc = (prec == FM_F64) ? make_tables_and_green<double>(p, st, false)
                          : make_tables_and_green<float>(p, st, false);
  if (rc != FM_OK) {
    free_plan(p);
    return rc;
  }
  *out = p;
  return FM_OK;
}

}  // namespace

namespace fm {
int plan_create_deferred(fm_plan* out, const int n[3], const double h[3], const int bc[3][2],
                         int layout, int green, int prec, int kind, int ncomp, hipStream_t st,
                         hipEvent_t* ready) {
  if (!ready) return FM_E_NULL;
  const int rc = create_plan(out, n, h, bc, layout, green, prec, kind, ncomp, st, true);
  *ready = rc == FM_OK ? (*out)->ready : nullptr;
  return rc;
}

void plan_generation_done(fm_plan p) {
  if (!p || !p->ready) return;
  release_generation(p);
  (void)hipEventDestroy(p->ready);
  p->ready = nullptr;
}
}  // namespace fm

extern "C" {

const char* fm_error_string(int status) {
  switch (status) {
    case FM_OK: return "ok";
    case FM_E_NULL: return "null pointer argument";
    case FM_E_BC: return "invalid boundary condition (periodic must pair with periodic)";
    case FM_E_SIZE: return "unsupported size (N < 2, h <= 0, or FFT length not 2^a 3^b 5^c 7^d <= 4096)";
    case FM_E_KIND: return "unsupported kind / green / precision / layout combination";
    case FM_E_NOMEM: return "device allocation failed";
    case FM_E_HIP: return "HIP runtime error";
    case FM_E_ARG: return "inconsistent arguments";
    case FM_E_SCRATCH: return "workspace exceeds the static scratch of fm_solve_static (FM_STATIC_WORKSPACE_BYTES)";
    default: return "unknown status";
  }
}

int fm_last_hip_error(void) { return g_last_hip; }

int fm_plan_create(fm_plan* out, const int n[3], const double h[3], const int bc[3][2], int layout,
                   int green, int prec, int kind, int ncomp, void* hip_stream) {
  return create_plan(out, n, h, bc, layout, green, prec, kind, ncomp,
                     reinterpret_cast<hipStream_t>(hip_stream), false);
}

int fm_plan_create_vector(fm_plan* out, const int n[3], const double h[3], const int bc[3][3][2],
                          int layout, int green, int prec, int kind, void* hip_stream) {
  return create_vector_plan(out, n, h, bc, layout, green, prec, kind,
                            reinterpret_cast<hipStream_t>(hip_stream));
}

int fm_plan_inspect(const int n[3], const double h[3], const int bc[3][2], int layout, int green,
                    int prec, int kind, int ncomp, fm_plan_info* info) {
  if (!n || !h || !bc || !info) return FM_E_NULL;
  const int rc0 = check_enums(layout, green, prec, kind, ncomp);
  if (rc0) return rc0;
  fm_plan_s* p = new_plan(n, h, bc, layout, green, prec, kind, ncomp);
  if (!p) return FM_E_NOMEM;
  const int rc = build_plan(p);
  if (rc == FM_OK) {
    for (int a = 0; a < 3; ++a) {
      info->order[a] = p->order[a];
      info->axis_class[a] = p->ax[a].cls;
      info->fft_len[a] = p->ax[a].M;
      info->spec_len[a] = p->ax[a].nspec;
      info->green_dims[a] = p->ax[p->order[a]].F;
    }
    info->workspace_bytes = p->ws_bytes;
    for (int i = 0; i < 5; ++i) {
      info->tiles[i] = p->pass[i].tiles;
      info->lines_per_tile[i] = p->pass[i].B;
      info->lds_bytes[i] = p->pass[i].lds_bytes;
    }
    // algorithmic bytes: every live element read once and written once per pass
    const double e = (double)p->elem, nc = p->ncomp;
    const double wu = (double)p->Vu, w1 = (double)p->V1 * (p->cplx1 ? 2 : 1);
    const double w2 = (double)p->V2 * (p->cplx2 ? 2 : 1);
    const double wg = (double)p->ax[p->order[0]].F * p->ax[p->order[1]].F * p->ax[p->order[2]].F;
    info->algo_bytes[0] = e * nc * (wu + w1);
    info->algo_bytes[1] = e * nc * (w1 + w2);
    info->algo_bytes[2] = e * (nc * 2 * w2 + wg);
    info->algo_bytes[3] = e * nc * (w2 + w1);
    info->algo_bytes[4] = e * nc * (w1 + wu);
  }
  delete p;
  return rc;
}

int fm_plan_destroy(fm_plan p) {
  free_plan(p);
  return FM_OK;
}

int fm_plan_workspace_bytes(fm_plan p, size_t* bytes) {
  if (!p || !bytes) return FM_E_NULL;
  *bytes = p->ws_bytes;
  return FM_OK;
}

int fm_plan_shape(fm_plan p, int user_dims[3]) {
  if (!p || !user_dims) return FM_E_NULL;
  for (int a = 0; a < 3; ++a) user_dims[a] = p->ax[a].nuser;
  return FM_OK;
}

int fm_solve(fm_plan p, const void* rhs_dev, void* out_dev, void* workspace_dev, void* hip_stream) {
  if (!p || !rhs_dev || !out_dev) return FM_E_NULL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(workspace_dev);
  if (!ws && !(ws = own_workspace(p))) return FM_E_NOMEM;
  const void* ins[5];
  void* outs[5];
  bind_buffers(p, rhs_dev, out_dev, ws, ins, outs);
  return launch_all(p, ins, outs, st);
}

int fm_solve_passes(fm_plan p, const void* rhs_dev, void* out_dev, void* workspace_dev, int first_pass,
                    int last_pass, void* hip_stream) {
  if (!p || !rhs_dev || !out_dev) return FM_E_NULL;
  if (first_pass < 0 || last_pass > 4 || first_pass > last_pass) return FM_E_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(workspace_dev);
  if (!ws && !(ws = own_workspace(p))) return FM_E_NOMEM;
  const void* ins[5];
  void* outs[5];
  bind_buffers(p, rhs_dev, out_dev, ws, ins, outs);
  return launch_all(p, ins, outs, st, first_pass, last_pass);
}

int fm_plan_spectrum_layout(fm_plan p, int dims[3], int axes[3], int* is_complex, size_t* bytes) {
  if (!p || !dims || !axes || !is_complex || !bytes) return FM_E_NULL;
  for (int i = 0; i < 3; ++i) {
    axes[i] = p->L2[i];
    dims[i] = p->ext_spec[p->L2[i]];
  }
  *is_complex = p->cplx_spec ? 1 : 0;
  *bytes = (size_t)p->ncomp * (size_t)p->Vspec * p->elem * (p->cplx_spec ? 2 : 1);
  return FM_OK;
}

int fm_fft_forward(fm_plan p, const void* in_dev, void* spec_dev, void* workspace_dev, void* hip_stream) {
  if (!p || !in_dev || !spec_dev) return FM_E_NULL;
  if (p->vec) return FM_E_KIND;  // the spectrum of a vector plan is not exposed
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(workspace_dev);
  if (!ws && !(ws = own_workspace(p))) return FM_E_NOMEM;
  char* A = ws;
  char* B = ws + p->ncomp * p->bytesA;
  int rc = launch_one(p, 0, in_dev, A, st);
  if (rc == FM_OK) rc = launch_one(p, 1, A, B, st);
  if (rc == FM_OK) rc = launch_one(p, 5, B, spec_dev, st);
  return rc;
}

int fm_fft_backward(fm_plan p, const void* spec_dev, void* out_dev, void* workspace_dev, void* hip_stream) {
  if (!p || !spec_dev || !out_dev) return FM_E_NULL;
  if (p->vec) return FM_E_KIND;  // the spectrum of a vector plan is not exposed
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(workspace_dev);
  if (!ws && !(ws = own_workspace(p))) return FM_E_NOMEM;
  char* A = ws;
  char* B = ws + p->ncomp * p->bytesA;
  int rc = launch_one(p, 6, spec_dev, B, st);
  if (rc == FM_OK) rc = launch_one(p, 3, B, A, st);
  if (rc == FM_OK) rc = launch_one(p, 4, A, out_dev, st);
  return rc;
}

int fm_batched_workspace_bytes(int count, const fm_plan* plans, size_t* bytes) {
  if (!plans || !bytes) return FM_E_NULL;
  if (count < 0) return FM_E_ARG;
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return FM_E_NULL;
    total += round256(plans[i]->ws_bytes);
  }
  // descriptor tables: 5 passes x (count descriptors + prefixes), at most 5 * count
  // length groups each rounded up to 256 bytes twice
  total += 5 * ((size_t)count * (sizeof(fm::PassDesc) + sizeof(int) + 512) + 512);
  *bytes = total;
  return FM_OK;
}

int fm_solve_batched(int count, const fm_plan* plans, const void* const* rhs_dev, void* const* out_dev,
                     void* workspace_dev, size_t workspace_bytes, void* hip_stream) {
  if (count == 0) return FM_OK;
  fm_batch_s b;
  std::vector<char> host;
  int rc = build_batch(count, plans, rhs_dev, out_dev, workspace_dev, workspace_bytes, &b, &host);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if (!host.empty()) {
    // the tables go through pinned host memory, reused once the previous copy finished
    if (!g_stage_ptr) g_stage_ptr = new (std::nothrow) BatchStaging();
    if (!g_stage_ptr) return FM_E_NOMEM;
    BatchStaging& sg = *g_stage_ptr;
    if (sg.pending) {
      FM_HIP(hipEventSynchronize(sg.done));
      sg.pending = false;
    }
    if (sg.bytes < host.size()) {
      if (sg.host) (void)hipHostFree(sg.host);
      sg.host = nullptr;
      sg.bytes = 0;
      if (hipHostMalloc(&sg.host, host.size(), hipHostMallocDefault) != hipSuccess) return FM_E_NOMEM;
      sg.bytes = host.size();
    }
    if (!sg.done) FM_HIP(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming));
    std::memcpy(sg.host, host.data(), host.size());
    FM_HIP(hipMemcpyAsync(b.dev_tables, sg.host, host.size(), hipMemcpyHostToDevice, st));
    FM_HIP(hipEventRecord(sg.done, st));
    sg.pending = true;
  }
  return run_batch(b, st);
}

// Launch mode of a descriptor, as fm_plan_tiling reports it: 1 persistent with LDS
// tables, 0 one tile per workgroup with LDS tables, 2 one tile per workgroup with global
// tables (the only mode of the runtime-length and long FP64 kernels).
int launch_mode(const fm::PassDesc& d, size_t elem) {
  if (d.wave) return d.wave == 16 ? 3 : (d.wave == 8 ? 4 : 5);
  const bool pipelined = compile_time_kernel(d, elem) && fm::pipelined_kernel((int)elem, d.M);
  if (!pipelined || !d.lds_tabs) return 2;
  return d.persist ? 1 : 0;
}

// A pass re-tiled with at most bmax lines per tile, in launch mode `mode` (1 persistent
// with LDS tables, 0 one tile per workgroup with LDS tables, 2 one tile per workgroup
// with global tables, 3 / 4 / 5 the per-wavefront kernels with 16 / 8 / 32 values per
// lane);
// false if no such tiling is valid for this plan (the compile-time-length kernels
// address a tile with 32-bit offsets).
bool retile(const fm_plan_s* p, int i, int bmax, int mode, fm::PassDesc* out) {
  fm::PassDesc d = p->pass[i];
  const bool fused_curl = (i == 2) && p->kind != FM_POISSON;
  const int64_t sizes_in[5] = {p->Vu, p->V1, p->V2, p->vec2 ? 2 * p->V2 : p->V2, p->V1};
  const int64_t sizes_out[5] = {p->V1, p->V2, p->V2, p->V1, p->Vu};
  d.wave = 0;
  // the per-wavefront kernel has the compile-time length; the LDS-tile kernel takes the
  // class the plan chose
  const bool wave_mode = mode >= 3;
  d.long_rt = wave_mode ? 0 : p->long_rt[i];
  d.stw = p->stw_plan[i];
  if (wave_mode) {
    // the per-wavefront kernel (16 or 8 values per lane): the most wavefronts per
    // workgroup within bmax lines; launched in the compile-time class, which the stage
    // table selects
    const int E = mode == 3 ? 16 : (mode == 4 ? 8 : 32);
    if (!wave_capable(d, p->elem, E)) return false;
    if (!d.stw) {
      const auto t = p->stw.find(d.M);
      if (t == p->stw.end()) return false;
      d.stw = t->second;
    }
    for (const int W : {4, 2, 1}) {
      fm::PassDesc w = d;
      const int lines = W * fm::wave_lines(d.M, E) * (d.fused ? 1 : wave_plain_pk(d));
      if (lines > bmax || !set_wave(&w, p->elem, W, fused_curl ? 1 : d.ncomp, E)) continue;
      if (!pass_in_bounds(w, sizes_in[i], sizes_out[i], p->elem)) return false;
      *out = w;
      return true;
    }
    return false;
  }
  d.persist = mode == 1;
  d.lds_tabs = mode != 2;
  if (choose_tile(&d, p->elem, fused_curl ? 3 : 1, (i == 2) && d.gather == fm::G_R2R, d.nb, bmax))
    return false;
  d.tiles = ((d.nb + d.B - 1) / d.B) * d.nc * (fused_curl ? 1 : d.ncomp);
  set_magics(&d);
  if (d.stw && tile_in_span_bytes(d, p->elem) >= (int64_t(1) << 32)) return false;
  if (!pass_in_bounds(d, sizes_in[i], sizes_out[i], p->elem)) return false;
  *out = d;
  return true;
}

extern "C++" {
namespace {

// A tiling as fm_plan_tiling reports it, validated pass by pass and applied.
int apply_tiling(fm_plan p, const int lines_per_tile[5], const int persist[5], hipStream_t st) {
  fm::PassDesc next[5];
  for (int i = 0; i < 5; ++i) {
    const int mode = persist[i];
    if (lines_per_tile[i] < 1 || mode < 0 || mode > 5) return FM_E_ARG;
    if (!retile(p, i, lines_per_tile[i], mode, &next[i])) return FM_E_ARG;
    // exactly the requested tiling (retile takes the largest tile up to the bound)
    if (next[i].B != lines_per_tile[i] || launch_mode(next[i], p->elem) != mode) return FM_E_ARG;
  }
  for (int i = 0; i < 5; ++i) p->pass[i] = next[i];
  FM_HIP(hipMemcpyAsync(p->dpass, p->pass, sizeof(fm::PassDesc) * 5, hipMemcpyHostToDevice, st));
  FM_HIP(hipStreamSynchronize(st));
  if (p->vec) FM_HIP(upload_vec_descs(p, st));
  return FM_OK;
}

// Tuning cache (FLUXMI_TUNE_CACHE): one line per tuned problem,
//   <device>/<CUs> p<prec> k<kind> c<ncomp> l<layout> g<green> n<nx,ny,nz> b<6 faces> B<5> M<5>
// read before tuning (a valid entry is applied instead of timing) and appended after.
std::mutex g_tune_cache_mu;

std::string tune_key(const fm_plan_s* p) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    cus = prop.multiProcessorCount;
  }
  for (char& ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/%d p%d k%d c%d l%d g%d n%d,%d,%d b%d,%d,%d,%d,%d,%d", arch.c_str(), cus,
                p->prec, p->kind, p->ncomp, p->layout, p->green, p->n[0], p->n[1], p->n[2], p->bc[0][0],
                p->bc[0][1], p->bc[1][0], p->bc[1][1], p->bc[2][0], p->bc[2][1]);
  std::string key = buf;
  if (p->vec) {  // the faces of components 1 and 2
    key += " v";
    for (int q = 1; q < 3; ++q)
      for (int a = 0; a < 3; ++a) key += std::to_string(p->bcv[q][a][0]) + std::to_string(p->bcv[q][a][1]);
  }
  return key;
}

bool tune_cache_lookup(const char* path, const std::string& key, int lines[5], int modes[5]) {
  std::lock_guard<std::mutex> lock(g_tune_cache_mu);
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    const size_t kl = key.size();
    if (std::strncmp(line, key.c_str(), kl) != 0 || line[kl] != ' ') continue;
    int b[5], m[5];
    if (std::sscanf(line + kl, " B%d,%d,%d,%d,%d M%d,%d,%d,%d,%d", &b[0], &b[1], &b[2], &b[3], &b[4], &m[0],
                    &m[1], &m[2], &m[3], &m[4]) == 10) {
      for (int i = 0; i < 5; ++i) {
        lines[i] = b[i];
        modes[i] = m[i];
      }
      found = true;  // the last entry of a key wins
    }
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const char* path, const std::string& key, const fm_plan_s* p) {
  std::lock_guard<std::mutex> lock(g_tune_cache_mu);
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s B%d,%d,%d,%d,%d M%d,%d,%d,%d,%d\n", key.c_str(), p->pass[0].B, p->pass[1].B, p->pass[2].B,
               p->pass[3].B, p->pass[4].B, launch_mode(p->pass[0], p->elem), launch_mode(p->pass[1], p->elem),
               launch_mode(p->pass[2], p->elem), launch_mode(p->pass[3], p->elem), launch_mode(p->pass[4], p->elem));
  std::fclose(f);
}

}  // namespace
}  // extern "C++"

int fm_plan_tune(fm_plan p, void* workspace_dev, void* hip_stream) {
  if (!p) return FM_E_NULL;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const char* cache = std::getenv("FLUXMI_TUNE_CACHE");
  std::string key;
  if (cache && *cache) {
    key = tune_key(p);
    int lines[5], modes[5];
    if (tune_cache_lookup(cache, key, lines, modes) && apply_tiling(p, lines, modes, st) == FM_OK) {
      p->tuned_from_cache = 1;
      return FM_OK;
    }
  }
  p->tuned_from_cache = 0;
  char* ws = reinterpret_cast<char*>(workspace_dev);
  if (!ws && !(ws = own_workspace(p))) return FM_E_NOMEM;
  // scratch right-hand side and output (their values do not change the timing)
  const size_t ubytes = (size_t)p->Vu * p->ncomp * p->elem;
  void* rhs = nullptr;
  void* out = nullptr;
  if (plan_malloc(&rhs, ubytes) != hipSuccess) return FM_E_NOMEM;
  if (plan_malloc(&out, ubytes) != hipSuccess) {
    (void)hipFree(rhs);
    return FM_E_NOMEM;
  }
  int rc = FM_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipMemsetAsync(rhs, 0, ubytes, st);
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  const void* ins[5];
  void* outs[5];
  bind_buffers(p, rhs, out, ws, ins, outs);
  // time one pass with descriptor d (uploaded to the plan's device slot): a sample is n
  // launches back to back between two events, n chosen so that a sample lasts about 0.2
  // ms (launch jitter of passes of ten microseconds would otherwise decide); best of 3
  auto time_pass = [&](int i, const fm::PassDesc& d, float* ms) -> hipError_t {
    hipError_t e = hipMemcpyAsync(p->dpass + i, &d, sizeof(fm::PassDesc), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(st);
    auto sample = [&](int n, float* t) {
      hipError_t r = hipEventRecord(e0, st);
      for (int k = 0; k < n && r == hipSuccess; ++k)
        r = (p->prec == FM_F64) ? fm::launch_pass<double>(d, p->dpass + i, ins[i], outs[i], st)
                                : fm::launch_pass<float>(d, p->dpass + i, ins[i], outs[i], st);
      if (r == hipSuccess) r = hipEventRecord(e1, st);
      if (r == hipSuccess) r = hipEventSynchronize(e1);
      if (r == hipSuccess) r = hipEventElapsedTime(t, e0, e1);
      *t /= (float)n;
      return r;
    };
    float t1 = 0.f;
    if (e == hipSuccess) e = sample(1, &t1);  // warms up
    if (e == hipSuccess) e = sample(1, &t1);
    const int n = std::max(1, std::min(64, (int)std::ceil(0.2f / std::max(t1, 1e-4f))));
    float best = 1e30f;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
      float t = 0.f;
      e = sample(n, &t);
      best = std::min(best, t);
    }
    *ms = best;
    return e;
  };
  for (int i = 0; i < 5 && he == hipSuccess; ++i) {
    if (i == 2 && p->vec3) continue;  // not launched (the real curl replaces it)
    fm::PassDesc best = p->pass[i];
    float best_ms = 0.f;
    he = time_pass(i, best, &best_ms);
    std::vector<std::pair<int, int>> seen{{best.B, launch_mode(best, p->elem)}};
    for (const int bmax : {64, 32, 16, 8, 4, 2, 1}) {
      for (const int mode : {1, 0, 2, 3, 4, 5}) {
        fm::PassDesc d;
        if (he != hipSuccess || !retile(p, i, bmax, mode, &d)) continue;
        const std::pair<int, int> key{d.B, launch_mode(d, p->elem)};
        if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
        seen.push_back(key);
        float ms = 0.f;
        he = time_pass(i, d, &ms);
        if (he == hipSuccess && ms < best_ms) {
          best_ms = ms;
          best = d;
        }
      }
    }
    p->pass[i] = best;
    if (he == hipSuccess)
      he = hipMemcpyAsync(p->dpass + i, &p->pass[i], sizeof(fm::PassDesc), hipMemcpyHostToDevice, st);
  }
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he == hipSuccess && p->vec) he = upload_vec_descs(p, st);
  if (he != hipSuccess) {
    g_last_hip = (int)he;
    rc = FM_E_HIP;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(rhs);
  (void)hipFree(out);
  if (rc == FM_OK && cache && *cache) tune_cache_store(cache, key, p);
  return rc;
}

int fm_plan_device_bytes(fm_plan p, size_t* bytes) {
  if (!p || !bytes) return FM_E_NULL;
  *bytes = p->table_bytes;
  return FM_OK;
}

int fm_plan_tiling(fm_plan p, int lines_per_tile[5], int tiles[5], int persist[5]) {
  if (!p || !lines_per_tile || !tiles || !persist) return FM_E_NULL;
  for (int i = 0; i < 5; ++i) {
    lines_per_tile[i] = p->pass[i].B;
    tiles[i] = p->pass[i].tiles;
    persist[i] = launch_mode(p->pass[i], p->elem);
  }
  return FM_OK;
}

int fm_plan_set_tiling(fm_plan p, const int lines_per_tile[5], const int persist[5], void* hip_stream) {
  if (!p || !lines_per_tile || !persist) return FM_E_NULL;
  return apply_tiling(p, lines_per_tile, persist, reinterpret_cast<hipStream_t>(hip_stream));
}

int fm_plan_tuned_from_cache(fm_plan p, int* from_cache) {
  if (!p || !from_cache) return FM_E_NULL;
  *from_cache = p->tuned_from_cache;
  return FM_OK;
}

int fm_batch_prepare(fm_batch* out, int count, const fm_plan* plans, const void* const* rhs_dev,
                     void* const* out_dev, void* workspace_dev, size_t workspace_bytes,
                     void* hip_stream) {
  if (!out) return FM_E_NULL;
  *out = nullptr;
  if (count <= 0) return FM_E_ARG;
  fm_batch_s* b = new (std::nothrow) fm_batch_s();
  if (!b) return FM_E_NOMEM;
  std::vector<char> host;
  int rc = build_batch(count, plans, rhs_dev, out_dev, workspace_dev, workspace_bytes, b, &host);
  if (rc == FM_OK && !host.empty()) {
    // uploaded once, synchronously: fm_batch_run then only launches kernels
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = hipMemcpyAsync(b->dev_tables, host.data(), host.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      rc = FM_E_HIP;
    }
  }
  if (rc == FM_OK && b->prec == FM_F32) {
    const int K = count < kBatchLanes ? count : kBatchLanes;
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    b->lanes.assign(K, nullptr);
    b->joins.assign(K, nullptr);
    for (int k = 0; k < K && e == hipSuccess; ++k) {
      e = hipStreamCreateWithFlags(&b->lanes[k], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->joins[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      rc = FM_E_HIP;
    }
  }
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return FM_OK;
}

int fm_batch_run(fm_batch b, void* hip_stream) {
  if (!b) return FM_E_NULL;
  return run_batch(*b, reinterpret_cast<hipStream_t>(hip_stream));
}

int fm_batch_destroy(fm_batch b) {
  delete b;
  return FM_OK;
}

}  // extern "C"
