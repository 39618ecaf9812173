/*
 * fluxmi — Fourier-convolution Poisson and Biot-Savart solver for one AMD MI355X
 * (gfx950), after the FLUPS method (Balty, Chatelain, Gillis, arXiv 2211.07777).
 *
 * The solve computes u = G * f (Poisson, lap(u) = f; Eq. of Sec. II) or
 * u = G * curl(f) (Biot-Savart, lap(u) = curl(f); Sec. V) on a uniform 3-D grid whose
 * six faces each carry one boundary condition: even, odd (Sec. II-B, Table I),
 * periodic (Sec. II-B) or unbounded (Sec. II-C; with a symmetric face opposite it the
 * direction is semi-unbounded).  Each solve zero-pads unbounded directions (domain
 * doubling), runs per-axis DFT / DCT / DST passes chosen from the boundary
 * conditions, multiplies by a cached Green's spectrum (optionally through a spectral
 * curl) and runs the inverse passes.
 *
 * Conventions shared by every entry point
 *   - All functions use the C ABI, never throw, and return an int status:
 *     FM_OK (0) or one of the negative FM_E_* codes below.
 *   - Device pointers are plain HIP device addresses (e.g. from a torch tensor's
 *     data_ptr()); `hip_stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  All device work is stream-ordered; no entry point synchronises the
 *     host with the device except fm_plan_create, which waits for the Green's spectrum.
 *   - Arrays are contiguous, row-major, x fastest: [ncomp][nz][ny][nx] where n_a is
 *     N_a cells (cell-centred: x_j = (j + 1/2) h) or N_a + 1 nodes (node-centred:
 *     x_j = j h), Sec. II-A.  Element type double (FM_F64) or float (FM_F32).
 *   - Axis a spans L_a = N_a * h_a.  Face order is (x-left, x-right, y-left, ...).
 */
#ifndef FLUXMI_H
#define FLUXMI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary condition of one face (Sec. II-B, II-C). */
typedef enum { FM_BC_EVEN = 0, FM_BC_ODD = 1, FM_BC_PER = 2, FM_BC_UNB = 3 } fm_bc;

/* Data layout (Sec. II-A). */
typedef enum { FM_CELL = 0, FM_NODE = 1 } fm_layout;

/* Green's function (Sec. IV names the CHAT2 kernel; its singular value at the origin
 * is not printed in the paper):
 *   FM_GREEN_CHAT2     -1/(4 pi r) with the origin value equal to the mean over the
 *                      equal-volume sphere times the cell volume (the reading that
 *                      reproduces the CHAT2 errors printed in Sec. IV);
 *   FM_GREEN_CHAT2_VOL the same kernel with the plain equal-volume-sphere mean.
 * With two convolution directions both use, at the origin, the square-cell mean of
 * ln(rho)/(2 pi) (footnote of Sec. V) for the zero spectral wavenumber and the disc
 * mean of -K0(k rho)/(2 pi) otherwise.
 * Regularised kernels (Sec. IV, the HEJ family; their formulas come from the work the
 * paper cites for them): the Green's function of a smoothed point source
 *   FM_GREEN_HEJ2 ... FM_GREEN_HEJ10  order m = 2, 4, 6, 8, 10: the Gaussian-Laguerre
 *                      source of width eps whose moments vanish up to order m,
 *                      Fourier transform exp(-s) sum_{j < m/2} s^j / j!,
 *                      s = (k eps)^2 / 2;
 *   FM_GREEN_HEJ0      the spectrally truncated point source: wavenumbers with
 *                      |k| <= pi / h kept, the rest cut off.
 * eps = 2 h with h = (hx hy hz)^(1/3) (the reading that reproduces the printed errors of
 * every HEJ kernel).  These need three unbounded directions (the real-space form
 * -(1/4 pi r)[erf(r / (sqrt 2 eps)) + ...], finite at r = 0) or none (the spectral form
 * -zeta_hat(k) / k^2); other mixes return FM_E_KIND.
 * FM_GREEN_LGF2 (Sec. IV, the lattice Green's function): the Green's function of the
 * second-difference (7-point) Laplacian, so that the solve inverts that discrete operator
 * exactly: sampled at the integer offsets of three unbounded-type directions, or
 * -1 / sum_a (2 sin(k_a h_a / 2) / h_a)^2 with no unbounded direction; other mixes return
 * FM_E_KIND. */
typedef enum {
  FM_GREEN_CHAT2 = 0,
  FM_GREEN_CHAT2_VOL = 1,
  FM_GREEN_HEJ2 = 2,
  FM_GREEN_HEJ4 = 3,
  FM_GREEN_HEJ6 = 4,
  FM_GREEN_HEJ8 = 5,
  FM_GREEN_HEJ10 = 6,
  FM_GREEN_HEJ0 = 7,
  FM_GREEN_LGF2 = 8
} fm_green;

/* Arithmetic of the transforms.  FM_F32 plans take their twiddles and Green's
 * spectrum from FP64 evaluations rounded once to FP32. */
typedef enum { FM_F64 = 0, FM_F32 = 1 } fm_prec;

/* Poisson: lap(u) = f.  Biot-Savart: lap(u) = curl(f) with the curl taken in
 * spectral space as i*omega x f_hat (Sec. V); needs periodic or fully unbounded
 * conditions on every axis and ncomp = 3.  The _FD kinds replace the derivative i*omega
 * by the symbol of the central difference of order 2, 4 or 6 (Sec. V):
 * (i/h) sin(w h), (i/h) (4/3 sin(w h) - 1/6 sin(2 w h)),
 * (i/h) (3/2 sin(w h) - 3/10 sin(2 w h) + 1/30 sin(3 w h)), h the spacing of the axis. */
typedef enum {
  FM_POISSON = 0,
  FM_BIOT_SAVART = 1,
  FM_BIOT_SAVART_FD2 = 2,
  FM_BIOT_SAVART_FD4 = 3,
  FM_BIOT_SAVART_FD6 = 4
} fm_kind;

/* Status codes. */
#define FM_OK 0
#define FM_E_NULL (-1)   /* a required pointer is NULL                                */
#define FM_E_BC (-2)     /* periodic on one face only, or an unknown code             */
#define FM_E_SIZE (-3)   /* N < 2, h <= 0, or an FFT length with a prime factor > 7
                            or longer than 4096                                       */
#define FM_E_KIND (-4)   /* unknown kind / green / precision / layout, Biot-Savart with
                            ncomp != 3, or with a symmetric / semi-unbounded axis in
                            fm_plan_create (fm_plan_create_vector takes one)          */
#define FM_E_NOMEM (-5)  /* device allocation failed                                 */
#define FM_E_HIP (-6)    /* a HIP call failed; fm_last_hip_error() has its code      */
#define FM_E_ARG (-7)    /* inconsistent arguments (count, workspace too small, ...) */
#define FM_E_SCRATCH (-8) /* fm_solve_static: the plan's workspace exceeds
                             FM_STATIC_WORKSPACE_BYTES                                */

/* Size of the library's fixed device workspace used by fm_solve_static. */
#define FM_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)

typedef struct fm_plan_s* fm_plan;

/* Create a plan: classifies every axis (Table I and Sec. II-C), orders the axes by
 * transform cost (symmetric, semi-unbounded, periodic, unbounded; Sec. I), sizes the
 * padded transforms, and builds the twiddle tables and the Green's spectrum in FP64
 * on the device (once per plan).
 *   out       receives the plan (set to NULL on failure)
 *   n[3]      N per axis (x, y, z): cells, or intervals for node-centred data
 *   h[3]      grid spacing per axis
 *   bc[3][2]  per-axis (left, right) face conditions
 *   ncomp     independent right-hand sides per solve (Poisson), 3 for Biot-Savart
 *   hip_stream  stream on which the spectrum is generated (synchronised on return)
 * The plan owns its device memory (spectrum, twiddles, internal workspace). */
int fm_plan_create(fm_plan* out, const int n[3], const double h[3], const int bc[3][2],
                   int layout, int green, int prec, int kind, int ncomp, void* hip_stream);

/* Biot-Savart with boundary conditions per component (Sec. V): lap(u) = curl(f) for a
 * source f whose components have their own faces, bc[q][a][f] for component q (x, y, z),
 * axis a, face f (left, right).  The faces must be those of a mirror-symmetric vector
 * field: periodic and unbounded faces are shared by the three components; on a symmetric
 * (even or odd) face of axis a, component a has one symmetry and the two other
 * components the opposite one (else FM_E_BC).  A derivative along a symmetric direction
 * turns even into odd and odd into even, so component p of the solution has the faces of
 * component p of f with even and odd swapped; in spectral space the derivative of a sine
 * coefficient is +w times it and that of a cosine coefficient -w times it (Sec. V).
 * Any number of axes may be symmetric or semi-unbounded (Sec. II-B, II-C), the others
 * periodic or unbounded; without a symmetric face the plan is fm_plan_create's
 * Biot-Savart plan.  kind: FM_BIOT_SAVART or one of its _FD forms; the other arguments,
 * the ownership and the solve calls as for fm_plan_create with ncomp = 3.  Such a plan
 * is solved one request at a time: fm_solve_batched, fm_batch_prepare, fm_fft_forward
 * and fm_fft_backward return FM_E_KIND for it.
 * Errors: FM_E_NULL, FM_E_BC, FM_E_SIZE, FM_E_KIND, FM_E_NOMEM, FM_E_HIP. */
int fm_plan_create_vector(fm_plan* out, const int n[3], const double h[3], const int bc[3][3][2],
                          int layout, int green, int prec, int kind, void* hip_stream);

/* Release a plan and its device memory.  The caller must make sure no solve that
 * uses it is still in flight.  NULL is accepted and ignored. */
int fm_plan_destroy(fm_plan p);

/* Bytes of device workspace a solve with this plan needs: per component, the spectrum
 * after the first transform and the spectrum after the first two (Sec. III: the data
 * between two topology switches), each with its complex or real extent per axis
 * (Sec. II-B, II-C); the zero padding of unbounded directions is never stored.
 * Errors: FM_E_NULL. */
int fm_plan_workspace_bytes(fm_plan p, size_t* bytes);

/* The user array extents (nx, ny, nz): N cells, or N + 1 nodes, per axis (the point
 * numbering of Sec. II-A).  Errors: FM_E_NULL. */
int fm_plan_shape(fm_plan p, int user_dims[3]);

/* Solve for one set of right-hand sides: forward transforms along the three axes, the
 * product with the Green's spectrum (Poisson; the convolution of Sec. II) or with the
 * Green's spectrum times i*omega x (Biot-Savart; Sec. V), inverse transforms and the
 * crop of the padded directions (Sec. II-C), in the axis order of Sec. III.
 *   rhs_dev   [ncomp][nz][ny][nx] input, never written
 *   out_dev   same shape; may alias rhs_dev (in-place mode)
 *   workspace_dev  at least fm_plan_workspace_bytes bytes, or NULL to use the plan's
 *             own workspace, allocated on first use (then concurrent solves with one plan
 *             must not overlap)
 * The caller keeps ownership of every buffer.  Output conventions: nodes on an odd face
 * are exactly 0; the node-centred periodic duplicate f_N equals f_0 (Sec. II-A); input
 * values at those positions are ignored.
 * Errors: FM_E_NULL, FM_E_NOMEM (the plan's own workspace), FM_E_HIP (a launch). */
int fm_solve(fm_plan p, const void* rhs_dev, void* out_dev, void* workspace_dev, void* hip_stream);

/* fm_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the workspace is a
 * fixed device array of the library, FM_STATIC_WORKSPACE_BYTES (128 MiB) per GPU, held
 * from the library's load until the process ends.  The call allocates nothing (no
 * hipMalloc, no allocating library routine); rhs_dev and out_dev are the caller's, as
 * for fm_solve, and the results are those of fm_solve with the same plan.
 * Every call on one GPU uses that GPU's one array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other host threads) race and
 * must be serialised by the caller.
 * Errors: FM_E_NULL; FM_E_SCRATCH if fm_plan_workspace_bytes exceeds
 * FM_STATIC_WORKSPACE_BYTES (e.g. FP32 fully unbounded grids beyond about 180^3);
 * FM_E_HIP (symbol lookup or launch). */
int fm_solve_static(fm_plan p, const void* rhs_dev, void* out_dev, void* hip_stream);

/* Run passes [first_pass, last_pass] (0-based, of the five: 0 first-axis forward,
 * 1 second-axis forward, 2 last-axis forward + spectral multiply + inverse,
 * 3 second-axis inverse, 4 first-axis inverse) of fm_solve with the same arguments.
 * Running 0..4 in one or several calls, in order on one stream, equals fm_solve; the
 * workspace carries the intermediate results between calls, so it must be passed
 * explicitly (NULL selects the plan's own workspace). */
int fm_solve_passes(fm_plan p, const void* rhs_dev, void* out_dev, void* workspace_dev,
                    int first_pass, int last_pass, void* hip_stream);

/* The plain transforms of a plan, without the spectral multiplication: the forward
 * operation of every axis chosen by its boundary conditions (DFT of the zero-padded
 * data along unbounded axes, DFT along periodic axes, the DCT / DST of Table I along
 * symmetric axes, the padded DCT / DST along semi-unbounded axes; Sec. II-B, II-C), and
 * the backward operation with the crop and the output conventions of fm_solve.  Both
 * are unnormalised (backward(forward(f)) = prod_a n_log,a * f, where n_log is N for a
 * periodic axis, 2N for an unbounded or symmetric one and 4N for a semi-unbounded one).
 * The first DFT axis in the plan's order holds the half spectrum (k <= M/2) of its
 * real-to-complex transform.  The spectrum is laid out as fm_plan_spectrum_layout
 * reports: [ncomp][dims[0]][dims[1]][dims[2]] (dims[2] fastest), where axes[i] is the
 * physical axis (0 x, 1 y, 2 z) of dimension i, complex interleaved if is_complex, in the
 * plan's precision; *bytes is its size.  This is the layout the solve works in (the last
 * transformed axis fastest), so a forward transform costs three passes and moves no
 * data twice.  rhs / out as for fm_solve; the workspace as for fm_solve (its contents
 * do not carry over between the two calls).
 * Errors: FM_E_NULL, FM_E_NOMEM (the plan's own workspace), FM_E_HIP. */
int fm_plan_spectrum_layout(fm_plan p, int dims[3], int axes[3], int* is_complex, size_t* bytes);
int fm_fft_forward(fm_plan p, const void* in_dev, void* spec_dev, void* workspace_dev, void* hip_stream);
int fm_fft_backward(fm_plan p, const void* spec_dev, void* out_dev, void* workspace_dev, void* hip_stream);

/* Solve `count` independent problems (plans may differ in shape, boundary conditions
 * and layout, but must share one precision).  FP64 batches run with one launch per pass
 * and length class for the whole batch, except fused passes in the per-wavefront kernel
 * (fm_plan_tiling mode 3), which are launched plan by plan; FP32 batches run plan by plan
 * with the single-solve kernels.  Each result is bitwise identical to fm_solve of the same plan.
 *   workspace_dev  at least fm_batched_workspace_bytes(count, plans) bytes
 * Errors: FM_E_ARG if the plans mix precisions or the workspace is too small, FM_E_NULL
 * for a null plan array, buffer array or buffer. */
int fm_solve_batched(int count, const fm_plan* plans, const void* const* rhs_dev,
                     void* const* out_dev, void* workspace_dev, size_t workspace_bytes,
                     void* hip_stream);

/* Autotuner: times every pass of the plan on the device for candidate tilings (lines
 * per tile; a persistent grid, or one tile per workgroup with the twiddle tables in LDS
 * or read from global memory), keeps the fastest valid one
 * per pass in the plan, and uses it for every later solve.  Results can change at the
 * rounding level only: two real lines share one complex FFT, and which lines are paired
 * follows the tiling.  workspace_dev as for fm_solve (NULL: the plan's own);
 * the call allocates two scratch arrays of the user shape and synchronises hip_stream.
 * Not to be called while solves with this plan are in flight.
 * With the environment variable FLUXMI_TUNE_CACHE naming a file, the call first looks
 * up the plan's problem (device name and CU count, precision, kind, components, layout,
 * Green's function, sizes and boundary conditions) there and, when an entry validates
 * for this plan, applies it without timing anything; otherwise it tunes and appends the
 * result as one text line.  Concurrent calls in one process are serialised on the file. */
int fm_plan_tune(fm_plan p, void* workspace_dev, void* hip_stream);

/* *from_cache = 1 when the last fm_plan_tune of p applied a FLUXMI_TUNE_CACHE entry,
 * else 0. */
int fm_plan_tuned_from_cache(fm_plan p, int* from_cache);

/* Device memory held by the plan's tables (Green's spectrum, twiddles, descriptors),
 * not counting its own workspace. */
int fm_plan_device_bytes(fm_plan p, size_t* bytes);

/* The plan's current tiling per pass: lines per tile, tiles, and the launch mode
 * persist[i]: 1 persistent grid (twiddle tables in LDS), 0 one tile per workgroup with
 * the tables in LDS, 2 one tile per workgroup with the tables read from global memory,
 * 3, 4 and 5 the per-wavefront kernels with 16, 8 and 32 values per lane (lines of a
 * power-of-two length: each 64-lane wavefront transforms whole lines in registers,
 * exchanging values through its own LDS; for the fused pass it also multiplies and
 * inverts them; lines_per_tile is then the lines of one workgroup).  Mode 5 serves the
 * fused pass of FP32 Poisson plans only. */
int fm_plan_tiling(fm_plan p, int lines_per_tile[5], int tiles[5], int persist[5]);

/* Set the tiling of every pass, as fm_plan_tiling reports it (for example a tiling that
 * fm_plan_tune found earlier for the same problem and device): lines_per_tile[i] lines
 * per tile and launch mode persist[i] for pass i.  The result of a solve can change at
 * the rounding level only (as after fm_plan_tune).  The descriptors are uploaded on
 * hip_stream, which is synchronised.  Not to be called while solves with this plan are
 * in flight.  Errors: FM_E_NULL; FM_E_ARG if a pass cannot run with exactly that
 * tiling (register, LDS or addressing limits of its kernel); FM_E_HIP. */
int fm_plan_set_tiling(fm_plan p, const int lines_per_tile[5], const int persist[5], void* hip_stream);

/* A batch prepared once and launched many times: the same work as fm_solve_batched on
 * fixed buffers.  fm_batch_prepare binds the plans, right-hand sides, outputs and
 * workspace (arguments as for fm_solve_batched; the workspace must stay allocated and
 * untouched by others while the batch exists), uploads the batch's descriptor tables
 * into the workspace and waits for that copy on hip_stream.  fm_batch_run enqueues the
 * kernels only (no copies, no allocation, no host synchronisation), so it can be
 * recorded into a HIP graph and replayed; each replay recomputes the outputs from the
 * current contents of the right-hand sides.  FP32 batches run their solves side by side
 * on up to 8 streams of the batch's own (default priority), forked from hip_stream and
 * joined back into it with events, so that hip_stream's later work (and a capture of
 * hip_stream) sees every solve finished.  The plans must outlive the batch.
 * Errors: as fm_solve_batched; FM_E_NULL for a null handle. */
typedef struct fm_batch_s* fm_batch;
int fm_batch_prepare(fm_batch* out, int count, const fm_plan* plans, const void* const* rhs_dev,
                     void* const* out_dev, void* workspace_dev, size_t workspace_bytes,
                     void* hip_stream);
int fm_batch_run(fm_batch b, void* hip_stream);
int fm_batch_destroy(fm_batch b);

/* Serving loop (continuous admission).  A server owns one device arena of
 * workspace_budget_bytes for the workspaces of running requests and a cache of plans
 * whose tables may use up to plan_budget_bytes (least recently used plans with no
 * waiting or running request are destroyed beyond that).  Each request is one solve
 * (fm_solve semantics; rhs_dev / out_dev are the caller's and must stay valid until the
 * request has finished).  fm_server_submit records an event on hip_stream, the
 * stream on which the caller produced rhs_dev and last used out_dev (NULL: the null
 * stream): the request's solve runs after that work.  A request that needs a new plan
 * has it generated on the server's own stream; neither submission nor admission waits
 * for the device (except with tune_plans, which times the new plan's kernels).
 * Requests wait in FIFO order until one of `slots` device streams and their workspace
 * are free; then they run, overlapping on the device with the other running requests.
 * fm_server_progress retires finished requests, admits waiting ones and returns the
 * finished tickets in completion order, with status[i] FM_OK or the error that kept
 * the request from running (status may be NULL); it never blocks.  fm_server_wait_all
 * blocks until every submitted request has finished.  tune_plans != 0 autotunes each
 * new plan (fm_plan_tune).  One host thread drives a server.  Errors: FM_E_ARG (slots
 * outside 1..64, zero budget), FM_E_NOMEM (arena, or a request whose workspace exceeds
 * the whole budget), FM_E_HIP, and those of fm_plan_create for a request (the request
 * is then not queued). */
typedef struct fm_server_s* fm_server;
typedef struct {
  long long submitted, finished;               /* requests (finished counts failed) */
  long long plan_hits, plan_misses, plan_evictions;
  size_t peak_workspace_bytes;                 /* arena bytes in use, maximum */
  int peak_inflight;                           /* requests running at once, maximum */
  int cached_plans, waiting, running;          /* now */
  size_t plan_bytes;                           /* device bytes of the cached plans, now */
  long long failed;                            /* requests finished with an error */
} fm_server_stats;
int fm_server_create(fm_server* out, size_t workspace_budget_bytes, size_t plan_budget_bytes,
                     int slots, int tune_plans);
int fm_server_submit(fm_server s, const int n[3], const double h[3], const int bc[3][2], int layout,
                     int green, int prec, int kind, int ncomp, const void* rhs_dev, void* out_dev,
                     void* hip_stream, long long* ticket);
int fm_server_progress(fm_server s, long long* finished, int* status, int max_finished,
                       int* n_finished);
int fm_server_wait_all(fm_server s);
int fm_server_get_stats(fm_server s, fm_server_stats* stats);
int fm_server_destroy(fm_server s);

/* Workspace for fm_solve_batched: the sum over plans of fm_plan_workspace_bytes,
 * each rounded up to 256 bytes, plus the batch's descriptor table. */
int fm_batched_workspace_bytes(int count, const fm_plan* plans, size_t* bytes);

/* Planning information, available without a device (host-only arithmetic). */
typedef struct {
  int order[3];         /* transform order, as axis indices (0 x, 1 y, 2 z)           */
  int axis_class[3];    /* per axis x, y, z: 0 P, 1 EE, 2 OO, 3 EO, 4 OE, 5 UU, 6 EU,
                           7 OU, 8 UE, 9 UO (left face first)                          */
  int fft_len[3];       /* FFT length used along each axis                           */
  int spec_len[3];      /* extent of each axis after its forward transform           */
  int green_dims[3];    /* Green table extents, in transform order                   */
  size_t workspace_bytes;
  int tiles[5];         /* workgroups of the five passes                             */
  int lines_per_tile[5];
  int lds_bytes[5];
  double algo_bytes[5]; /* bytes each pass must move (reads + writes of the live
                           volumes, zero padding never read, the Green's spectrum read
                           once by the fused pass), all components                          */
} fm_plan_info;

/* Run the planner of fm_plan_create (classification, order, sizes, layouts, tiles and
 * the bounds check of every pass) without touching a device.  Same arguments and
 * status codes as fm_plan_create; nothing is allocated. */
int fm_plan_inspect(const int n[3], const double h[3], const int bc[3][2], int layout, int green,
                    int prec, int kind, int ncomp, fm_plan_info* info);

/* Human-readable text for a status code (static storage). */
const char* fm_error_string(int status);

/* The last HIP error code seen by this library in the calling thread (0 if none). */
int fm_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FLUXMI_H */
