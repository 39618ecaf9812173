// Replays solves on the CPU emulation of the device code (test infrastructure): each
// case is planned and solved alone and compared with the FP64 oracle, then all cases of
// one precision are solved again in one fm_solve_batched call and compared bitwise with
// the single solves.  Each case is also solved in every launch mode its passes accept
// (fm_plan_set_tiling) and with fm_solve_static, on a stream of its own.  Finally
// Biot-Savart plans with faces per component (one, two and three symmetric axes, the
// spectral and a finite-difference curl) against the oracle's vector solve; and every
// case twice through a server (fm_server_*: three slots, a plan budget that forces
// evictions) with its right-hand side copied from pinned memory on a producer stream
// the server must wait for.  Cases come from a text file, one per line:
//   prec nx ny nz hx hy hz bx0 bx1 by0 by1 bz0 bz1 layout seed
// Prints one line per case and exits non-zero on any failure.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fluxmi.h"

extern "C" int oracle_solve(const int* n, const double* h, const int* bc, int layout, int green, int kind,
                            int mode, const double* rhs, double* out);
extern "C" int oracle_solve_vector(const int* n, const double* h, const int* bcv, int layout, int green,
                                   int kind, int mode, const double* rhs, double* out);

namespace {

struct Case {
  int prec, n[3], bc[3][2], layout;
  double h[3];
  unsigned seed;
};

// a reproducible field in [-1, 1) (64-bit LCG)
void fill(std::vector<double>& v, unsigned seed) {
  uint64_t s = 0x9e3779b97f4a7c15ull ^ seed;
  for (double& x : v) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    x = (double)(s >> 11) / (double)(1ull << 53) * 2.0 - 1.0;
  }
}

double rel_linf(const std::vector<double>& a, const std::vector<double>& ref) {
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    if (!std::isfinite(a[i])) return INFINITY;  // a NaN from uninitialised memory fails
    num = std::fmax(num, std::fabs(a[i] - ref[i]));
    den = std::fmax(den, std::fabs(ref[i]));
  }
  return den > 0 ? num / den : num;
}

struct Run {
  fm_plan plan = nullptr;
  size_t count = 0, bytes = 0;
  void* rhs = nullptr;
  void* out = nullptr;
  std::vector<double> f64;
};

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s cases.txt\n", argv[0]);
    return 2;
  }
  std::setvbuf(stdout, nullptr, _IOLBF, 0);
  FILE* fh = std::fopen(argv[1], "r");
  if (!fh) return 2;
  std::vector<Case> cases;
  Case c;
  while (std::fscanf(fh, "%d %d %d %d %lf %lf %lf %d %d %d %d %d %d %d %u", &c.prec, &c.n[0], &c.n[1], &c.n[2],
                     &c.h[0], &c.h[1], &c.h[2], &c.bc[0][0], &c.bc[0][1], &c.bc[1][0], &c.bc[1][1], &c.bc[2][0],
                     &c.bc[2][1], &c.layout, &c.seed) == 15)
    cases.push_back(c);
  std::fclose(fh);
  int failures = 0;
  for (int prec : {FM_F64, FM_F32}) {
    std::vector<Run> runs;
    for (const Case& k : cases) {
      if (k.prec != prec) continue;
      Run r;
      int rc = fm_plan_create(&r.plan, k.n, k.h, k.bc, k.layout, FM_GREEN_CHAT2, prec, FM_POISSON, 1, nullptr);
      if (rc) {
        std::printf("case n=%d,%d,%d plan failed: %s\n", k.n[0], k.n[1], k.n[2], fm_error_string(rc));
        ++failures;
        continue;
      }
      int dims[3];
      fm_plan_shape(r.plan, dims);
      r.count = (size_t)dims[0] * dims[1] * dims[2];
      const size_t es = prec == FM_F64 ? 8 : 4;
      r.bytes = r.count * es;
      r.f64.resize(r.count);
      fill(r.f64, k.seed);
      r.rhs = std::malloc(r.bytes);
      r.out = std::malloc(r.bytes);
      for (size_t i = 0; i < r.count; ++i) {
        if (es == 8) static_cast<double*>(r.rhs)[i] = r.f64[i];
        else static_cast<float*>(r.rhs)[i] = (float)r.f64[i];
      }
      std::vector<double> fin(r.count), ref(r.count);
      for (size_t i = 0; i < r.count; ++i) fin[i] = es == 8 ? r.f64[i] : (double)static_cast<float*>(r.rhs)[i];
      const int orc = oracle_solve(k.n, k.h, &k.bc[0][0], k.layout, 0, 0, 0, fin.data(), ref.data());
      const double tol = prec == FM_F64 ? 1e-12 : 1e-5;
      auto check = [&](const char* what, int status, const void* out) {
        std::vector<double> u(r.count);
        for (size_t i = 0; i < r.count; ++i)
          u[i] = es == 8 ? static_cast<const double*>(out)[i] : (double)static_cast<const float*>(out)[i];
        const double err = (status || orc) ? INFINITY : rel_linf(u, ref);
        const bool ok = err <= tol;
        failures += !ok;
        std::printf("%s %s n=%d,%d,%d bc=%d%d/%d%d/%d%d layout=%d: status %d rel_linf %.3e %s\n",
                    prec == FM_F64 ? "FP64" : "FP32", what, k.n[0], k.n[1], k.n[2], k.bc[0][0], k.bc[0][1],
                    k.bc[1][0], k.bc[1][1], k.bc[2][0], k.bc[2][1], k.layout, status, err, ok ? "ok" : "FAIL");
      };
      hipStream_t st = nullptr;
      hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      // every launch mode the passes accept, then the default tiling again
      int lines0[5], tiles0[5], mode0[5];
      fm_plan_tiling(r.plan, lines0, tiles0, mode0);
      void* tmp = std::malloc(r.bytes);
      for (int mode = 0; mode <= 5; ++mode) {
        // each pass in this mode where the pass accepts it
        // (with the first tile height of a short list that the pass takes in it)
        int modes[5], lines[5], changed = 0;
        for (int i = 0; i < 5; ++i) {
          modes[i] = mode0[i];
          lines[i] = lines0[i];
        }
        for (int i = 0; i < 5; ++i) {
          if (modes[i] == mode) continue;
          for (int b : {lines0[i], 1, 2, 4, 8, 16, 32, 64, 128, 256}) {
            modes[i] = mode;
            lines[i] = b;
            if (fm_plan_set_tiling(r.plan, lines, modes, st) == FM_OK) {
              ++changed;
              break;
            }
            modes[i] = mode0[i];
            lines[i] = lines0[i];
          }
        }
        if (!changed || fm_plan_set_tiling(r.plan, lines, modes, st) != FM_OK) continue;
        char what[32];
        std::snprintf(what, sizeof(what), "mode %d", mode);
        std::printf("  solving in mode %d (modes %d %d %d %d %d, lines %d %d %d %d %d)\n", mode, modes[0], modes[1],
                    modes[2], modes[3], modes[4], lines[0], lines[1], lines[2], lines[3], lines[4]);
        const int s1 = fm_solve(r.plan, r.rhs, tmp, nullptr, st);
        hipStreamSynchronize(st);
        check(what, s1, tmp);
      }
      rc = fm_plan_set_tiling(r.plan, lines0, mode0, st);
      const int s2 = rc ? rc : fm_solve_static(r.plan, r.rhs, tmp, st);
      hipStreamSynchronize(st);
      check("static", s2, tmp);
      std::free(tmp);
      rc = fm_solve(r.plan, r.rhs, r.out, nullptr, st);
      hipStreamSynchronize(st);
      check("single", rc, r.out);
      if (k.n[0] == 12 && k.n[1] == 10 && k.n[2] == 9) {
        // the silenced probe's sequence: the passes one call at a time with the second
        // repeated, and a batch of this one plan; both bitwise equal to the single solve
        size_t wsb = 0;
        fm_plan_workspace_bytes(r.plan, &wsb);
        void* ws = std::malloc(wsb ? wsb : 1);
        void* o1 = std::malloc(r.bytes);
        void* o2 = std::malloc(r.bytes);
        int s3 = fm_solve_passes(r.plan, r.rhs, o1, ws, 0, 0, st);
        for (int rep = 0; rep < 3 && !s3; ++rep) s3 = fm_solve_passes(r.plan, r.rhs, o1, ws, 1, 1, st);
        if (!s3) s3 = fm_solve_passes(r.plan, r.rhs, o1, ws, 2, 4, st);
        size_t bb = 0;
        int s4 = fm_batched_workspace_bytes(1, &r.plan, &bb);
        void* bws = std::malloc(bb ? bb : 1);
        const void* in1 = r.rhs;
        if (!s4) s4 = fm_solve_batched(1, &r.plan, &in1, &o2, bws, bb, st);
        hipStreamSynchronize(st);
        const bool same3 = !s3 && std::memcmp(o1, r.out, r.bytes) == 0;
        const bool same4 = !s4 && std::memcmp(o2, r.out, r.bytes) == 0;
        failures += !same3 + !same4;
        std::printf("%s probe sequence n=12,10,9: passes one by one (second repeated) status %d %s, "
                    "one-plan batch status %d %s\n",
                    prec == FM_F64 ? "FP64" : "FP32", s3, same3 ? "bitwise equal" : "FAIL", s4,
                    same4 ? "bitwise equal" : "FAIL");
        std::free(ws);
        std::free(o1);
        std::free(o2);
        std::free(bws);
      }
      hipStreamDestroy(st);
      runs.push_back(std::move(r));
    }
    if (runs.empty()) continue;
    // the same plans in one batched call, compared bitwise with the single solves
    std::vector<fm_plan> plans;
    std::vector<const void*> ins;
    std::vector<void*> outs;
    for (Run& r : runs) {
      plans.push_back(r.plan);
      ins.push_back(r.rhs);
      outs.push_back(std::malloc(r.bytes));
    }
    size_t wsb = 0;
    int rc = fm_batched_workspace_bytes((int)plans.size(), plans.data(), &wsb);
    void* ws = rc ? nullptr : std::malloc(wsb ? wsb : 1);
    if (!rc) rc = fm_solve_batched((int)plans.size(), plans.data(), ins.data(), outs.data(), ws, wsb, nullptr);
    hipDeviceSynchronize();
    int same = 0;
    for (size_t i = 0; i < runs.size(); ++i) same += !rc && std::memcmp(outs[i], runs[i].out, runs[i].bytes) == 0;
    const bool ok = !rc && same == (int)runs.size();
    failures += !ok;
    std::printf("%s batched: %d plans, status %d, %d bitwise equal to single solves %s\n",
                prec == FM_F64 ? "FP64" : "FP32", (int)runs.size(), rc, same, ok ? "ok" : "FAIL");
    std::free(ws);
    for (void* o : outs) std::free(o);
    for (Run& r : runs) {
      fm_plan_destroy(r.plan);
      std::free(r.rhs);
      std::free(r.out);
    }
  }
  // Biot-Savart with faces per component: axis a symmetric means component a even and
  // the two others odd on its faces; the other axes unbounded
  const int U = 3, E = 0, O = 1;
  for (int prec : {FM_F64, FM_F32})
    for (int nsym = 1; nsym <= 3; ++nsym)
      for (int layout = 0; layout <= 1; ++layout) {
        const int n[3] = {8, 6, 8};
        const double h[3] = {0.1, 0.12, 0.09};
        int bcv[3][3][2];
        for (int q = 0; q < 3; ++q)
          for (int a = 0; a < 3; ++a) {
            const bool sym = a >= 3 - nsym;
            bcv[q][a][0] = bcv[q][a][1] = sym ? (q == a ? E : O) : U;
          }
        const int kind = nsym == 2 ? FM_BIOT_SAVART_FD4 : FM_BIOT_SAVART;
        fm_plan plan = nullptr;
        int rc = fm_plan_create_vector(&plan, n, h, bcv, layout, FM_GREEN_CHAT2, prec, kind, nullptr);
        if (rc) {
          std::printf("vector plan failed: %s\n", fm_error_string(rc));
          ++failures;
          continue;
        }
        int dims[3];
        fm_plan_shape(plan, dims);
        const size_t count = 3 * (size_t)dims[0] * dims[1] * dims[2];
        const size_t es = prec == FM_F64 ? 8 : 4;
        std::vector<double> f(count), ref(count), u(count);
        fill(f, 100 + nsym);
        void* rhs = std::malloc(count * es);
        void* out = std::malloc(count * es);
        for (size_t i = 0; i < count; ++i) {
          if (es == 8) static_cast<double*>(rhs)[i] = f[i];
          else {
            static_cast<float*>(rhs)[i] = (float)f[i];
            f[i] = (double)static_cast<float*>(rhs)[i];
          }
        }
        rc = fm_solve(plan, rhs, out, nullptr, nullptr);
        hipDeviceSynchronize();
        const int orc = oracle_solve_vector(n, h, &bcv[0][0][0], layout, 0, kind, 0, f.data(), ref.data());
        for (size_t i = 0; i < count; ++i)
          u[i] = es == 8 ? static_cast<double*>(out)[i] : (double)static_cast<float*>(out)[i];
        const double err = (rc || orc) ? INFINITY : rel_linf(u, ref);
        const double tol = prec == FM_F64 ? 1e-12 : 1e-5;
        const bool ok = err <= tol;
        failures += !ok;
        std::printf("%s vector %d symmetric axes kind %d layout %d: status %d rel_linf %.3e %s\n",
                    prec == FM_F64 ? "FP64" : "FP32", nsym, kind, layout, rc, err, ok ? "ok" : "FAIL");
        std::free(rhs);
        std::free(out);
        fm_plan_destroy(plan);
      }
  // serving: the producer stream is created before the server's streams, so that the
  // scheduler would run an unordered solve before the copy that fills its input
  {
    hipStream_t prod = nullptr;
    hipStreamCreateWithFlags(&prod, hipStreamNonBlocking);
    fm_server srv = nullptr;
    int rc = fm_server_create(&srv, (size_t)64 << 20, (size_t)1 << 20, 3, 0);
    struct Req {
      const Case* k;
      void *pin, *rhs, *out;
      size_t count, es;
      std::vector<double> ref;
    };
    std::vector<Req> reqs;
    for (int rep = 0; rep < 2 && !rc; ++rep)
      for (const Case& k : cases) {
        Req q{&k, nullptr, nullptr, nullptr, 1, k.prec == FM_F64 ? 8u : 4u, {}};
        for (int a = 0; a < 3; ++a) q.count *= (size_t)(k.n[a] + (k.layout == FM_NODE ? 1 : 0));
        std::vector<double> f(q.count);
        fill(f, k.seed + 1000);
        hipHostMalloc(&q.pin, q.count * q.es, 0);
        for (size_t i = 0; i < q.count; ++i) {
          if (q.es == 8) static_cast<double*>(q.pin)[i] = f[i];
          else {
            static_cast<float*>(q.pin)[i] = (float)f[i];
            f[i] = (double)static_cast<float*>(q.pin)[i];
          }
        }
        q.rhs = std::malloc(q.count * q.es);
        q.out = std::malloc(q.count * q.es);
        std::memset(q.rhs, 0xff, q.count * q.es);
        q.ref.resize(q.count);
        oracle_solve(k.n, k.h, &k.bc[0][0], k.layout, 0, 0, 0, f.data(), q.ref.data());
        hipMemcpyAsync(q.rhs, q.pin, q.count * q.es, hipMemcpyHostToDevice, prod);
        long long ticket = 0;
        const int sr = fm_server_submit(srv, k.n, k.h, k.bc, k.layout, FM_GREEN_CHAT2, k.prec, FM_POISSON, 1,
                                        q.rhs, q.out, prod, &ticket);
        if (sr) {
          std::printf("serving submit failed: %s\n", fm_error_string(sr));
          ++failures;
        }
        reqs.push_back(std::move(q));
        // the second sweep reuses the cached plans: nothing in its submissions waits for
        // the device, so its copies are still queued when its solves are admitted
        if (&k == &cases.back() && rep == 0) rc = fm_server_wait_all(srv);
      }
    if (!rc) rc = fm_server_wait_all(srv);
    fm_server_stats stats{};
    if (!rc) rc = fm_server_get_stats(srv, &stats);
    int good = 0;
    for (Req& q : reqs) {
      std::vector<double> u(q.count);
      for (size_t i = 0; i < q.count; ++i)
        u[i] = q.es == 8 ? static_cast<double*>(q.out)[i] : (double)static_cast<float*>(q.out)[i];
      good += !rc && rel_linf(u, q.ref) <= (q.es == 8 ? 1e-12 : 1e-5);
    }
    const bool ok = !rc && good == (int)reqs.size() && stats.failed == 0;
    failures += !ok;
    std::printf("serving: %d requests, status %d, %d within tolerance, %lld plan hits, %lld evictions, "
                "peak in flight %d, failed %lld %s\n",
                (int)reqs.size(), rc, good, stats.plan_hits, stats.plan_evictions, stats.peak_inflight,
                stats.failed, ok ? "ok" : "FAIL");
    if (srv) fm_server_destroy(srv);
    for (Req& q : reqs) {
      hipHostFree(q.pin);
      std::free(q.rhs);
      std::free(q.out);
    }
    hipStreamDestroy(prod);
  }
  std::printf("emulated cases done, %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
