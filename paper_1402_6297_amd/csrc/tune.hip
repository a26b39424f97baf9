// Launch-tiling autotuner: times the A_r apply of a plan under candidate
// tilings of its FFT passes and keeps the fastest.  The knobs are the pass
// family (two-level register passes, generic LDS-staged passes, single-wave x
// and z passes) and, for the two-level family, the workgroup tiles: one field
// pair or all six fields per workgroup of the fused z pass and its pencils per
// workgroup, rows per workgroup of the x passes and pencils per workgroup of
// the y / z passes.  The search is
// coordinate descent from the defaults, two sweeps over the knobs.  Every
// candidate computes the same transforms; only the arithmetic order of the CG
// reductions (partials per workgroup) can change, so results agree to rounding.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "nsf_internal.h"

namespace nsf {
namespace {

struct Tiling {
  int path, mid, xr, yz, pairs;
  bool operator==(const Tiling& o) const {
    return path == o.path && mid == o.mid && xr == o.xr && yz == o.yz && pairs == o.pairs;
  }
};

void apply_tiling(nsf_plan p, const Tiling& t) {
  p->opt_fft_path = t.path;
  p->opt_mid_cols = t.mid;
  p->geom.x_rows = t.xr;
  p->geom.yz_cols = t.yz;
  p->geom.mid_pairs = t.pairs;
}

// Average milliseconds of one A_r apply (after two untimed ones).
int time_apply(nsf_plan p, const double2* u, double2* out, int reps, hipEvent_t e0, hipEvent_t e1, double* ms) {
  for (int i = 0; i < 2; ++i) {
    const int rc = apply_Ar_dev(p, u, out, nullptr);
    if (rc) return rc;
  }
  NSF_HIP(p, hipEventRecord(e0, p->stream));
  for (int i = 0; i < reps; ++i) {
    const int rc = apply_Ar_dev(p, u, out, nullptr);
    if (rc) return rc;
  }
  NSF_HIP(p, hipEventRecord(e1, p->stream));
  NSF_HIP(p, hipEventSynchronize(e1));
  float f = 0;
  NSF_HIP(p, hipEventElapsedTime(&f, e0, e1));
  *ms = (double)f / reps;
  return NSF_OK;
}

// NSF_TUNE_CACHE lines: "nsf-tune n1 n2 n3 kind path mid xr yz pairs us_best us_default".
// Cache key of a plan's medium: its kind, plus 16 x (1 + the share of z-pass
// tiles at 16 columns that are not all vacuum, in tenths) when vacuum
// skipping is on, since the best tiling then depends on that share.
int tune_key(nsf_plan p) {
  const Geom& g = p->geom;
  int key = p->medium_kind;
  // (from the plan's medium and options, not from the tiling being tried)
  const bool vac = p->opt_vacuum && p->d_ztiles && (key == kMedChiral || key == kMedPseudo);
  if (vac && p->ztile_cnt[4] >= 0 && g.n1 % 16 == 0) {
    const double all = (double)(g.n1 / 16) * (double)g.n2;
    key += 16 * (1 + (int)std::lround(10.0 * p->ztile_cnt[4] / all));
  }
  return key;
}

bool cache_lookup(const Geom& g, int kind, Tiling* t, double* us_best, double* us_dflt) {
  const char* path = std::getenv("NSF_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char tag[16];
  int n1, n2, n3, k;
  Tiling c{};
  double b, d;
  bool hit = false;
  while (std::fscanf(f, "%15s %d %d %d %d %d %d %d %d %d %lf %lf", tag, &n1, &n2, &n3, &k, &c.path, &c.mid,
                     &c.xr, &c.yz, &c.pairs, &b, &d) == 12) {
    if (std::strcmp(tag, "nsf-tune") || n1 != g.n1 || n2 != g.n2 || n3 != g.n3 || k != kind) continue;
    *t = c;  // the last matching line wins
    *us_best = b;
    *us_dflt = d;
    hit = true;
  }
  std::fclose(f);
  return hit;
}

void cache_store(const Geom& g, int kind, const Tiling& t, double us_best, double us_dflt) {
  const char* path = std::getenv("NSF_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "nsf-tune %d %d %d %d %d %d %d %d %d %.3f %.3f\n", g.n1, g.n2, g.n3, kind, t.path, t.mid, t.xr,
               t.yz, t.pairs, us_best, us_dflt);
  std::fclose(f);
}

}  // namespace
}  // namespace nsf

using namespace nsf;

extern "C" {

int nsf_plan_autotune(nsf_plan p, int reps, nsf_tune* result) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (reps < 1 || reps > 1000) return set_error(p, NSF_E_ARG, "reps must be in 1..1000");
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  int rc = ensure_device(p);
  if (rc) return rc;
  const Geom& g = p->geom;
  const long long len = 4 * g.n;
  const Tiling dflt{0, 16, 4, 16, 1};
  {
    Tiling c{};
    double b = 0, d = 0;
    if (cache_lookup(g, tune_key(p), &c, &b, &d)) {
      apply_tiling(p, c);
      if (result) {
        result->fft_path = c.path;
        result->mid_cols = c.mid;
        result->x_rows = c.xr;
        result->yz_cols = c.yz;
        result->mid_pairs = c.pairs;
        result->us_best = b;
        result->us_default = d;
        result->tried = 0;
      }
      return NSF_OK;
    }
  }
  const bool fast = fast_axis(g.n1) || fast_axis(g.n2) || fast_axis(g.n3);
  const bool wave = wave_axis(g.n1) || wave_mid_ok(g);
  const Tiling saved{p->opt_fft_path, p->opt_mid_cols, g.x_rows, g.yz_cols, g.mid_pairs};
  double2* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (buf) {
      hipStreamSynchronize(p->stream);
      hipFree(buf);
    }
  };
  auto fail = [&](int code) {
    apply_tiling(p, saved);
    cleanup();
    return code;
  };
  if (hipMalloc(&buf, sizeof(double2) * 2 * (size_t)len) != hipSuccess) {
    buf = nullptr;
    return set_error(p, NSF_E_NOMEM, "autotune: device allocation failed");
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(set_error(p, NSF_E_HIP, "autotune: event creation failed"));
  if (launch_randn(buf, len, 0x5eedULL, p->stream) != hipSuccess)
    return fail(set_error(p, NSF_E_HIP, "autotune: launch failed"));
  std::vector<std::pair<Tiling, double>> seen;
  auto measure = [&](const Tiling& t, double* ms) -> int {
    for (auto& sm : seen)
      if (sm.first == t) {
        *ms = sm.second;
        return NSF_OK;
      }
    apply_tiling(p, t);
    const int r = time_apply(p, buf, buf + len, reps, e0, e1, ms);
    if (r) return r;
    seen.emplace_back(t, *ms);
    return NSF_OK;
  };
  Tiling best = dflt;
  double best_ms = 0, dflt_ms = 0;
  if ((rc = measure(dflt, &dflt_ms))) return fail(rc);
  best_ms = dflt_ms;
  auto try_one = [&](Tiling t) -> int {
    double ms = 0;
    const int r = measure(t, &ms);
    if (r) return r;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
    return NSF_OK;
  };
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int path : {0, 1, 2}) {
      if ((path == 0 && !fast) || (path == 2 && !wave)) continue;
      Tiling t = best;
      t.path = path;
      if ((rc = try_one(t))) return fail(rc);
    }
    if (best.path != 0) continue;  // the remaining knobs tile the two-level passes
    for (int pairs : {1, 0}) {
      Tiling t = best;
      t.pairs = pairs;
      if ((rc = try_one(t))) return fail(rc);
    }
    for (int mid : {4, 8, 16}) {
      Tiling t = best;
      t.mid = mid;
      if ((rc = try_one(t))) return fail(rc);
    }
    for (int xr : {1, 2, 4}) {
      Tiling t = best;
      t.xr = xr;
      if ((rc = try_one(t))) return fail(rc);
    }
    for (int yz : {4, 8, 16}) {
      Tiling t = best;
      t.yz = yz;
      if ((rc = try_one(t))) return fail(rc);
    }
  }
  const int tried = (int)seen.size();
  apply_tiling(p, best);
  cleanup();
  cache_store(g, tune_key(p), best, best_ms * 1e3, dflt_ms * 1e3);
  if (result) {
    result->fft_path = best.path;
    result->mid_cols = best.mid;
    result->x_rows = best.xr;
    result->yz_cols = best.yz;
    result->mid_pairs = best.pairs;
    result->us_best = best_ms * 1e3;
    result->us_default = dflt_ms * 1e3;
    result->tried = tried;
  }
  return NSF_OK;
}

}  // extern "C"
