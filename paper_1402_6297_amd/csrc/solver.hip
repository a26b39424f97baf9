// CG for A_r u = b and invert Lanczos for B_r y = theta A_r y (host drivers).
//
// CG (Sec. 4.2): every recurrence scalar lives on the device, each kernel of
// an iteration returns at once when the device "done" flag is set, and the
// host reads the state only between chunks of iterations whose length it
// predicts from the observed convergence rate.
//
// Invert Lanczos (Sec. 4.2, Algorithm 1 step 5): the operator A_r^{-1} B_r is
// self-adjoint in the A_r inner product; its largest eigenvalues theta are the
// inverses of the smallest positive omega.  The basis V is kept A_r-orthonormal
// together with A_r V (classical Gram-Schmidt, two passes), and the projected
// matrix H = V^* B_r V is formed exactly from B_r applied to each new basis
// vector, so Ritz values are exact Rayleigh quotients even though the inner
// solves are inexact.  After m expansions the basis is compressed to the best
// Ritz vectors plus the last Lanczos vector (thick restart).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <mutex>
#include <string>

#include "nsf_internal.h"

namespace nsf {

// Caller workspace layout, each part aligned to 256 bytes:
// [fields 6n][CG 24n][V, A_r V: 2 (m+1) 4n][small m x m] (double2 units).
namespace {
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t workspace_bytes(long long n, int m) {
  const size_t d2 = sizeof(double2);
  return al256(d2 * 6 * (size_t)n) + al256(d2 * 24 * (size_t)n) + al256(d2 * 2 * (size_t)(m + 1) * 4 * n) +
         al256(d2 * (size_t)m * m) + 256;
}

// Part `which` (0 fields, 1 CG, 2 basis, 3 small) of the caller workspace, or
// nullptr when there is none; *cap receives the basis capacity in vectors.
double2* ws_part(nsf_plan p, int which, size_t* basis_cap) {
  if (!p->ws) return nullptr;
  const size_t d2 = sizeof(double2);
  const long long n = p->geom.n;
  char* base = reinterpret_cast<char*>(al256(reinterpret_cast<size_t>(p->ws)));
  const size_t used0 = (size_t)(base - p->ws);
  const size_t f = al256(d2 * 6 * (size_t)n), c = al256(d2 * 24 * (size_t)n);
  if (which == 0) return reinterpret_cast<double2*>(base);
  if (which == 1) return reinterpret_cast<double2*>(base + f);
  // the rest holds V, A_r V for v vectors and a (v-1) x (v-1) matrix
  const size_t rest = p->ws_bytes > used0 + f + c ? p->ws_bytes - used0 - f - c : 0;
  size_t v = 0;
  while (al256(d2 * 2 * (v + 1) * 4 * (size_t)n) + al256(d2 * v * v) <= rest) ++v;
  if (basis_cap) *basis_cap = v;
  if (which == 2) return reinterpret_cast<double2*>(base + f + c);
  return reinterpret_cast<double2*>(base + f + c + al256(d2 * 2 * (v ? v : 1) * 4 * (size_t)n));
}

// workspace for CG and the Lanczos step: r, p, q, w, z, b (six 4n vectors)
int ensure_cg(nsf_plan p) {
  int rc = ensure_device(p);
  if (rc) return rc;
  if (p->ws) {
    p->d_cg = ws_part(p, 1);
    return NSF_OK;
  }
  if (!p->d_cg) NSF_HIP(p, hipMalloc(&p->d_cg, sizeof(double2) * 6 * 4 * (size_t)p->geom.n));
  return NSF_OK;
}

int ensure_basis(nsf_plan p, size_t vectors) {
  if (p->ws) {
    size_t cap = 0;
    p->d_basis = ws_part(p, 2, &cap);
    p->basis_vectors = cap;
    if (cap < vectors)
      return set_error(p, NSF_E_NOMEM, "the caller workspace holds a basis of " + std::to_string(cap) +
                                           " vectors, " + std::to_string(vectors) + " needed");
    return NSF_OK;
  }
  if (p->basis_vectors >= vectors) return NSF_OK;
  if (p->d_basis) {
    NSF_HIP(p, hipStreamSynchronize(p->stream));
    NSF_HIP(p, hipFree(p->d_basis));
    p->d_basis = nullptr;
    p->basis_vectors = 0;
  }
  NSF_HIP(p, hipMalloc(&p->d_basis, sizeof(double2) * 2 * vectors * 4 * (size_t)p->geom.n));
  p->basis_vectors = vectors;
  return NSF_OK;
}

int ensure_small(nsf_plan p, size_t count) {
  if (p->ws) {
    size_t cap = 0;
    p->d_small = ws_part(p, 3, &cap);
    p->small_cap = cap ? (cap - 1) * (cap - 1) : 0;
    if (p->small_cap < count) return set_error(p, NSF_E_NOMEM, "the caller workspace is too small");
    return NSF_OK;
  }
  if (p->small_cap >= count) return NSF_OK;
  if (p->d_small) {
    NSF_HIP(p, hipStreamSynchronize(p->stream));
    NSF_HIP(p, hipFree(p->d_small));
    p->d_small = nullptr;
    p->small_cap = 0;
  }
  NSF_HIP(p, hipMalloc(&p->d_small, sizeof(double2) * count));
  p->small_cap = count;
  return NSF_OK;
}

bool cg_fusable(nsf_plan p) {
  const Geom& g = p->geom;
  const int xr = fast_x_rows(g);
  return p->opt_fft_path != 1 && xr > 0 && ((long long)g.n2 * g.n3 + xr - 1) / xr <= 65536;
}

// Kept CG directions for the next solve of plan p: allocated when that solve
// runs the q-free fused schedule in plan memory with NSF_OPT_CG_RING on, else
// released (the kernels keep x updated every iteration then).  An allocation
// failure also leaves the plan on the per-iteration x update.
int ensure_ring(nsf_plan p, bool want) {
  want = want && p->opt_cg_ring && !p->ws;
  if (!want) {
    if (p->d_ring) {
      NSF_HIP(p, hipStreamSynchronize(p->stream));
      NSF_HIP(p, hipFree(p->d_ring));
      p->d_ring = nullptr;
    }
    return NSF_OK;
  }
  if (p->d_ring) return NSF_OK;
  if (hipMalloc(&p->d_ring, sizeof(double2) * kCgRing * 4 * (size_t)p->geom.n) != hipSuccess) {
    (void)hipGetLastError();
    p->d_ring = nullptr;
  }
  return NSF_OK;
}

CgFuse cg_fuse_of(nsf_plan p, double2* x, double2* cgv) {
  const long long len = 4 * p->geom.n;
  double2* c = cgv ? cgv : p->d_cg;
  return CgFuse{x, c, c + len, c + 2 * len, cgv ? nullptr : p->d_ring, p->d_state,
                reinterpret_cast<double*>(p->d_partial), reinterpret_cast<double*>(p->d_partial) + 65536,
                reinterpret_cast<double*>(p->d_partial + kPartialSlots + kCoefSlots + kResSlots)};
}

// One CG iteration of plan p, enqueued (every kernel returns at once when the
// plan's CG state is done).  With `fused` the recurrences ride in the first
// and last FFT pass.
int cg_iteration(nsf_plan p, double2* x, bool fused, double2* cgv) {
  const long long len = 4 * p->geom.n;
  hipStream_t s = p->stream;
  CgState* st = p->d_state;
  const int* skip = &st->done;
  double2* r = cgv ? cgv : p->d_cg;
  double2* pp = r + len;
  double2* q = pp + len;
  if (fused) {
    CgFuse cgf = cg_fuse_of(p, x, cgv);
    const bool qf = z_mid_pq_items(p) > 0;
    const VacSkip v = qf ? vac_of(p) : VacSkip{};  // vacuum skipping needs the q-free schedule
    cgf.pnorm = v.on ? 1 : 0;
    int np1 = 0, np5 = 0;
    NSF_HIP(p, launch_fast_cg_first(p->geom, p->tabs, cgf, p->d_fields, skip, &np1, s, nullptr, 1, qf));
    if (!qf) NSF_HIP(p, launch_cgf_check(cgf.part_in, np1, st, s));
    NSF_HIP(p, pass_yz(p, 1, +1, 6, p->d_fields, 0, 0, skip, &v));
    int npm = 0;
    NSF_HIP(p, pass_z_mid(p, p->d_fields, skip, cgf.part_mid, &npm, &v));
    if (!v.on && (npm > 0) != qf)
      return set_error(p, NSF_E_HIP, "fused CG: the z pass does not match the schedule");
    if (qf) NSF_HIP(p, launch_cgf_alpha(cgf.part_mid, npm, st, s, nullptr, 1, cgf.part_in, v.on ? np1 : 0));
    if (qf && cgf.ring) NSF_HIP(p, launch_cg_fold(x, cgf.ring, len, st, false, s));
    NSF_HIP(p, pass_yz(p, 1, -1, 6, p->d_fields, 0, 0, skip, &v));
    NSF_HIP(p, launch_fast_cg_last(p->geom, p->tabs, cgf, p->d_fields, skip, &np5, s, nullptr, 1, qf,
                                   v.on ? v.pscale : 1.0));
    if (qf)
      NSF_HIP(p, launch_cgf_step_qf(cgf.part_out, np5, st, s));
    else
      NSF_HIP(p, launch_cgf_step(cgf.part_out, np5, st, s, nullptr, 1, cgf.part_mid, npm));
    return NSF_OK;
  }
  const int nparts = reduce_parts_for(len);
  int rc = apply_Ar_dev(p, pp, q, skip);
  if (rc) return rc;
  NSF_HIP(p, launch_dot_partials(pp, q, len, p->d_partial, skip, s));
  NSF_HIP(p, launch_cg_alpha(p->d_partial, nparts, st, s));
  NSF_HIP(p, launch_cg_update(x, r, pp, q, len, p->d_partial, st, s));
  NSF_HIP(p, launch_cg_beta(p->d_partial, nparts, st, s));
  NSF_HIP(p, launch_cg_p(pp, r, len, st, s));
  return NSF_OK;
}

// Fused CG of plan p in the q-free schedule (its z pass sums p^* A_r p).
bool cg_qfree(nsf_plan p) { return cg_fusable(p) && z_mid_pq_items(p) > 0; }

// Predicted CG iterations still needed, from the convergence rate observed
// between two reads of the state (fused: one more, as the fused schedule tests
// convergence one pass later).
int cg_predict(const CgState& h, double rr_prev, int it_prev, bool fused) {
  int next = 8;
  if (rr_prev > 0 && h.rr > 0 && h.rr < rr_prev && h.iter > it_prev) {
    const double rate = std::log(rr_prev / h.rr) / (h.iter - it_prev);
    const double need = std::log(h.rr / h.thresh) / rate;
    next = (int)std::ceil(need) + (fused ? 1 : 0);
  }
  return std::min(std::max(next, 1), 16);
}

int cg_solve_dev(nsf_plan p, const double2* b, double2* x, double rtol, int maxit, int* iters,
                 double* relres, long long* matvecs, double2* cgv) {
  int rc = cgv ? NSF_OK : ensure_cg(p);
  if (rc) return rc;
  const long long len = 4 * p->geom.n;
  double2* r = cgv ? cgv : p->d_cg;
  double2* pp = r + len;
  hipStream_t s = p->stream;
  CgState* st = p->d_state;
  const int nparts = reduce_parts_for(len);
  // Fused iterations when the x axis has a two-level pass: the CG updates
  // ride in the first and last FFT pass of every A_r apply.
  const Geom& g = p->geom;
  const bool fused = cg_fusable(p);
  const bool qf = fused && cg_qfree(p);
  if (!cgv && (rc = ensure_ring(p, qf))) return rc;  // (caller vectors: no allocation, no ring)
  double2* ring = cgv ? nullptr : p->d_ring;
  NSF_HIP(p, launch_cg_init(b, x, r, ring ? ring : pp, len, p->d_partial, st, rtol, maxit, s, nullptr, 0, 0,
                            nullptr, ring ? kCgRing : 0));
  (void)nparts;
  (void)g;
  int chunk = 4;
  double rr_prev = -1.0;
  int it_prev = 0;
  for (;;) {
    for (int c = 0; c < chunk; ++c) {
      rc = cg_iteration(p, x, fused, cgv);
      if (rc) return rc;
    }
    NSF_HIP(p, hipMemcpyAsync(p->h_state, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    NSF_HIP(p, hipStreamSynchronize(s));
    const CgState& h = *p->h_state;
    if (h.done) break;
    chunk = cg_predict(h, rr_prev, it_prev, fused && !qf);
    rr_prev = h.rr;
    it_prev = h.iter;
  }
  if (qf && ring)
    NSF_HIP(p, launch_cg_fold(x, ring, len, st, true, s));
  else if (qf)
    NSF_HIP(p, launch_cg_finish(x, pp, len, st, s));
  const CgState& h = *p->h_state;
  if (iters) *iters = h.iter;
  if (relres) *relres = (h.bb > 0) ? std::sqrt(h.rr / h.bb) : 0.0;
  if (matvecs) *matvecs += h.iter;
  if (h.status == NSF_E_BREAKDOWN)
    return set_error(p, NSF_E_BREAKDOWN, "CG breakdown: p^* A_r p <= 0 or not finite");
  return h.status;
}

// ---------------------------------------------- CG without allocations
// nsf_cg_solve_noalloc keeps its three CG vectors in this array instead of
// plan memory.  Every GPU the library runs on holds its own copy until the
// process ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (kept per device below).
constexpr long long kNoAllocVoxels = 1LL << 16;
static __device__ __align__(256) double2 scratch[3 * 4 * kNoAllocVoxels];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(nsf_plan p, double2** out) {
  int dev = 0;
  NSF_HIP(p, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(p, NSF_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    NSF_HIP(p, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_error(p, NSF_E_HIP, "no device address for the CG scratch array");
    g_scratch[dev] = static_cast<double2*>(ptr);
  }
  *out = g_scratch[dev];
  return NSF_OK;
}
}  // namespace

// --------------------------------------------------- dense Hermitian eigen
// Cyclic Jacobi: each rotation J = diag(1, e^{-i phi}) R(theta) zeroes one
// off-diagonal pair (p, q) of the Hermitian matrix; sweeps continue until the
// off-diagonal mass is negligible.
int hermitian_eig(int m, const double2* Hin, double* w, double2* Vout) {
  typedef std::complex<double> cd;
  std::vector<cd> A((size_t)m * m), V((size_t)m * m, cd(0, 0));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double2 h = Hin[(size_t)i * m + j];
      const double2 hc = Hin[(size_t)j * m + i];
      A[(size_t)i * m + j] = 0.5 * (cd(h.x, h.y) + std::conj(cd(hc.x, hc.y)));  // Hermitian part
    }
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  auto at = [&](int i, int j) -> cd& { return A[(size_t)i * m + j]; };
  double fro = 0;
  for (auto& z : A) fro += std::norm(z);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += std::norm(at(i, j));
    if (off <= 1e-32 * fro || off == 0.0) break;
    for (int pp = 0; pp < m; ++pp)
      for (int qq = pp + 1; qq < m; ++qq) {
        const cd apq = at(pp, qq);
        const double r = std::abs(apq);
        if (r == 0.0) continue;
        const double app = at(pp, pp).real(), aqq = at(qq, qq).real();
        const cd ph = apq / r;  // e^{i phi}
        const double tau = (aqq - app) / (2.0 * r);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        // J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (pp, qq)
        const cd Jpp = c, Jpq = sn, Jqp = -sn * std::conj(ph), Jqq = c * std::conj(ph);
        for (int k = 0; k < m; ++k) {  // A <- A J
          const cd akp = at(k, pp), akq = at(k, qq);
          at(k, pp) = akp * Jpp + akq * Jqp;
          at(k, qq) = akp * Jpq + akq * Jqq;
        }
        for (int k = 0; k < m; ++k) {  // A <- J^* A
          const cd apk = at(pp, k), aqk = at(qq, k);
          at(pp, k) = std::conj(Jpp) * apk + std::conj(Jqp) * aqk;
          at(qq, k) = std::conj(Jpq) * apk + std::conj(Jqq) * aqk;
        }
        at(pp, qq) = 0.0;
        at(qq, pp) = 0.0;
        at(pp, pp) = at(pp, pp).real();
        at(qq, qq) = at(qq, qq).real();
        for (int k = 0; k < m; ++k) {  // V <- V J
          const cd vkp = V[(size_t)k * m + pp], vkq = V[(size_t)k * m + qq];
          V[(size_t)k * m + pp] = vkp * Jpp + vkq * Jqp;
          V[(size_t)k * m + qq] = vkp * Jpq + vkq * Jqq;
        }
      }
  }
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return at(x, x).real() < at(y, y).real(); });
  for (int j = 0; j < m; ++j) {
    w[j] = at(order[j], order[j]).real();
    if (Vout)
      for (int i = 0; i < m; ++i) {
        const cd v = V[(size_t)i * m + order[j]];
        Vout[(size_t)i * m + j] = make_double2(v.real(), v.imag());
      }
  }
  return NSF_OK;
}

}  // namespace nsf

using namespace nsf;

extern "C" {

int nsf_hermitian_eig(int m, const nsf_c128* H, double* w, nsf_c128* V) {
  if (m < 1 || m > 512 || !H || !w) return set_error(nullptr, NSF_E_ARG, "bad argument to nsf_hermitian_eig");
  return hermitian_eig(m, reinterpret_cast<const double2*>(H), w, reinterpret_cast<double2*>(V));
}

int nsf_cg_solve(nsf_plan p, const nsf_c128* b, nsf_c128* x, double rtol, int maxit, int* iters,
                 double* relres) {
  if (!p || !b || !x) return set_error(p, NSF_E_ARG, "NULL argument");
  if ((const void*)b == (const void*)x) return set_error(p, NSF_E_ARG, "b and x must be distinct");
  if (!(rtol >= 0.0)) return set_error(p, NSF_E_ARG, "rtol must be >= 0");
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  if (p->medium_kind == kMedNfsep)
    return set_error(p, NSF_E_STATE, "an NFSEP medium has no positive definite A_r; use nsf_nfsep_solve");
  long long mv = 0;
  return cg_solve_dev(p, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), rtol, maxit,
                      iters, relres, &mv);
}

int nsf_cg_solve_noalloc(nsf_plan p, const nsf_c128* b, nsf_c128* x, double rtol, int maxit, int* iters,
                         double* relres) {
  if (!p || !b || !x) return set_error(p, NSF_E_ARG, "NULL argument");
  if ((const void*)b == (const void*)x) return set_error(p, NSF_E_ARG, "b and x must be distinct");
  if (p->geom.n > kNoAllocVoxels)
    return set_error(p, NSF_E_ARG, "nsf_cg_solve_noalloc takes grids of at most " +
                                       std::to_string(kNoAllocVoxels) + " voxels (this plan has " +
                                       std::to_string(p->geom.n) + ")");
  if (!(rtol >= 0.0)) return set_error(p, NSF_E_ARG, "rtol must be >= 0");
  if (p->medium_kind == kMedNone || !p->dev_ready) return set_error(p, NSF_E_STATE, "no medium set");
  if (p->medium_kind == kMedNfsep)
    return set_error(p, NSF_E_STATE, "an NFSEP medium has no positive definite A_r; use nsf_nfsep_solve");
  double2* cgv = nullptr;
  int rc = scratch_address(p, &cgv);
  if (rc) return rc;
  long long mv = 0;
  return cg_solve_dev(p, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), rtol, maxit,
                      iters, relres, &mv, cgv);
}

}  // extern "C"
