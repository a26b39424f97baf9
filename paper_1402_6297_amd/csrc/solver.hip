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

#include "nsf_internal.h"

namespace nsf {

// workspace for CG and the Lanczos step: r, p, q, w, z, b (six 4n vectors)
static int ensure_cg(nsf_plan p) {
  int rc = ensure_device(p);
  if (rc) return rc;
  if (!p->d_cg) NSF_HIP(p, hipMalloc(&p->d_cg, sizeof(double2) * 6 * 4 * (size_t)p->geom.n));
  return NSF_OK;
}

int ensure_basis(nsf_plan p, size_t vectors) {
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

int cg_solve_dev(nsf_plan p, const double2* b, double2* x, double rtol, int maxit, int* iters,
                 double* relres, long long* matvecs) {
  int rc = ensure_cg(p);
  if (rc) return rc;
  const long long len = 4 * p->geom.n;
  double2* r = p->d_cg;
  double2* pp = r + len;
  double2* q = pp + len;
  hipStream_t s = p->stream;
  CgState* st = p->d_state;
  const int nparts = reduce_parts_for(len);
  const int* skip = &st->done;
  NSF_HIP(p, launch_cg_init(b, x, r, pp, len, p->d_partial, st, rtol, maxit, s));
  // Fused iterations when the x axis has a two-level pass: the CG updates
  // ride in the first and last FFT pass of every A_r apply.
  const Geom& g = p->geom;
  const int xr = fast_x_rows(g);
  const bool fused = p->opt_fft_path != 1 && xr > 0 && ((long long)g.n2 * g.n3 + xr - 1) / xr <= 65536;
  CgFuse cgf{x, r, pp, q, st, reinterpret_cast<double*>(p->d_partial),
             reinterpret_cast<double*>(p->d_partial) + 65536};
  int chunk = 4;
  double rr_prev = -1.0;
  int it_prev = 0;
  for (;;) {
    for (int c = 0; c < chunk; ++c) {
      if (fused) {
        int np1 = 0, np5 = 0;
        NSF_HIP(p, launch_fast_cg_first(g, p->tabs, cgf, p->d_fields, skip, &np1, s));
        NSF_HIP(p, launch_cgf_check(cgf.part_in, np1, st, s));
        NSF_HIP(p, pass_yz(p, 1, +1, 6, p->d_fields, 0, 0, skip));
        NSF_HIP(p, pass_z_mid(p, p->d_fields, skip));
        NSF_HIP(p, pass_yz(p, 1, -1, 6, p->d_fields, 0, 0, skip));
        NSF_HIP(p, launch_fast_cg_last(g, p->tabs, cgf, p->d_fields, skip, &np5, s));
        NSF_HIP(p, launch_cgf_step(cgf.part_out, np5, st, s));
        continue;
      }
      rc = apply_Ar_dev(p, pp, q, skip);
      if (rc) return rc;
      NSF_HIP(p, launch_dot_partials(pp, q, len, p->d_partial, skip, s));
      NSF_HIP(p, launch_cg_alpha(p->d_partial, nparts, st, s));
      NSF_HIP(p, launch_cg_update(x, r, pp, q, len, p->d_partial, st, s));
      NSF_HIP(p, launch_cg_beta(p->d_partial, nparts, st, s));
      NSF_HIP(p, launch_cg_p(pp, r, len, st, s));
    }
    NSF_HIP(p, hipMemcpyAsync(p->h_state, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    NSF_HIP(p, hipStreamSynchronize(s));
    const CgState& h = *p->h_state;
    if (h.done) break;
    // Predict the iterations still needed from the observed rate.
    int next = 8;
    if (rr_prev > 0 && h.rr > 0 && h.rr < rr_prev && h.iter > it_prev) {
      const double rate = std::log(rr_prev / h.rr) / (h.iter - it_prev);
      const double need = std::log(h.rr / h.thresh) / rate;
      next = (int)std::ceil(need) + (fused ? 1 : 0);
    }
    rr_prev = h.rr;
    it_prev = h.iter;
    chunk = std::min(std::max(next, 1), 16);
  }
  const CgState& h = *p->h_state;
  if (iters) *iters = h.iter;
  if (relres) *relres = (h.bb > 0) ? std::sqrt(h.rr / h.bb) : 0.0;
  if (matvecs) *matvecs += h.iter;
  if (h.status == NSF_E_BREAKDOWN)
    return set_error(p, NSF_E_BREAKDOWN, "CG breakdown: p^* A_r p <= 0 or not finite");
  return h.status;
}

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

namespace {

// Host value of sum conj(x) y over len entries.
int dot_host(nsf_plan p, const double2* x, const double2* y, long long len, double2* out) {
  NSF_HIP(p, launch_dot_partials(x, y, len, p->d_partial, nullptr, p->stream));
  double2* dres = p->d_res;
  NSF_HIP(p, launch_reduce_partials(p->d_partial, reduce_parts_for(len), dres, p->stream));
  NSF_HIP(p, hipMemcpyAsync(out, dres, sizeof(double2), hipMemcpyDeviceToHost, p->stream));
  NSF_HIP(p, hipStreamSynchronize(p->stream));
  return NSF_OK;
}

}  // namespace

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
  long long mv = 0;
  return cg_solve_dev(p, reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(x), rtol, maxit,
                      iters, relres, &mv);
}

int nsf_eigs(nsf_plan p, int nev, double res_tol, double cg_rtol, int max_basis, int max_restarts,
             unsigned long long seed, double* omega_host, nsf_c128* Y_dev, double* resid_host,
             nsf_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p || !omega_host) return set_error(p, NSF_E_ARG, "NULL argument");
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  const long long n = p->geom.n, len = 4 * n;
  if (nev < 1 || nev > 256 || 2LL * nev >= len) return set_error(p, NSF_E_ARG, "nev out of range");
  if (!(res_tol > 0.0) || !(cg_rtol > 0.0)) return set_error(p, NSF_E_ARG, "tolerances must be > 0");
  int m = max_basis > 0 ? max_basis : std::max(3 * nev, nev + 8);
  if (m < nev + 2) m = nev + 2;
  if (m > 510) m = 510;
  if (m >= len) m = (int)len - 1;
  if (m < nev + 2) return set_error(p, NSF_E_ARG, "grid too small for nev");
  const int kkeep = std::min(m - 1, nev + (m - nev) / 2);
  if (max_restarts <= 0) max_restarts = 1000;

  int rc = ensure_cg(p);
  if (rc) return rc;
  rc = ensure_basis(p, (size_t)m + 1);
  if (rc) return rc;
  hipStream_t s = p->stream;
  double2* V = p->d_basis;
  double2* AV = V + (size_t)(m + 1) * len;
  double2* w = p->d_cg + 3 * len;
  double2* z = w + len;
  double2* bv = z + len;
  double2* dcoef = p->d_coef;
  rc = ensure_small(p, (size_t)m * m);
  if (rc) return rc;
  double2* dS = p->d_small;

  nsf_stats st{};
  const int ldh = m + 1;
  std::vector<double2> H((size_t)ldh * ldh, make_double2(0, 0));
  std::vector<double2> hc(m + 2);
  auto Hat = [&](int i, int j) -> double2& { return H[(size_t)i * ldh + j]; };
  int status = NSF_OK;
  std::vector<double> theta(m), eta(nev, INFINITY);
  std::vector<double2> S((size_t)m * m), Sk((size_t)m * kkeep);

  // Make V[j] the A_r-normalised copy of `w` (AV[j] from z) and fill row/col j
  // of H; leaves B_r V[j] in bv.
  auto admit = [&](int j, double nrm2) -> int {
    if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
      return set_error(p, NSF_E_BREAKDOWN, "A_r-norm of a new basis vector is not positive");
    const double sc = 1.0 / std::sqrt(nrm2);
    NSF_HIP(p, launch_scale_copy(w, V + (size_t)j * len, sc, 0.0, len, s));
    NSF_HIP(p, launch_scale_copy(z, AV + (size_t)j * len, sc, 0.0, len, s));
    NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, V + (size_t)j * len, bv, nullptr, s));
    NSF_HIP(p, launch_multi_dot(V, len, j + 1, bv, len, p->d_partial, dcoef, s));
    NSF_HIP(p, hipMemcpyAsync(hc.data(), dcoef, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, s));
    NSF_HIP(p, hipStreamSynchronize(s));
    for (int i = 0; i <= j; ++i) {  // H[i][j] = V_i^* B V_j
      Hat(i, j) = hc[i];
      Hat(j, i) = cconj(hc[i]);
    }
    Hat(j, j).y = 0.0;
    return NSF_OK;
  };
  // Orthogonalise (w, z) against V[0..nb) in the A_r inner product by
  // classical Gram-Schmidt; a second pass runs only when the first removed
  // more than half of the A-norm squared (the Daniel-Gragg-Kaufman-Stewart
  // test), which is when cancellation can leave w short of orthogonal.
  auto orthogonalise = [&](int nb, double* norm2, double* norm2_in) -> int {
    double2 before, after;
    int r2 = dot_host(p, w, z, len, &before);
    if (r2) return r2;
    *norm2_in = before.x;
    for (int pass = 0; pass < 2; ++pass) {
      NSF_HIP(p, launch_multi_dot(AV, len, nb, w, len, p->d_partial, dcoef, s));
      NSF_HIP(p, launch_multi_axpy(V, len, nb, dcoef, w, len, s));
      NSF_HIP(p, launch_multi_axpy(AV, len, nb, dcoef, z, len, s));
      r2 = dot_host(p, w, z, len, &after);
      if (r2) return r2;
      st.ortho_passes += 1;
      if (after.x > 0.5 * before.x) break;
      before = after;
    }
    *norm2 = after.x;
    return NSF_OK;
  };
  auto cleanup = [&](int code) { return code; };

  // Start vector: seeded complex normal, A_r-normalised.
  NSF_HIP(p, launch_randn(w, len, seed, s));
  rc = apply_Ar_dev(p, w, z, nullptr);
  if (rc) return cleanup(rc);
  st.matvecs += 1;
  {
    double2 n0;
    rc = dot_host(p, w, z, len, &n0);
    if (rc) return cleanup(rc);
    rc = admit(0, n0.x);
    if (rc) return cleanup(rc);
  }
  int nb = 1;
  bool converged = false;
  for (;;) {
    // Expand from the last basis vector: w = A_r^{-1} B_r V[nb-1].
    int it = 0;
    double rel = 0;
    rc = cg_solve_dev(p, bv, w, cg_rtol, 5000, &it, &rel, &st.matvecs);
    st.cg_solves += 1;
    st.cg_iters_total += it;
    if (rc < 0) return cleanup(rc);
    rc = apply_Ar_dev(p, w, z, nullptr);
    if (rc) return cleanup(rc);
    st.matvecs += 1;
    double nw = 0.0, nw_in = 0.0;
    rc = orthogonalise(nb, &nw, &nw_in);
    if (rc) return cleanup(rc);
    if (!(nw > 1e-20 * nw_in)) {
      // invariant subspace: continue from a fresh random direction
      NSF_HIP(p, launch_randn(w, len, seed + 7919ULL * (st.lanczos_steps + 1), s));
      rc = apply_Ar_dev(p, w, z, nullptr);
      if (rc) return cleanup(rc);
      st.matvecs += 1;
      rc = orthogonalise(nb, &nw, &nw_in);
      if (rc) return cleanup(rc);
    }
    rc = admit(nb, nw);
    if (rc) return cleanup(rc);
    nb += 1;
    st.lanczos_steps += 1;
    if (nb < m + 1) continue;

    // Rayleigh-Ritz on V[0..m): H_m S = S diag(theta).
    std::vector<double2> Hm((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Hm[(size_t)i * m + j] = Hat(i, j);
    std::vector<double> wv(m);
    hermitian_eig(m, Hm.data(), wv.data(), S.data());
    // descending theta: column c of Sk is eigenvector m-1-c
    for (int c = 0; c < kkeep; ++c) {
      theta[c] = wv[m - 1 - c];
      for (int i = 0; i < m; ++i) Sk[(size_t)c * m + i] = S[(size_t)i * m + (m - 1 - c)];
    }
    NSF_HIP(p, hipMemcpyAsync(dS, Sk.data(), sizeof(double2) * (size_t)m * kkeep, hipMemcpyHostToDevice, s));
    NSF_HIP(p, launch_rotate(V, len, m, kkeep, dS, len, s));
    NSF_HIP(p, launch_rotate(AV, len, m, kkeep, dS, len, s));
    // residuals of the wanted pairs
    bool all = true;
    double2* dres = p->d_res;
    for (int i = 0; i < nev; ++i) {
      double2 r2;
      NSF_HIP(p, launch_residual_norms(p->geom, p->tabs, V + (size_t)i * len, AV + (size_t)i * len, theta[i],
                                       p->d_partial, reinterpret_cast<double*>(dres), s));
      NSF_HIP(p, hipMemcpyAsync(&r2, dres, sizeof(double2), hipMemcpyDeviceToHost, s));
      NSF_HIP(p, hipStreamSynchronize(s));
      eta[i] = std::sqrt(r2.x) / (std::fabs(theta[i]) * std::sqrt(r2.y));
      if (!(theta[i] > 0.0) || !(eta[i] <= res_tol)) all = false;
    }
    // New projected matrix for [Ritz vectors, V[m]].
    std::vector<double2> row(kkeep);
    for (int c = 0; c < kkeep; ++c) {
      double2 acc = make_double2(0, 0);
      for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(Hat(m, i), Sk[(size_t)c * m + i]));
      row[c] = acc;
    }
    const double2 hmm = Hat(m, m);
    std::fill(H.begin(), H.end(), make_double2(0, 0));
    for (int c = 0; c < kkeep; ++c) {
      Hat(c, c) = make_double2(theta[c], 0);
      Hat(kkeep, c) = row[c];
      Hat(c, kkeep) = cconj(row[c]);
    }
    Hat(kkeep, kkeep) = hmm;
    NSF_HIP(p, hipMemcpyAsync(V + (size_t)kkeep * len, V + (size_t)m * len, sizeof(double2) * len,
                              hipMemcpyDeviceToDevice, s));
    NSF_HIP(p, hipMemcpyAsync(AV + (size_t)kkeep * len, AV + (size_t)m * len, sizeof(double2) * len,
                              hipMemcpyDeviceToDevice, s));
    nb = kkeep + 1;
    if (all) {
      converged = true;
      break;
    }
    st.restarts += 1;
    if (st.restarts > max_restarts) break;
  }
  // Results: omega ascending = 1 / theta descending.
  int nconv = 0;
  for (int i = 0; i < nev; ++i) {
    omega_host[i] = 1.0 / theta[i];
    if (resid_host) resid_host[i] = eta[i];
    if (eta[i] <= res_tol) ++nconv;
  }
  if (Y_dev)
    NSF_HIP(p, hipMemcpyAsync(Y_dev, V, sizeof(double2) * (size_t)nev * len, hipMemcpyDeviceToDevice, s));
  NSF_HIP(p, hipStreamSynchronize(s));
  status = converged ? NSF_OK : NSF_NOT_CONVERGED;
  st.converged = nconv;
  st.cg_iters_avg = st.cg_solves ? (double)st.cg_iters_total / st.cg_solves : 0.0;
  st.bytes_alg = 336.0 * (double)n * (double)st.matvecs;
  st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return cleanup(status);
}

}  // extern "C"
