// Plan construction, medium upload and the basis / A_r / B_r applies (host).
#include <chrono>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>

#include "nsf_internal.h"

namespace {
thread_local std::string g_plain_error;  // errors of calls without a plan

long double kPi = 3.141592653589793238462643383279502884L;

// exp(i 2 pi num / den) evaluated with the phase reduced in long double.
double2 unit_phase(long double num, long double den) {
  long double t = num / den;
  t -= floorl(t);
  const long double ang = 2.0L * kPi * t;
  return make_double2((double)cosl(ang), (double)sinl(ang));
}

bool factor_axis(int N, nsf::AxisPlan& ax) {
  ax.N = N;
  ax.nst = 0;
  int m = N;
  for (int r : {8, 4, 2, 3, 5}) {
    while (m % r == 0) {
      if (ax.nst >= nsf::kMaxStages) return false;
      ax.radix[ax.nst++] = r;
      m /= r;
    }
  }
  return m == 1;
}
}  // namespace

namespace nsf {

int set_error(nsf_plan p, int code, const std::string& msg) {
  if (p) p->last_error = msg;
  else g_plain_error = msg;
  return code;
}

bool debug_sync() {
  const char* e = std::getenv("NSF_SYNC_CHECK");
  return e && *e && *e != '0';
}

int hip_check(nsf_plan p, hipError_t e, const char* what) {
  std::string suffix;
  if (e == hipSuccess && debug_sync()) {  // NSF_SYNC_CHECK: surface errors of asynchronous work here
    e = hipDeviceSynchronize();
    suffix = " (device synchronisation after the call)";
  }
  if (e == hipSuccess) return NSF_OK;
  std::string msg = std::string(what) + ": " + hipGetErrorString(e) + suffix;
  const int code = (e == hipErrorOutOfMemory) ? NSF_E_NOMEM : NSF_E_HIP;
  return set_error(p, code, msg);
}

long long medium_voxel_bytes(nsf_plan p) {
  const int k = p->medium_kind;
  const int entries = k == kMedGeneral ? kGenEntries : k == kMedNfsep ? kFullEntries : 0;
  if (k == kMedNone) return 0;
  if (!entries) return (long long)sizeof(double2);  // (eps, gamma) per voxel
  if (p->palette > 0) return (long long)sizeof(unsigned short);
  return (long long)sizeof(double2) * entries;
}

void trace_solve(const char* call, nsf_plan p, int instance, int nev, int status, const nsf_stats& st,
                 const double* resid) {
  const char* dest = std::getenv("NSF_TRACE");
  if (!dest || !*dest || !std::strcmp(dest, "0")) return;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  FILE* f = (!std::strcmp(dest, "1") || !std::strcmp(dest, "stderr")) ? stderr : std::fopen(dest, "a");
  if (!f) return;
  double rmax = 0;
  for (int i = 0; resid && i < nev; ++i) rmax = std::max(rmax, resid[i]);
  const Geom& g = p->geom;
  std::fprintf(f,
               "{\"call\": \"%s\", \"instance\": %d, \"grid\": [%d, %d, %d], \"medium_kind\": %d, "
               "\"nev\": %d, \"status\": %d, \"converged\": %d, \"max_residual\": %.6e, "
               "\"matvecs\": %lld, \"inner_iters_total\": %lld, \"inner_solves\": %d, "
               "\"inner_iters_avg\": %.3f, \"steps\": %d, \"restarts\": %d, \"ortho_passes\": %d, "
               "\"ms_total\": %.3f, \"ms_inner\": %.3f, \"ms_orth\": %.3f, \"ms_restart\": %.3f, "
               "\"bytes_alg\": %.6e}\n",
               call, instance, g.n1, g.n2, g.n3, p->medium_kind, nev, status, st.converged, rmax, st.matvecs,
               st.cg_iters_total, st.cg_solves, st.cg_iters_avg, st.lanczos_steps, st.restarts, st.ortho_passes,
               st.ms_total, st.ms_cg, st.ms_orth, st.ms_restart, st.bytes_alg);
  if (f != stderr) std::fclose(f);
}

int ensure_device(nsf_plan p) {
  if (p->dev_ready) return NSF_OK;
  NSF_HIP(p, hipGetDevice(&p->device));
  const Geom& g = p->geom;
  const size_t ntab = (size_t)g.n1 + g.n2 + g.n3;
  NSF_HIP(p, hipMalloc(&p->d_tables, sizeof(double2) * 3 * ntab));
  std::vector<double2> all;
  all.reserve(3 * ntab);
  all.insert(all.end(), p->h_lam.begin(), p->h_lam.end());
  all.insert(all.end(), p->h_twist.begin(), p->h_twist.end());
  all.insert(all.end(), p->h_tw.begin(), p->h_tw.end());
  NSF_HIP(p, hipMemcpy(p->d_tables, all.data(), sizeof(double2) * all.size(), hipMemcpyHostToDevice));
  p->tabs.lam = p->d_tables;
  p->tabs.twist = p->d_tables + ntab;
  p->tabs.tw = p->d_tables + 2 * ntab;
  if (p->ws)
    p->d_fields = ws_part(p, 0);
  else
    NSF_HIP(p, hipMalloc(&p->d_fields, sizeof(double2) * 6 * (size_t)g.n));
  NSF_HIP(p, hipMalloc(&p->d_partial,
                       sizeof(double2) * (size_t)(kPartialSlots + kCoefSlots + kResSlots + kMidSlots)));
  p->d_coef = p->d_partial + kPartialSlots;
  p->d_res = p->d_coef + kCoefSlots;
  NSF_HIP(p, hipHostMalloc(&p->h_res, sizeof(double2) * kResSlots));
  NSF_HIP(p, hipMalloc(&p->d_state, sizeof(CgState)));
  NSF_HIP(p, hipHostMalloc(&p->h_state, sizeof(CgState)));
  NSF_HIP(p, hipMalloc(&p->d_flags, sizeof(int) * 16));
  NSF_HIP(p, hipMemset(p->d_flags, 0, sizeof(int) * 16));
  NSF_HIP(p, hipHostMalloc(&p->h_flags, sizeof(int) * 16));
  p->dev_ready = true;
  return NSF_OK;
}

MediumView medium_view(nsf_plan p) {
  MediumView m;
  m.kind = p->medium_kind;
  m.pa = p->pa;
  m.pb = p->pb;
  m.po = p->po;
  m.eg = p->d_medium;
  m.mg = p->d_mgen;
  m.mf = p->d_mfull;
  m.pidx = p->palette > 0 ? p->d_pidx : nullptr;
  m.ztiles = nullptr;
  m.nztiles = 0;
  m.xgroups = nullptr;
  m.nxgroups = 0;
  if ((m.kind == kMedChiral || m.kind == kMedPseudo) && p->d_ztiles) {
    auto log2_of = [](int P) {
      int k = 0;
      while (k < 5 && (1 << k) != P) ++k;
      return P > 0 ? k : 5;
    };
    const int kz = log2_of(fast_z_pair_cols(p->geom, m.kind, p->opt_mid_cols));
    const int ky = log2_of(fast_yz_cols(p->geom, 1));
    if (kz < 5 && ky < 5 && p->ztile_cnt[kz] >= 0 && p->xgrp_cnt[ky] >= 0) {
      m.ztiles = p->d_ztiles + p->ztile_off[kz];
      m.nztiles = p->ztile_cnt[kz];
      m.xgroups = p->d_ztiles + p->xgrp_off[ky];
      m.nxgroups = p->xgrp_cnt[ky];
    }
  }
  return m;
}

VacSkip vac_of(nsf_plan p) {
  VacSkip v;
  const Geom& g = p->geom;
  if (!p->opt_vacuum || p->opt_fft_path != 0 || !fast_axis(g.n1) || !fast_axis(g.n2) || !fast_axis(g.n3))
    return v;
  const MediumView m = medium_view(p);
  if (!m.ztiles) return v;
  v.on = true;
  v.zscale = 1.0 / (double)g.n3;
  v.yscale = 1.0 / (double)g.n2;
  v.pscale = 1.0 / (double)g.n1;
  v.ntiles = m.nztiles;
  v.nxg = m.nxgroups;
  return v;
}

hipError_t pass_x_inv(nsf_plan p, int part, const double2* y, double2* fld, const int* skip) {
  const Geom& g = p->geom;
  if (p->opt_fft_path == 2 && wave_axis(g.n1) && g.n <= (1LL << 32) / 96)
    return launch_wave_x_inv_synth(g, p->tabs, part, y, fld, skip, p->stream);
  if (p->opt_fft_path != 1 && fast_axis(g.n1))
    return launch_fast_x_inv_synth(g, p->tabs, part, y, fld, skip, p->stream);
  return launch_x_inv_synth(g, p->ax[0], p->tabs, part, y, fld, skip, p->stream);
}

hipError_t pass_yz(nsf_plan p, int axis, int dir, int nf, double2* fld, int post_twist, int pre_twist,
                   const int* skip, const VacSkip* vac) {
  const Geom& g = p->geom;
  if (vac && vac->on && axis == 1)  // (vac_of chose the two-level passes)
    return launch_fast_yz(g, p->tabs, axis, dir, nf, fld, post_twist, pre_twist, skip, p->stream, nullptr, 1,
                          medium_view(p).xgroups, vac->nxg, dir > 0 ? 1.0 : vac->yscale);
  if (p->opt_fft_path != 1 && fast_axis(axis == 1 ? g.n2 : g.n3))
    return launch_fast_yz(g, p->tabs, axis, dir, nf, fld, post_twist, pre_twist, skip, p->stream);
  return launch_yz_pass(g, p->ax[axis], p->tabs, axis, dir, nf, fld, post_twist, pre_twist, skip, p->stream);
}

int z_mid_pq_items(nsf_plan p) {
  const Geom& g = p->geom;
  if (p->opt_fft_path == 2 && wave_mid_ok(g) && !six_coupled(p->medium_kind)) return 0;
  if (p->opt_fft_path != 1 && fast_axis(g.n3)) return fast_z_mid_pq_items(g, p->medium_kind, p->opt_mid_cols);
  return 0;
}

hipError_t pass_z_mid(nsf_plan p, double2* fld, const int* skip, double* part_mid, int* np_mid,
                      const VacSkip* vac) {
  const Geom& g = p->geom;
  if (np_mid) *np_mid = 0;
  if (vac && vac->on)  // (vac_of chose the field-pair kernel of the two-level passes)
    return launch_fast_z_mid(g, p->tabs, medium_view(p), fld, p->opt_mid_cols, skip, p->stream, nullptr, 1,
                             part_mid, np_mid, vac->zscale, vac->ntiles);
  if (p->opt_fft_path == 2 && wave_mid_ok(g) && !six_coupled(p->medium_kind))
    return launch_wave_z_mid(g, p->tabs, medium_view(p), fld, skip, p->stream);
  if (p->opt_fft_path != 1 && fast_axis(g.n3))
    return launch_fast_z_mid(g, p->tabs, medium_view(p), fld, p->opt_mid_cols, skip, p->stream, nullptr, 1,
                             part_mid, np_mid);
  return launch_z_mid(g, p->ax[2], p->tabs, medium_view(p), fld, skip, p->stream);
}

hipError_t pass_x_fwd(nsf_plan p, int part, const double2* fld, double2* out, const int* skip, double pscale) {
  const Geom& g = p->geom;
  if (pscale != 1.0)  // after a vacuum-skipping z pass (two-level passes only)
    return launch_fast_x_fwd_proj(g, p->tabs, part, fld, out, skip, p->stream, nullptr, 1, pscale);
  if (p->opt_fft_path == 2 && wave_axis(g.n1) && g.n <= (1LL << 32) / 96)
    return launch_wave_x_fwd_proj(g, p->tabs, part, fld, out, skip, p->stream);
  if (p->opt_fft_path != 1 && fast_axis(g.n1))
    return launch_fast_x_fwd_proj(g, p->tabs, part, fld, out, skip, p->stream);
  return launch_x_fwd_proj(g, p->ax[0], p->tabs, part, fld, out, skip, p->stream);
}

// A_r u in five passes: [synthesis + inverse x] [inverse y]
// [inverse z, middle factor, forward z] [forward y] [forward x + projection].
int apply_Ar_dev(nsf_plan p, const double2* u, double2* out, const int* skip) {
  double2* F = p->d_fields;
  const VacSkip v = vac_of(p);
  NSF_HIP(p, pass_x_inv(p, kPartBoth, u, F, skip));
  NSF_HIP(p, pass_yz(p, 1, +1, 6, F, 0, 0, skip, &v));
  NSF_HIP(p, pass_z_mid(p, F, skip, nullptr, nullptr, &v));
  NSF_HIP(p, pass_yz(p, 1, -1, 6, F, 0, 0, skip, &v));
  NSF_HIP(p, pass_x_fwd(p, kPartBoth, F, out, skip, v.on ? v.pscale : 1.0));
  return NSF_OK;
}

}  // namespace nsf

using namespace nsf;

extern "C" {

const char* nsf_status_string(int status) {
  switch (status) {
    case NSF_OK: return "ok";
    case NSF_NOT_CONVERGED: return "not converged";
    case NSF_E_ARG: return "invalid argument";
    case NSF_E_KPOINT: return "Bloch vector makes Lambda_q singular";
    case NSF_E_BASIS: return "alpha, beta make Lambda_p rank deficient";
    case NSF_E_NOT_HHPD: return "medium violates mu > 0, Phi > 0, xi^* = zeta";
    case NSF_E_BREAKDOWN: return "CG breakdown (p^*Ap <= 0 or not finite)";
    case NSF_E_NOMEM: return "device out of memory";
    case NSF_E_HIP: return "HIP runtime error";
    case NSF_E_STATE: return "plan is missing required state";
    default: return "unknown status";
  }
}

int nsf_device_info(int device, nsf_device* out) {
  if (!out) return set_error(nullptr, NSF_E_ARG, "out is NULL");
  hipDeviceProp_t prop;
  NSF_HIP(nullptr, hipGetDeviceProperties(&prop, device));
  std::memset(out, 0, sizeof(*out));
  std::snprintf(out->name, sizeof(out->name), "%s", prop.gcnArchName);
  out->compute_units = prop.multiProcessorCount;
  out->clock_khz = prop.clockRate;
  out->memory_clock_khz = prop.memoryClockRate;
  out->memory_bus_bits = prop.memoryBusWidth;
  out->total_memory = (long long)prop.totalGlobalMem;
  out->l2_bytes = prop.l2CacheSize;
  out->lds_per_block = (int)prop.sharedMemPerBlock;
  out->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
  out->warp_size = prop.warpSize;
  return NSF_OK;
}

const char* nsf_last_error(nsf_plan plan) {
  return plan ? plan->last_error.c_str() : g_plain_error.c_str();
}

int nsf_plan_create(nsf_plan* out, int n1, int n2, int n3, double a, const double k[3], double alpha,
                    double beta, void* hip_stream) {
  if (!out) return set_error(nullptr, NSF_E_ARG, "out is NULL");
  *out = nullptr;
  if (!k) return set_error(nullptr, NSF_E_ARG, "k is NULL");
  const int dims[3] = {n1, n2, n3};
  AxisPlan ax[3];
  for (int l = 0; l < 3; ++l) {
    if (dims[l] < 2 || dims[l] > kMaxAxis || !factor_axis(dims[l], ax[l]))
      return set_error(nullptr, NSF_E_ARG,
                       "grid size " + std::to_string(dims[l]) +
                           " unsupported (2..512, prime factors 2, 3, 5 only)");
  }
  if (!(a > 0.0) || !std::isfinite(a)) return set_error(nullptr, NSF_E_ARG, "lattice constant a must be > 0");
  if (!std::isfinite(k[0]) || !std::isfinite(k[1]) || !std::isfinite(k[2]))
    return set_error(nullptr, NSF_E_ARG, "k must be finite");
  if (!std::isfinite(alpha) || !std::isfinite(beta) || alpha == 0.0 || beta == 0.0)
    return set_error(nullptr, NSF_E_ARG, "alpha and beta must be finite and nonzero (Lemma 2.2)");

  auto* p = new (std::nothrow) nsf_plan_s();
  if (!p) return set_error(nullptr, NSF_E_NOMEM, "host allocation failed");
  p->geom.n1 = n1;
  p->geom.n2 = n2;
  p->geom.n3 = n3;
  p->geom.n = (long long)n1 * n2 * n3;
  p->geom.alpha = alpha;
  p->geom.beta = beta;
  p->a = a;
  for (int l = 0; l < 3; ++l) {
    p->k[l] = k[l];
    p->delta[l] = a / dims[l];
    p->ax[l] = ax[l];
  }
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);

  // Per-axis tables.  lambda_l(i) = (exp(i 2 pi (i + k_l a)/n_l) - 1)/delta_l
  // (Thm 2.1), evaluated as (-2 sin^2(t/2) + i sin t)/delta_l so that small
  // phases keep their relative accuracy; twist d_l(j) = exp(i 2 pi k_l a j/n_l)
  // (D_{a,m}); FFT roots exp(2 pi i m / n_l).
  double smin2 = 0, smax2 = 0;
  for (int l = 0; l < 3; ++l) {
    const int m = dims[l];
    double amin = 1e300, amax = 0;
    for (int i = 0; i < m; ++i) {
      long double t = ((long double)i + (long double)k[l] * (long double)a) / (long double)m;
      t -= floorl(t);
      const long double ang = 2.0L * kPi * t;
      const long double sh = sinl(0.5L * ang);
      const double re = (double)(-2.0L * sh * sh / (long double)p->delta[l]);
      const double im = (double)(sinl(ang) / (long double)p->delta[l]);
      p->h_lam.push_back(make_double2(re, im));
      const double a2 = re * re + im * im;
      amin = std::min(amin, a2);
      amax = std::max(amax, a2);
    }
    smin2 += amin;
    smax2 += amax;
  }
  for (int l = 0; l < 3; ++l)
    for (int j = 0; j < dims[l]; ++j)
      p->h_twist.push_back(unit_phase((long double)k[l] * (long double)a * j, (long double)dims[l]));
  for (int l = 0; l < 3; ++l)
    for (int j = 0; j < dims[l]; ++j) p->h_tw.push_back(unit_phase(j, dims[l]));
  p->sigma_min = std::sqrt(smin2);
  p->sigma_max = std::sqrt(smax2);
  // Lemma 2.2 (a): Lambda_q > 0.  sigma^2 is a sum of per-axis terms, so its
  // minimum is the sum of the per-axis minima.
  if (!(p->sigma_min > 1e-12 * p->sigma_max)) {
    delete p;
    return set_error(nullptr, NSF_E_KPOINT, "Lambda_q is singular: every k_l * a is an integer");
  }
  // Lemma 2.2 (b): every column p_f = a x lambda_f of Lambda_p nonzero.
  {
    const double2* l1 = p->h_lam.data();
    const double2* l2 = l1 + n1;
    const double2* l3 = l2 + n2;
    double worst = 1e300;
    for (int i3 = 0; i3 < n3; ++i3)
      for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1) {
          const double2 p1 = csub(cscale(l3[i3], beta), l2[i2]);
          const double2 p2 = csub(l1[i1], cscale(l3[i3], alpha));
          const double2 p3 = csub(cscale(l2[i2], alpha), cscale(l1[i1], beta));
          const double s2 = cabs2(l1[i1]) + cabs2(l2[i2]) + cabs2(l3[i3]);
          const double r = (cabs2(p1) + cabs2(p2) + cabs2(p3)) / ((alpha * alpha + beta * beta + 1.0) * s2);
          worst = std::min(worst, r);
        }
    if (!(worst > 1e-24)) {
      delete p;
      return set_error(nullptr, NSF_E_BASIS, "Lambda_p has a (near) zero column for these alpha, beta");
    }
  }
  *out = p;
  return NSF_OK;
}

void nsf_plan_destroy(nsf_plan p) {
  if (!p) return;
  if (p->dev_ready) {
    hipStreamSynchronize(p->stream);
    hipFree(p->d_tables);
    if (!p->ws) hipFree(p->d_fields);
    hipFree(p->d_partial);
    hipFree(p->d_state);
    hipHostFree(p->h_state);
    hipFree(p->d_flags);
    hipHostFree(p->h_flags);
    hipHostFree(p->h_res);
    if (p->d_medium) hipFree(p->d_medium);
    if (p->d_mgen) hipFree(p->d_mgen);
    if (p->d_mfull) hipFree(p->d_mfull);
    if (p->d_pidx) hipFree(p->d_pidx);
    if (p->d_cg && !p->ws) hipFree(p->d_cg);
    if (p->d_ring) hipFree(p->d_ring);
    if (p->d_ztiles) hipFree(p->d_ztiles);
    if (p->d_basis && !p->ws) hipFree(p->d_basis);
    if (p->d_small && !p->ws) hipFree(p->d_small);
  }
  delete p;
}

int nsf_plan_workspace_size(nsf_plan p, int nev, int max_basis, size_t* bytes) {
  if (!p || !bytes) return set_error(p, NSF_E_ARG, "NULL argument");
  const long long len = 4 * p->geom.n;
  if (nev < 1 || nev > 256 || 2LL * nev >= len) return set_error(p, NSF_E_ARG, "nev out of range");
  int m = max_basis > 0 ? max_basis : std::max(3 * nev, nev + 8);
  if (m < nev + 2) m = nev + 2;
  if (m > 510) m = 510;
  if (m >= len) m = (int)len - 1;
  *bytes = workspace_bytes(p->geom.n, m);
  return NSF_OK;
}

int nsf_plan_set_workspace(nsf_plan p, void* dev_ptr, size_t bytes) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  const long long n = p->geom.n;
  if (dev_ptr && bytes < workspace_bytes(n, 1))
    return set_error(p, NSF_E_ARG, "workspace smaller than the fields, CG vectors and a 2-vector basis");
  if (p->dev_ready) NSF_HIP(p, hipStreamSynchronize(p->stream));
  // release what the plan allocated itself (or drop the old workspace's parts)
  if (!p->ws) {
    if (p->d_fields) NSF_HIP(p, hipFree(p->d_fields));
    if (p->d_cg) NSF_HIP(p, hipFree(p->d_cg));
    if (p->d_basis) NSF_HIP(p, hipFree(p->d_basis));
    if (p->d_small) NSF_HIP(p, hipFree(p->d_small));
  }
  if (p->d_ring) NSF_HIP(p, hipFree(p->d_ring));  // the plan's own memory in either case
  p->d_ring = nullptr;
  p->d_fields = p->d_cg = p->d_basis = p->d_small = nullptr;
  p->basis_vectors = 0;
  p->small_cap = 0;
  p->ws = static_cast<char*>(dev_ptr);
  p->ws_bytes = dev_ptr ? bytes : 0;
  if (p->dev_ready) {
    if (p->ws)
      p->d_fields = ws_part(p, 0);
    else
      NSF_HIP(p, hipMalloc(&p->d_fields, sizeof(double2) * 6 * (size_t)n));
  }
  return NSF_OK;
}

int nsf_plan_set_option(nsf_plan p, int option, int value) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  switch (option) {
    case NSF_OPT_FFT_PATH:
      if (value < 0 || value > 2) return set_error(p, NSF_E_ARG, "NSF_OPT_FFT_PATH takes 0, 1 or 2");
      p->opt_fft_path = value;
      return NSF_OK;
    case NSF_OPT_MID_COLS:
      if (value < 1 || value > 16 || (value & (value - 1))) return set_error(p, NSF_E_ARG, "NSF_OPT_MID_COLS takes 1, 2, 4, 8 or 16");
      p->opt_mid_cols = value;
      return NSF_OK;
    case NSF_OPT_X_ROWS:
      if (value != 1 && value != 2 && value != 4) return set_error(p, NSF_E_ARG, "NSF_OPT_X_ROWS takes 1, 2 or 4");
      p->geom.x_rows = value;
      return NSF_OK;
    case NSF_OPT_YZ_COLS:
      if (value < 1 || value > 16 || (value & (value - 1)))
        return set_error(p, NSF_E_ARG, "NSF_OPT_YZ_COLS takes 1, 2, 4, 8 or 16");
      p->geom.yz_cols = value;
      return NSF_OK;
    case NSF_OPT_MID_PAIRS:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_MID_PAIRS takes 0 or 1");
      p->geom.mid_pairs = value;
      return NSF_OK;
    case NSF_OPT_CG_START:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_CG_START takes 0 or 1");
      p->opt_cg_start = value;
      return NSF_OK;
    case NSF_OPT_VERIFY:
      if (value < 0 || value > 16) return set_error(p, NSF_E_ARG, "NSF_OPT_VERIFY takes 0..16");
      p->opt_verify = value;
      return NSF_OK;
    case NSF_OPT_MEDIUM_PALETTE:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_MEDIUM_PALETTE takes 0 or 1");
      p->opt_palette = value;
      return NSF_OK;
    case NSF_OPT_GMRES_RESTART:
      if (value < 4 || value > 500) return set_error(p, NSF_E_ARG, "NSF_OPT_GMRES_RESTART takes 4..500");
      p->opt_gmres_restart = value;
      return NSF_OK;
    case NSF_OPT_ORTHO_GATE:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_ORTHO_GATE takes 0 or 1");
      p->opt_ortho_gate = value;
      return NSF_OK;
    case NSF_OPT_CG_RELAX:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_CG_RELAX takes 0 or 1");
      p->opt_cg_relax = value;
      return NSF_OK;
    case NSF_OPT_WARM_CHAIN:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_WARM_CHAIN takes 0 or 1");
      p->opt_warm_chain = value;
      return NSF_OK;
    case NSF_OPT_CG_RING:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_CG_RING takes 0 or 1");
      p->opt_cg_ring = value;
      return NSF_OK;
    case NSF_OPT_VACUUM:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_VACUUM takes 0 or 1");
      p->opt_vacuum = value;
      return NSF_OK;
    case NSF_OPT_CG_GRAPH:
      if (value < 0 || value > 1) return set_error(p, NSF_E_ARG, "NSF_OPT_CG_GRAPH takes 0 or 1");
      p->opt_cg_graph = value;
      return NSF_OK;
    default:
      return set_error(p, NSF_E_ARG, "unknown option");
  }
}

int nsf_plan_medium_info(nsf_plan p, int* palette, long long* voxel_bytes) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  const int k = p->medium_kind;
  const int entries = k == kMedGeneral ? kGenEntries : k == kMedNfsep ? kFullEntries : 0;
  if (palette) *palette = entries ? p->palette : 0;
  if (voxel_bytes) *voxel_bytes = medium_voxel_bytes(p);
  return NSF_OK;
}

int nsf_plan_query(nsf_plan p, long long* n, int* medium_kind, double* sigma_min, double* sigma_max) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (n) *n = p->geom.n;
  if (medium_kind) *medium_kind = p->medium_kind;
  if (sigma_min) *sigma_min = p->sigma_min;
  if (sigma_max) *sigma_max = p->sigma_max;
  return NSF_OK;
}

}  // extern "C"

namespace {

// Host validation of (eps, gamma) against the assumption of Sec. 4.1 for the
// compact media: mu = I > 0, xi^* = zeta holds by construction, and Phi > 0
// (chiral: eps - gamma^2; pseudochiral: eps - gamma^2 and eps).
int validate_eg(nsf_plan p, const double* eps, const double* gam, long long n) {
  for (long long g = 0; g < n; ++g) {
    const double e = eps[g], c = gam[g];
    if (!std::isfinite(e) || !std::isfinite(c))
      return set_error(p, NSF_E_ARG, "medium has a non-finite value at voxel " + std::to_string(g));
    if (!(e - c * c > 0.0) || !(e > 0.0))
      return set_error(p, NSF_E_NOT_HHPD,
                       "Phi = eps - gamma^2 is not positive at voxel " + std::to_string(g));
  }
  return NSF_OK;
}

int set_medium(nsf_plan p, int kind, int pa, int pb, const double* eps, const double* gam,
               int on_device) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (!eps || !gam) return set_error(p, NSF_E_ARG, "eps or gamma is NULL");
  const long long n = p->geom.n;
  std::vector<double> he, hg;
  const double* e = eps;
  const double* c = gam;
  if (on_device) {
    int rc = ensure_device(p);
    if (rc) return rc;
    he.resize(n);
    hg.resize(n);
    NSF_HIP(p, hipMemcpyAsync(he.data(), eps, sizeof(double) * n, hipMemcpyDeviceToHost, p->stream));
    NSF_HIP(p, hipMemcpyAsync(hg.data(), gam, sizeof(double) * n, hipMemcpyDeviceToHost, p->stream));
    NSF_HIP(p, hipStreamSynchronize(p->stream));
    e = he.data();
    c = hg.data();
  }
  int rc = validate_eg(p, e, c, n);
  if (rc) return rc;
  rc = ensure_device(p);
  if (rc) return rc;
  std::vector<double2> packed(n);
  for (long long g = 0; g < n; ++g) packed[g] = make_double2(e[g], c[g]);
  if (!p->d_medium) NSF_HIP(p, hipMalloc(&p->d_medium, sizeof(double2) * n));
  NSF_HIP(p, hipMemcpyAsync(p->d_medium, packed.data(), sizeof(double2) * n, hipMemcpyHostToDevice,
                            p->stream));
  // Tiles of the field-pair z pass (P columns x .. x + P - 1 of one y) that hold
  // a voxel other than vacuum (eps 1, gamma 0), for P = 1, 2, 4, 8, 16; a
  // vacuum-skipping apply transforms only these.
  {
    const int n1 = p->geom.n1, n2 = p->geom.n2, n3 = p->geom.n3;
    std::vector<unsigned char> col((size_t)n1 * n2, 0);
    for (long long z = 0; z < n3; ++z)
      for (long long yx = 0; yx < (long long)n1 * n2; ++yx) {
        const long long v = z * n1 * n2 + yx;
        if (e[v] != 1.0 || c[v] != 0.0) col[yx] = 1;
      }
    std::vector<int> list;
    for (int k = 0; k < 5; ++k) {
      const int P = 1 << k;
      p->ztile_off[k] = (int)list.size();
      p->ztile_cnt[k] = -1;
      if (n1 % P) continue;
      const int groups = n1 / P;
      for (int y = 0; y < n2; ++y)
        for (int gx = 0; gx < groups; ++gx) {
          bool any = false;
          for (int j = 0; j < P && !any; ++j) any = col[(size_t)y * n1 + gx * P + j] != 0;
          if (any) list.push_back(gx + groups * y);
        }
      p->ztile_cnt[k] = (int)list.size() - p->ztile_off[k];
    }
    // groups of P consecutive x (the y pass's pencils) holding such a voxel
    std::vector<unsigned char> xact(n1, 0);
    for (int y = 0; y < n2; ++y)
      for (int x = 0; x < n1; ++x)
        if (col[(size_t)y * n1 + x]) xact[x] = 1;
    for (int k = 0; k < 5; ++k) {
      const int P = 1 << k;
      p->xgrp_off[k] = (int)list.size();
      p->xgrp_cnt[k] = -1;
      if (n1 % P) continue;
      for (int gx = 0; gx < n1 / P; ++gx) {
        bool any = false;
        for (int j = 0; j < P && !any; ++j) any = xact[gx * P + j] != 0;
        if (any) list.push_back(gx);
      }
      p->xgrp_cnt[k] = (int)list.size() - p->xgrp_off[k];
    }
    const size_t need = std::max<size_t>(list.size(), 1);
    if (need > p->ztile_cap) {
      if (p->d_ztiles) NSF_HIP(p, hipFree(p->d_ztiles));
      p->d_ztiles = nullptr;
      p->ztile_cap = 0;
      NSF_HIP(p, hipMalloc(&p->d_ztiles, sizeof(int) * need));
      p->ztile_cap = need;
    }
    if (!list.empty())
      NSF_HIP(p, hipMemcpyAsync(p->d_ztiles, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice,
                                p->stream));
  }
  NSF_HIP(p, hipStreamSynchronize(p->stream));
  p->medium_kind = kind;
  p->pa = pa;
  p->pb = pb;
  p->po = 3 - pa - pb;
  return NSF_OK;
}

// ---- general media: 3 x 3 complex blocks per voxel
typedef std::complex<double> cplx;
struct M3 {
  cplx a[3][3];
};

M3 load3(const double2* src) {
  M3 m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = cplx(src[3 * i + j].x, src[3 * i + j].y);
  return m;
}
M3 mul3(const M3& x, const M3& y) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) s += x.a[i][k] * y.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}
M3 adj3(const M3& x) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = std::conj(x.a[j][i]);
  return r;
}
double absmax3(const M3& x) {
  double s = 0;
  for (auto& row : x.a)
    for (auto& v : row) s = std::max(s, std::abs(v));
  return s;
}
double herm_err3(const M3& x) {
  double s = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s = std::max(s, std::abs(x.a[i][j] - std::conj(x.a[j][i])));
  return s;
}
// Inverse of a Hermitian positive definite 3 x 3 block by Cholesky; false if
// the (Hermitian part of the) block is not positive definite.
bool hpd_inverse3(const M3& x, M3& inv) {
  cplx L[3][3] = {};
  for (int j = 0; j < 3; ++j) {
    double d = 0.5 * (x.a[j][j].real() + x.a[j][j].real());
    for (int k = 0; k < j; ++k) d -= std::norm(L[j][k]);
    if (!(d > 0.0)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 3; ++i) {
      cplx s = 0.5 * (x.a[i][j] + std::conj(x.a[j][i]));
      for (int k = 0; k < j; ++k) s -= L[i][k] * std::conj(L[j][k]);
      L[i][j] = s / L[j][j].real();
    }
  }
  // inverse of L, then inv = L^-* L^-1
  cplx Li[3][3] = {};
  for (int i = 0; i < 3; ++i) {
    Li[i][i] = 1.0 / L[i][i].real();
    for (int j = 0; j < i; ++j) {
      cplx s = 0;
      for (int k = j; k < i; ++k) s -= L[i][k] * Li[k][j];
      Li[i][j] = s / L[i][i].real();
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = std::max(i, j); k < 3; ++k) s += std::conj(Li[k][i]) * Li[k][j];
      inv.a[i][j] = s;
    }
  return true;
}

// Upload per-voxel factors (E complex values per voxel) to *dst: as a palette of
// the distinct voxel factors plus a 16-bit index per voxel when there are at
// most kPaletteMax of them (bitwise equality), else per voxel.  *dst has room
// for n E values once allocated.
int upload_factors(nsf_plan p, const std::vector<double2>& M, int E, double2** dst) {
  const long long n = p->geom.n;
  std::vector<double2> pal;
  std::vector<unsigned short> idx((size_t)n);
  std::unordered_map<unsigned long long, std::vector<int>> seen;
  bool fits = p->opt_palette != 0;
  for (long long g = 0; g < n && fits; ++g) {
    const double2* v = M.data() + (size_t)g * E;
    unsigned long long h = 1469598103934665603ULL;  // FNV-1a over the bytes
    const unsigned char* b = reinterpret_cast<const unsigned char*>(v);
    for (size_t i = 0; i < sizeof(double2) * E; ++i) h = (h ^ b[i]) * 1099511628211ULL;
    int found = -1;
    auto& cand = seen[h];
    for (int c : cand)
      if (!std::memcmp(pal.data() + (size_t)c * E, v, sizeof(double2) * E)) {
        found = c;
        break;
      }
    if (found < 0) {
      found = (int)(pal.size() / E);
      if (found >= kPaletteMax) {
        fits = false;
        break;
      }
      pal.insert(pal.end(), v, v + E);
      cand.push_back(found);
    }
    idx[(size_t)g] = (unsigned short)found;
  }
  if (!*dst) NSF_HIP(p, hipMalloc(dst, sizeof(double2) * (size_t)n * E));
  if (fits) {
    if (!p->d_pidx) NSF_HIP(p, hipMalloc(&p->d_pidx, sizeof(unsigned short) * (size_t)n));
    NSF_HIP(p, hipMemcpyAsync(*dst, pal.data(), sizeof(double2) * pal.size(), hipMemcpyHostToDevice, p->stream));
    NSF_HIP(p, hipMemcpyAsync(p->d_pidx, idx.data(), sizeof(unsigned short) * idx.size(), hipMemcpyHostToDevice,
                              p->stream));
    p->palette = (int)(pal.size() / E);
  } else {
    NSF_HIP(p, hipMemcpyAsync(*dst, M.data(), sizeof(double2) * M.size(), hipMemcpyHostToDevice, p->stream));
    p->palette = 0;
  }
  NSF_HIP(p, hipStreamSynchronize(p->stream));
  return NSF_OK;
}

// Inverse of a complex 6 x 6 matrix by Gauss-Jordan elimination with partial
// pivoting.  False when a pivot falls to tiny * max |entry| (numerically singular).
bool inverse6(cplx a[6][6], cplx inv[6][6], double tiny) {
  double amax = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      amax = std::max(amax, std::abs(a[i][j]));
      inv[i][j] = i == j ? 1.0 : 0.0;
    }
  if (!(amax > 0)) return false;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (std::abs(a[r][c]) > std::abs(a[piv][c])) piv = r;
    if (!(std::abs(a[piv][c]) > tiny * amax)) return false;
    if (piv != c)
      for (int j = 0; j < 6; ++j) {
        std::swap(a[c][j], a[piv][j]);
        std::swap(inv[c][j], inv[piv][j]);
      }
    const cplx d = 1.0 / a[c][c];
    for (int j = 0; j < 6; ++j) {
      a[c][j] *= d;
      inv[c][j] *= d;
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const cplx f = a[r][c];
      if (f == 0.0) continue;
      for (int j = 0; j < 6; ++j) {
        a[r][j] -= f * a[c][j];
        inv[r][j] -= f * inv[c][j];
      }
    }
  }
  return true;
}

}  // namespace

extern "C" {

int nsf_set_medium_nfsep(nsf_plan p, const nsf_c128* eps, const nsf_c128* mu, const nsf_c128* xi,
                         const nsf_c128* zeta, int on_device) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (!eps || !mu || !xi || !zeta) return set_error(p, NSF_E_ARG, "a tensor field is NULL");
  const long long n = p->geom.n;
  const size_t cnt = 9 * (size_t)n;
  std::vector<double2> h[4];
  const double2* src[4] = {reinterpret_cast<const double2*>(eps), reinterpret_cast<const double2*>(mu),
                           reinterpret_cast<const double2*>(xi), reinterpret_cast<const double2*>(zeta)};
  if (on_device) {
    const int rc = ensure_device(p);
    if (rc) return rc;
    for (int f = 0; f < 4; ++f) {
      h[f].resize(cnt);
      NSF_HIP(p, hipMemcpyAsync(h[f].data(), src[f], sizeof(double2) * cnt, hipMemcpyDeviceToHost, p->stream));
      src[f] = h[f].data();
    }
    NSF_HIP(p, hipStreamSynchronize(p->stream));
  }
  const cplx I(0.0, 1.0);
  std::vector<double2> N((size_t)n * kFullEntries);
  for (long long g = 0; g < n; ++g) {
    const M3 E = load3(src[0] + 9 * g), U = load3(src[1] + 9 * g), X = load3(src[2] + 9 * g),
             Z = load3(src[3] + 9 * g);
    for (const M3* t : {&E, &U, &X, &Z})
      for (auto& row : t->a)
        for (auto& v : row)
          if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
            return set_error(p, NSF_E_ARG, "medium has a non-finite value at voxel " + std::to_string(g));
    // B = i [[zeta, mu], [-eps, -xi]] (Sec. 3)
    cplx B[6][6], Bi[6][6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        B[i][j] = I * Z.a[i][j];
        B[i][3 + j] = I * U.a[i][j];
        B[3 + i][j] = -I * E.a[i][j];
        B[3 + i][3 + j] = -I * X.a[i][j];
      }
    if (!inverse6(B, Bi, 1e-13))
      return set_error(p, NSF_E_ARG, "B = i[[zeta, mu], [-eps, -xi]] is singular at voxel " + std::to_string(g));
    // N = i J B^{-1}: rows 0..2 = i (B^{-1}) rows 3..5, rows 3..5 = -i (B^{-1}) rows 0..2
    double2* out = N.data() + (size_t)g * kFullEntries;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        const cplx v = i < 3 ? I * Bi[3 + i][j] : -I * Bi[i - 3][j];
        out[6 * i + j] = make_double2(v.real(), v.imag());
      }
  }
  int rc = ensure_device(p);
  if (rc) return rc;
  if ((rc = upload_factors(p, N, kFullEntries, &p->d_mfull))) return rc;
  p->medium_kind = kMedNfsep;
  return NSF_OK;
}

int nsf_set_medium_tensor(nsf_plan p, const nsf_c128* eps, const nsf_c128* mu, const nsf_c128* xi,
                          const nsf_c128* zeta, int on_device) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (!eps || !mu || !xi || !zeta) return set_error(p, NSF_E_ARG, "a tensor field is NULL");
  const long long n = p->geom.n;
  const size_t cnt = 9 * (size_t)n;
  std::vector<double2> h[4];
  const double2* src[4] = {reinterpret_cast<const double2*>(eps), reinterpret_cast<const double2*>(mu),
                           reinterpret_cast<const double2*>(xi), reinterpret_cast<const double2*>(zeta)};
  if (on_device) {
    const int rc = ensure_device(p);
    if (rc) return rc;
    for (int f = 0; f < 4; ++f) {
      h[f].resize(cnt);
      NSF_HIP(p, hipMemcpyAsync(h[f].data(), src[f], sizeof(double2) * cnt, hipMemcpyDeviceToHost, p->stream));
      src[f] = h[f].data();
    }
    NSF_HIP(p, hipStreamSynchronize(p->stream));
  }
  std::vector<double2> M((size_t)n * kGenEntries);
  for (long long g = 0; g < n; ++g) {
    const M3 E = load3(src[0] + 9 * g), U = load3(src[1] + 9 * g), X = load3(src[2] + 9 * g),
             Z = load3(src[3] + 9 * g);
    const double scale = std::max({absmax3(E), absmax3(U), absmax3(X), absmax3(Z), 1.0});
    for (const M3* t : {&E, &U, &X, &Z})
      for (auto& row : t->a)
        for (auto& v : row)
          if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
            return set_error(p, NSF_E_ARG, "medium has a non-finite value at voxel " + std::to_string(g));
    const std::string at = " at voxel " + std::to_string(g);
    if (herm_err3(U) > 1e-14 * scale) return set_error(p, NSF_E_NOT_HHPD, "mu is not Hermitian" + at);
    if (herm_err3(E) > 1e-14 * scale) return set_error(p, NSF_E_NOT_HHPD, "eps is not Hermitian" + at);
    const M3 Xa = adj3(X);
    double dz = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) dz = std::max(dz, std::abs(Xa.a[i][j] - Z.a[i][j]));
    if (dz > 1e-14 * scale) return set_error(p, NSF_E_NOT_HHPD, "zeta differs from xi^*" + at);
    M3 Ui, Fi;
    if (!hpd_inverse3(U, Ui)) return set_error(p, NSF_E_NOT_HHPD, "mu is not positive definite" + at);
    const M3 XUi = mul3(X, Ui);                 // xi mu^-1
    const M3 UiZ = adj3(XUi);                   // mu^-1 zeta (zeta = xi^*, mu Hermitian)
    M3 Phi = mul3(XUi, Z);                      // xi mu^-1 zeta
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Phi.a[i][j] = E.a[i][j] - Phi.a[i][j];
    if (!hpd_inverse3(Phi, Fi))
      return set_error(p, NSF_E_NOT_HHPD, "Phi = eps - xi mu^-1 zeta is not positive definite" + at);
    const M3 M12 = mul3(UiZ, Fi);               // mu^-1 zeta Phi^-1
    M3 M11 = mul3(M12, XUi);                    // mu^-1 zeta Phi^-1 xi mu^-1
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M11.a[i][j] += Ui.a[i][j];
    // upper triangle of [[M11, M12], [M12^*, Fi]], row by row
    auto ent = [&](int i, int j) -> cplx {
      if (i < 3 && j < 3) return M11.a[i][j];
      if (i < 3) return M12.a[i][j - 3];
      return Fi.a[i - 3][j - 3];
    };
    double2* out = M.data() + (size_t)g * kGenEntries;
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j, ++k) {
        const cplx v = ent(i, j);
        out[k] = make_double2(v.real(), v.imag());
      }
  }
  int rc = ensure_device(p);
  if (rc) return rc;
  if ((rc = upload_factors(p, M, kGenEntries, &p->d_mgen))) return rc;
  p->medium_kind = kMedGeneral;
  return NSF_OK;
}

int nsf_set_medium_chiral(nsf_plan p, const double* eps, const double* gamma, int on_device) {
  return set_medium(p, kMedChiral, 0, 1, eps, gamma, on_device);
}

int nsf_set_medium_pseudochiral(nsf_plan p, int axis_a, int axis_b, const double* eps,
                                const double* gamma, int on_device) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (axis_a < 0 || axis_a > 2 || axis_b < 0 || axis_b > 2 || axis_a == axis_b)
    return set_error(p, NSF_E_ARG, "pseudochiral axes must be two distinct values in {0,1,2}");
  return set_medium(p, kMedPseudo, std::min(axis_a, axis_b), std::max(axis_a, axis_b), eps, gamma,
                    on_device);
}

int nsf_apply_Pr(nsf_plan p, const nsf_c128* y2n, nsf_c128* x3n) {
  if (!p || !y2n || !x3n) return set_error(p, NSF_E_ARG, "NULL argument");
  int rc = ensure_device(p);
  if (rc) return rc;
  auto* x = reinterpret_cast<double2*>(x3n);
  NSF_HIP(p, pass_x_inv(p, kPartP, reinterpret_cast<const double2*>(y2n), x, nullptr));
  NSF_HIP(p, pass_yz(p, 1, +1, 3, x, 0, 0, nullptr));
  NSF_HIP(p, pass_yz(p, 2, +1, 3, x, 1, 0, nullptr));
  return NSF_OK;
}

int nsf_apply_Qr(nsf_plan p, const nsf_c128* y2n, nsf_c128* x3n) {
  if (!p || !y2n || !x3n) return set_error(p, NSF_E_ARG, "NULL argument");
  int rc = ensure_device(p);
  if (rc) return rc;
  auto* x = reinterpret_cast<double2*>(x3n);
  NSF_HIP(p, pass_x_inv(p, kPartQ, reinterpret_cast<const double2*>(y2n), x, nullptr));
  NSF_HIP(p, pass_yz(p, 1, +1, 3, x, 0, 0, nullptr));
  NSF_HIP(p, pass_yz(p, 2, +1, 3, x, 1, 0, nullptr));
  return NSF_OK;
}

static int apply_adjoint(nsf_plan p, int part, const nsf_c128* x3n, nsf_c128* y2n) {
  if (!p || !x3n || !y2n) return set_error(p, NSF_E_ARG, "NULL argument");
  int rc = ensure_device(p);
  if (rc) return rc;
  const Geom& g = p->geom;
  double2* F = p->d_fields;
  NSF_HIP(p, hipMemcpyAsync(F, x3n, sizeof(double2) * 3 * g.n, hipMemcpyDeviceToDevice, p->stream));
  NSF_HIP(p, pass_yz(p, 2, -1, 3, F, 0, 1, nullptr));
  NSF_HIP(p, pass_yz(p, 1, -1, 3, F, 0, 0, nullptr));
  NSF_HIP(p, pass_x_fwd(p, part, F, reinterpret_cast<double2*>(y2n), nullptr));
  return NSF_OK;
}

int nsf_apply_PrH(nsf_plan p, const nsf_c128* x3n, nsf_c128* y2n) {
  return apply_adjoint(p, kPartP, x3n, y2n);
}

int nsf_apply_QrH(nsf_plan p, const nsf_c128* x3n, nsf_c128* y2n) {
  return apply_adjoint(p, kPartQ, x3n, y2n);
}

int nsf_apply_Ar(nsf_plan p, const nsf_c128* u4n, nsf_c128* out4n) {
  if (!p || !u4n || !out4n) return set_error(p, NSF_E_ARG, "NULL argument");
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  int rc = ensure_device(p);
  if (rc) return rc;
  return apply_Ar_dev(p, reinterpret_cast<const double2*>(u4n), reinterpret_cast<double2*>(out4n),
                      nullptr);
}

int nsf_profile_Ar(nsf_plan p, const nsf_c128* u4n, nsf_c128* out4n, int reps, double* ms_pass,
                   int max_pass, int* npass, double* ms_apply) {
  if (!p || !u4n || !out4n || reps < 1) return set_error(p, NSF_E_ARG, "bad argument");
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  int rc = ensure_device(p);
  if (rc) return rc;
  hipStream_t s = p->stream;
  double2* F = p->d_fields;
  const double2* u = reinterpret_cast<const double2*>(u4n);
  double2* out = reinterpret_cast<double2*>(out4n);
  constexpr int kPasses = 5;
  hipEvent_t ev[kPasses + 1];
  for (auto& e : ev) NSF_HIP(p, hipEventCreate(&e));
  double acc[kPasses] = {0, 0, 0, 0, 0};
  const VacSkip v = vac_of(p);
  for (int r = 0; r < reps; ++r) {
    NSF_HIP(p, hipEventRecord(ev[0], s));
    NSF_HIP(p, pass_x_inv(p, kPartBoth, u, F, nullptr));
    NSF_HIP(p, hipEventRecord(ev[1], s));
    NSF_HIP(p, pass_yz(p, 1, +1, 6, F, 0, 0, nullptr, &v));
    NSF_HIP(p, hipEventRecord(ev[2], s));
    NSF_HIP(p, pass_z_mid(p, F, nullptr, nullptr, nullptr, &v));
    NSF_HIP(p, hipEventRecord(ev[3], s));
    NSF_HIP(p, pass_yz(p, 1, -1, 6, F, 0, 0, nullptr, &v));
    NSF_HIP(p, hipEventRecord(ev[4], s));
    NSF_HIP(p, pass_x_fwd(p, kPartBoth, F, out, nullptr, v.on ? v.pscale : 1.0));
    NSF_HIP(p, hipEventRecord(ev[5], s));
    NSF_HIP(p, hipEventSynchronize(ev[5]));
    for (int i = 0; i < kPasses; ++i) {
      float ms = 0;
      NSF_HIP(p, hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      acc[i] += ms;
    }
  }
  if (npass) *npass = kPasses;
  if (ms_pass)
    for (int i = 0; i < kPasses && i < max_pass; ++i) ms_pass[i] = acc[i] / reps;
  if (ms_apply) {
    NSF_HIP(p, hipEventRecord(ev[0], s));
    for (int r = 0; r < reps; ++r) {
      rc = apply_Ar_dev(p, u, out, nullptr);
      if (rc) return rc;
    }
    NSF_HIP(p, hipEventRecord(ev[1], s));
    NSF_HIP(p, hipEventSynchronize(ev[1]));
    float ms = 0;
    NSF_HIP(p, hipEventElapsedTime(&ms, ev[0], ev[1]));
    *ms_apply = ms / reps;
  }
  for (auto& e : ev) hipEventDestroy(e);
  return NSF_OK;
}

int nsf_apply_Br(nsf_plan p, const nsf_c128* u4n, nsf_c128* out4n) {
  if (!p || !u4n || !out4n) return set_error(p, NSF_E_ARG, "NULL argument");
  int rc = ensure_device(p);
  if (rc) return rc;
  NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, reinterpret_cast<const double2*>(u4n),
                             reinterpret_cast<double2*>(out4n), nullptr, p->stream));
  return NSF_OK;
}

}  // extern "C"
