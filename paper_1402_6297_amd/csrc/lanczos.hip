// Invert Lanczos for B_r y = theta A_r y (Thm 4.2; Sec. 4.2; Algorithm 1
// step 5), for one instance or many in lock step.
//
// The operator A_r^{-1} B_r is self-adjoint in the A_r inner product and its
// largest eigenvalues theta are the inverses of the smallest positive omega.
// The basis V is kept A_r-orthonormal together with A_r V (classical
// Gram-Schmidt; a second pass only when the first removed more than half of
// the A-norm squared), and the projected matrix H = V^* B_r V is formed
// exactly from B_r applied to each new basis vector, so Ritz values are exact
// Rayleigh quotients of the pencil even though the inner CG solves are
// inexact.  After m expansions the basis is compressed to the best Ritz
// vectors plus the last Lanczos vector (thick restart).
//
// Many instances (k-points, grids, media) advance together: every CG
// iteration and every A_r apply is one launch per group of instances with
// the same grid (the instance is the grid's z index), each instance carrying
// its own convergence flag, and the host synchronises once per phase for the
// whole batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <tuple>

#include "nsf_internal.h"

namespace nsf {
namespace {

// Relaxed inner tolerance (relaxed_cg_tol, NSF_OPT_CG_RELAX = 1): tau =
// (theta_nev / theta_1) min(kRelaxC / max eta, kRelaxCap) res_tol.  Measured
// at res_tol 1e-8: without the theta_nev / theta_1 factor, 19 solves (128^3
// sphere and rods, twelve instances of the uneven batch, the chirality sweep
// near Phi = 0) converged with 6-15% fewer applies, but the 128^3 k-points
// next to Gamma (omega_10 / omega_1 = 17-35) stalled at 1-3.5e-8; with it those
// converge exactly as with fixed solves and the generic 128^3 points save 3-7%
// of the applies.  A cap of res_tol stalled two uneven instances, and c = 0.1
// with a cap of 1e-6 stalled the 128^3 sphere near 4e-8.
constexpr double kRelaxC = 0.1;
constexpr double kRelaxCap = 0.3;

struct Run {
  nsf_plan p = nullptr;
  int nev = 0, m = 0, kkeep = 0, max_restarts = 0;
  double res_tol = 0, cg_rtol = 0;
  double cg_tol = 0;  // inner CG tolerance of the next Lanczos steps (relaxed with the residuals)
  double eta_prev = INFINITY;  // largest wanted residual at the previous restart
  int stalls = 0;              // consecutive restarts that did not halve it
  bool relax = true;           // off for good after two such restarts
  unsigned long long seed = 0;
  long long len = 0;
  double2 *V = nullptr, *AV = nullptr, *w = nullptr, *z = nullptr, *bv = nullptr;
  std::vector<double2> H;
  int nb = 0;
  std::vector<double> theta, eta;
  double start_h2 = 0;  // |h|^2 of the projected CG start of the current step
  int start_m = 0;       // basis columns in that start (coefficients and indices in d_coef)
  int nlock = 0;        // V[0..nlock) (with A_r V) hold A_r-orthonormal vectors to keep
  std::vector<double2> Sk;
  nsf_stats st{};
  bool finished = false, converged = false;
  int status = NSF_OK;
  double2& Hat(int i, int j) { return H[(size_t)i * (m + 1) + j]; }
};

// Instances sharing one grid shape and pass configuration.
struct Group {
  std::vector<Run*> runs;
  std::vector<Run*> act;   // unfinished runs
  bool fast = false;       // batched register passes usable
  InstDesc* d_desc = nullptr;   // [act CG descriptors | act apply descriptors]
  InstDesc* h_desc = nullptr;   // pinned staging
  int cap = 0;
};

// Enqueue sum conj(x) y into d_res[slot] and copy it to h_res[slot].
int dot_async(nsf_plan p, const double2* x, const double2* y, long long len, int slot) {
  NSF_HIP(p, launch_dot_partials(x, y, len, p->d_partial, nullptr, p->stream));
  NSF_HIP(p, launch_reduce_partials(p->d_partial, reduce_parts_for(len), p->d_res + slot, p->stream));
  NSF_HIP(p, hipMemcpyAsync(p->h_res + slot, p->d_res + slot, sizeof(double2), hipMemcpyDeviceToHost,
                            p->stream));
  return NSF_OK;
}

InstDesc desc_of(Run* r, bool cg) {
  nsf_plan p = r->p;
  InstDesc d{};
  d.t = p->tabs;
  d.med = medium_view(p);
  d.fld = p->d_fields;
  if (cg) {
    d.skip = &p->d_state->done;
    d.cg = cg_fuse_of(p, r->w);
  } else {
    d.vin = r->w;
    d.vout = r->z;
  }
  return d;
}

// Whether the runs of G iterate in the q-free fused schedule.
bool group_qfree(const Group& G) {
  nsf_plan p0 = G.runs[0]->p;
  if (G.fast) return fast_z_mid_pq_items(p0->geom, p0->medium_kind, p0->opt_mid_cols) > 0;
  return cg_qfree(p0);
}

// Vacuum skipping for a group's shared launches: on when every run's plan has
// it (same shape and tiling in a group), with the largest listed counts of
// z tiles and y-pass x groups over the instances.
bool group_vac(const Group& G, VacSkip* out) {
  VacSkip acc;
  for (Run* r : G.act) {
    const VacSkip v = vac_of(r->p);
    if (!v.on) return false;
    const int zt = std::max(acc.ntiles, v.ntiles), xg = std::max(acc.nxg, v.nxg);
    acc = v;
    acc.ntiles = zt;
    acc.nxg = xg;
  }
  *out = acc;
  return !G.act.empty();
}

int upload_descs(Group& G, hipStream_t s) {
  G.act.clear();
  for (Run* r : G.runs)
    if (!r->finished) G.act.push_back(r);
  const int na = (int)G.act.size();
  if (!G.fast || na == 0) return NSF_OK;
  VacSkip gv;
  const bool vac = group_qfree(G) && group_vac(G, &gv);
  for (int i = 0; i < na; ++i) {
    G.h_desc[i] = desc_of(G.act[i], true);
    G.h_desc[i].cg.pnorm = vac ? 1 : 0;
    G.h_desc[na + i] = desc_of(G.act[i], false);
  }
  const hipError_t e = hipMemcpyAsync(G.d_desc, G.h_desc, sizeof(InstDesc) * 2 * na, hipMemcpyHostToDevice, s);
  return hip_check(G.act[0]->p, e, "descriptor upload");
}

// z = A_r w for every unfinished run.
int apply_all(std::vector<Group>& groups, hipStream_t s) {
  for (Group& G : groups) {
    const int na = (int)G.act.size();
    if (na == 0) continue;
    if (!G.fast) {
      for (Run* r : G.act) {
        const int rc = apply_Ar_dev(r->p, r->w, r->z, nullptr);
        if (rc) return rc;
      }
      continue;
    }
    nsf_plan p0 = G.act[0]->p;
    const Geom& g = p0->geom;
    const InstDesc* d = G.d_desc + na;
    VacSkip v;
    if (!group_vac(G, &v)) v = VacSkip{};
    NSF_HIP(p0, launch_fast_x_inv_synth(g, p0->tabs, kPartBoth, nullptr, nullptr, nullptr, s, d, na));
    NSF_HIP(p0, launch_fast_yz(g, p0->tabs, 1, +1, 6, nullptr, 0, 0, nullptr, s, d, na, nullptr, v.nxg,
                               v.on ? 1.0 : 0.0));
    NSF_HIP(p0, launch_fast_z_mid(g, p0->tabs, medium_view(p0), nullptr, p0->opt_mid_cols, nullptr, s, d, na,
                                  nullptr, nullptr, v.zscale, v.ntiles));
    NSF_HIP(p0, launch_fast_yz(g, p0->tabs, 1, -1, 6, nullptr, 0, 0, nullptr, s, d, na, nullptr, v.nxg,
                               v.on ? v.yscale : 0.0));
    NSF_HIP(p0, launch_fast_x_fwd_proj(g, p0->tabs, kPartBoth, nullptr, nullptr, nullptr, s, d, na, v.pscale));
  }
  return NSF_OK;
}

// One CG iteration of every unfinished run, enqueued on each run's plan stream
// (single instances) or on s (groups sharing launches).
int cg_iteration_all(std::vector<Group>& groups, hipStream_t s) {
  for (Group& G : groups) {
    const int na = (int)G.act.size();
    if (na == 0) continue;
    if (!G.fast) {
      for (Run* r : G.act) {
        const int rc = cg_iteration(r->p, r->w, cg_fusable(r->p));
        if (rc) return rc;
      }
      continue;
    }
    nsf_plan p0 = G.act[0]->p;
    const Geom& g = p0->geom;
    const InstDesc* d = G.d_desc;
    const CgFuse none{};
    const bool qf = group_qfree(G);
    VacSkip v;
    const bool vac = qf && group_vac(G, &v);  // the descriptors carry cg.pnorm = vac
    if (!vac) v = VacSkip{};
    int np1 = 0, np5 = 0, npm = 0;
    NSF_HIP(p0, launch_fast_cg_first(g, p0->tabs, none, nullptr, nullptr, &np1, s, d, na, qf));
    if (!qf) NSF_HIP(p0, launch_cgf_check(nullptr, np1, nullptr, s, d, na));
    NSF_HIP(p0, launch_fast_yz(g, p0->tabs, 1, +1, 6, nullptr, 0, 0, nullptr, s, d, na, nullptr, v.nxg,
                               vac ? 1.0 : 0.0));
    NSF_HIP(p0, launch_fast_z_mid(g, p0->tabs, medium_view(p0), nullptr, p0->opt_mid_cols, nullptr, s, d, na,
                                  nullptr, &npm, v.zscale, v.ntiles));
    if (!vac && (npm > 0) != qf)
      return set_error(p0, NSF_E_HIP, "fused CG: the z pass does not match the schedule");
    if (qf) NSF_HIP(p0, launch_cgf_alpha(nullptr, npm, nullptr, s, d, na, nullptr, vac ? np1 : 0));
    if (qf) NSF_HIP(p0, launch_cg_fold(nullptr, nullptr, 4 * g.n, nullptr, false, s, d, na));
    NSF_HIP(p0, launch_fast_yz(g, p0->tabs, 1, -1, 6, nullptr, 0, 0, nullptr, s, d, na, nullptr, v.nxg,
                               vac ? v.yscale : 0.0));
    NSF_HIP(p0, launch_fast_cg_last(g, p0->tabs, none, nullptr, nullptr, &np5, s, d, na, qf, v.pscale));
    if (qf)
      NSF_HIP(p0, launch_cgf_step_qf(nullptr, np5, nullptr, s, d, na));
    else
      NSF_HIP(p0, launch_cgf_step(nullptr, np5, nullptr, s, d, na, nullptr, npm));
  }
  return NSF_OK;
}

// The CG iteration of the current set of unfinished runs as one HIP graph,
// replayed between host reads of the CG states.  Every launch of an iteration
// takes its scalars (alpha, beta, iteration count, done flag) from device
// memory, so one captured iteration serves every iteration of every solve
// until the set of unfinished runs changes.  Captured and replayed on a
// private stream of default priority, ordered after the caller's stream by an
// event; the graph holds kernel nodes only.
struct CgGraph {
  static constexpr int kSizes = 4;  // graphs of 1, 2, 4 and 8 iterations
  hipStream_t cs = nullptr;
  hipEvent_t ev = nullptr;
  hipGraphExec_t exec[kSizes] = {};
  std::vector<const void*> sig;
  int captures = 0;
  void drop() {
    for (hipGraphExec_t& e : exec) {
      if (e) hipGraphExecDestroy(e);
      e = nullptr;
    }
  }
  ~CgGraph() {
    drop();
    if (ev) hipEventDestroy(ev);
    if (cs) hipStreamDestroy(cs);
  }
};

// Points the plans of the given runs at another stream for the guard's life.
struct StreamSwap {
  std::vector<std::pair<nsf_plan, hipStream_t>> saved;
  StreamSwap(std::vector<Run*>& act, hipStream_t to) {
    for (Run* r : act) {
      saved.emplace_back(r->p, r->p->stream);
      r->p->stream = to;
    }
  }
  ~StreamSwap() {
    for (auto& ps : saved) ps.first->stream = ps.second;
  }
};

// The graphs of 2^k consecutive CG iterations (k < kSizes) of the current set
// of unfinished runs, captured again when that set changes.  A chunk of c
// iterations replays the graphs of c's binary digits: a graph launch costs
// about as much host-to-GPU latency as one iteration's gaps otherwise would.
int cg_graph_ready(CgGraph& cg, std::vector<Group>& groups, std::vector<Run*>& act) {
  nsf_plan p0 = act[0]->p;
  std::vector<const void*> sig;
  for (Group& G : groups) {
    sig.push_back(reinterpret_cast<const void*>((size_t)G.act.size()));
    for (Run* r : G.act) sig.push_back(r->p);
  }
  if (cg.exec[0] && sig == cg.sig) return NSF_OK;
  cg.drop();
  for (int k = 0; k < CgGraph::kSizes; ++k) {
    NSF_HIP(p0, hipStreamBeginCapture(cg.cs, hipStreamCaptureModeRelaxed));
    int rc = NSF_OK;
    for (int i = 0; i < (1 << k) && !rc; ++i) rc = cg_iteration_all(groups, cg.cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cg.cs, &graph);
    if (rc) {
      if (graph) hipGraphDestroy(graph);
      cg.drop();
      return rc;
    }
    NSF_HIP(p0, e);
    const hipError_t ei = hipGraphInstantiate(&cg.exec[k], graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) cg.drop();
    NSF_HIP(p0, ei);
  }
  cg.sig = sig;
  cg.captures += 1;
  return NSF_OK;
}

// Whether run r iterates in the q-free fused schedule (by its group).
bool qfree_of(const std::vector<Group>& groups, const Run* r) {
  for (const Group& G : groups)
    for (const Run* q : G.runs)
      if (q == r) return group_qfree(G);
  return false;
}

// w = A_r^{-1} bv by CG for every unfinished run, all advancing together.
//
// With the projected start (the default) each run solves instead for the part
// of w that is A_r-orthogonal to the basis: the A_r-Galerkin solution in
// span(V) is V h with h = V^* A_r w = V^* B_r v, the H column already formed
// for the last basis vector v, so CG starts from r = bv - (A_r V) h and leaves
// e = w - V h in w.  The stopping test stays ||b - A_r (V h + e)|| <= rtol ||b||.
// The Gram-Schmidt pass that follows removes only what CG left in span(V),
// and the Lanczos direction is the same vector as from the plain start.
int cg_all(std::vector<Group>& groups, std::vector<Run*>& act, hipStream_t s, CgGraph* cgg) {
  for (Run* r : act) {
    nsf_plan p = r->p;
    int m = 0;
    r->start_h2 = 0;
    if (p->opt_cg_start && r->nb > 0 && r->nb <= 512) {
      // h; entries below 1e-8 max|h| are left to the Gram-Schmidt pass (h is
      // nearly tridiagonal between restarts, so this skips most of A_r V)
      const int nb = r->nb;
      double hmax = 0;
      for (int i = 0; i < nb; ++i) {
        const double2 h = r->Hat(i, nb - 1);
        hmax = std::max(hmax, std::hypot(h.x, h.y));
        r->start_h2 += h.x * h.x + h.y * h.y;
      }
      double2* hc = p->h_res + 64;
      for (int i = 0; i < nb; ++i) {
        const double2 h = r->Hat(i, nb - 1);
        if (std::hypot(h.x, h.y) > 1e-8 * hmax) {
          hc[m] = h;
          hc[512 + m] = make_double2((double)i, 0.0);
          ++m;
        }
      }
      for (int j = 0; j < m; ++j) hc[m + j] = hc[512 + j];
      if (m) NSF_HIP(p, hipMemcpyAsync(p->d_coef, hc, sizeof(double2) * 2 * m, hipMemcpyHostToDevice, s));
    }
    r->start_m = m;
    // kept directions when this run iterates q-free and its plan holds them
    const bool ring = p->d_ring && qfree_of(groups, r);
    NSF_HIP(p, launch_cg_init(r->bv, r->w, p->d_cg, ring ? p->d_ring : p->d_cg + r->len, r->len, p->d_partial,
                              p->d_state, r->cg_tol, 5000, s, m ? r->AV : nullptr, r->len, m,
                              m ? p->d_coef : nullptr, ring ? kCgRing : 0));
  }
  bool graph = cgg != nullptr && !debug_sync();
  for (Run* r : act) graph = graph && r->p->opt_cg_graph;
  hipStream_t ws = s;
  if (graph) {
    nsf_plan p0 = act[0]->p;
    if (!cgg->cs) NSF_HIP(p0, hipStreamCreateWithFlags(&cgg->cs, hipStreamNonBlocking));
    if (!cgg->ev) NSF_HIP(p0, hipEventCreateWithFlags(&cgg->ev, hipEventDisableTiming));
    NSF_HIP(p0, hipEventRecord(cgg->ev, s));
    NSF_HIP(p0, hipStreamWaitEvent(cgg->cs, cgg->ev, 0));
    ws = cgg->cs;
  }
  StreamSwap swap(act, ws);
  if (graph) {
    const int rc = cg_graph_ready(*cgg, groups, act);
    if (rc) return rc;
  }
  std::vector<double> rr_prev(act.size(), -1.0);
  std::vector<int> it_prev(act.size(), 0);
  int chunk = 4;
  for (;;) {
    if (graph) {
      for (int k = CgGraph::kSizes - 1, left = chunk; k >= 0; --k)
        for (; left >= (1 << k); left -= 1 << k) NSF_HIP(act[0]->p, hipGraphLaunch(cgg->exec[k], ws));
    } else {
      for (int c = 0; c < chunk; ++c) {
        const int rc = cg_iteration_all(groups, ws);
        if (rc) return rc;
      }
    }
    for (Run* r : act)
      NSF_HIP(r->p, hipMemcpyAsync(r->p->h_state, r->p->d_state, sizeof(CgState), hipMemcpyDeviceToHost, ws));
    NSF_HIP(act[0]->p, hipStreamSynchronize(ws));
    bool all = true;
    int next = 1;
    for (size_t i = 0; i < act.size(); ++i) {
      const CgState& h = *act[i]->p->h_state;
      if (h.done) continue;
      all = false;
      const bool lag = cg_fusable(act[i]->p) && !qfree_of(groups, act[i]);
      next = std::max(next, cg_predict(h, rr_prev[i], it_prev[i], lag));
      rr_prev[i] = h.rr;
      it_prev[i] = h.iter;
    }
    if (all) break;
    chunk = next;
  }
  for (Run* r : act) {
    const CgState& h = *r->p->h_state;
    r->st.cg_solves += 1;
    r->st.cg_iters_total += h.iter;
    r->st.matvecs += h.iter;
    if (h.status == NSF_E_BREAKDOWN)
      return set_error(r->p, NSF_E_BREAKDOWN, "CG breakdown: p^* A_r p <= 0 or not finite");
    if (qfree_of(groups, r) && r->p->d_ring)  // the directions since the last fold (ws has drained)
      NSF_HIP(r->p, launch_cg_fold(r->w, r->p->d_ring, r->len, r->p->d_state, true, s));
    else if (qfree_of(groups, r))  // the final x = x + alpha p
      NSF_HIP(r->p, launch_cg_finish(r->w, r->p->d_cg + r->len, r->len, r->p->d_state, s));
  }
  return NSF_OK;
}

// A_r-cosine between w and a basis vector below which the sparse Gram-Schmidt
// step leaves that component in w: 1e-2 of the residual tolerance, at most
// 1e-10.  After the projected CG start the new direction is already
// A_r-orthogonal to the basis to about the CG tolerance; a basis that is
// orthogonal to level c only reaches residuals of about c, hence the margin.
double ortho_skip_cos(const Run* r) { return std::min(1e-10, 1e-2 * r->res_tol); }

// Full classical Gram-Schmidt pass of (w, z) against V[0..nb) in the A_r inner
// product (c = (A_r V)^* w; w -= V c, z -= (A_r V) c); ||w||_A^2 after it into
// h_res[1].
int ortho_pass(Run* r) {
  nsf_plan p = r->p;
  hipStream_t s = p->stream;
  NSF_HIP(p, launch_multi_dot(r->AV, r->len, r->nb, r->w, r->len, p->d_partial, p->d_coef, s));
  NSF_HIP(p, launch_multi_axpy(r->V, r->len, r->nb, p->d_coef, r->w, r->len, s, r->AV, r->z));
  r->st.ortho_passes += 1;
  return dot_async(p, r->w, r->z, r->len, 1);
}

// Enqueue V[j] = w / sqrt(nrm2), A V[j] = z / sqrt(nrm2), bv = B_r V[j] and the
// H column V^* bv (copied to h_res[64 ..]).
int admit_enqueue(Run* r, int j, double nrm2) {
  nsf_plan p = r->p;
  hipStream_t s = p->stream;
  if (!(nrm2 > 0.0) || !std::isfinite(nrm2))
    return set_error(p, NSF_E_BREAKDOWN, "A_r-norm of a new basis vector is not positive");
  const double sc = 1.0 / std::sqrt(nrm2);
  NSF_HIP(p, launch_scale_copy(r->w, r->V + (size_t)j * r->len, sc, 0.0, r->len, s));
  NSF_HIP(p, launch_scale_copy(r->z, r->AV + (size_t)j * r->len, sc, 0.0, r->len, s));
  NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, r->V + (size_t)j * r->len, r->bv, nullptr, s));
  NSF_HIP(p, launch_multi_dot(r->V, r->len, j + 1, r->bv, r->len, p->d_partial, p->d_coef, s));
  NSF_HIP(p, hipMemcpyAsync(p->h_res + 64, p->d_coef, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, s));
  return NSF_OK;
}

void admit_finish(Run* r, int j) {
  const double2* hc = r->p->h_res + 64;
  for (int i = 0; i <= j; ++i) {  // H[i][j] = V_i^* B V_j
    r->Hat(i, j) = hc[i];
    r->Hat(j, i) = cconj(hc[i]);
  }
  r->Hat(j, j).y = 0.0;
}

// Rayleigh-Ritz on V[0..m) of one run: rotate to the kkeep best Ritz
// vectors, enqueue the residual norms of the wanted pairs.
int restart_enqueue(Run* r) {
  nsf_plan p = r->p;
  hipStream_t s = p->stream;
  const int m = r->m, kk = r->kkeep;
  std::vector<double2> Hm((size_t)m * m), S((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Hm[(size_t)i * m + j] = r->Hat(i, j);
  std::vector<double> wv(m);
  hermitian_eig(m, Hm.data(), wv.data(), S.data());
  r->Sk.assign((size_t)m * kk, make_double2(0, 0));
  for (int c = 0; c < kk; ++c) {  // descending theta: column c of Sk is eigenvector m-1-c
    r->theta[c] = wv[m - 1 - c];
    for (int i = 0; i < m; ++i) r->Sk[(size_t)c * m + i] = S[(size_t)i * m + (m - 1 - c)];
  }
  NSF_HIP(p, hipMemcpyAsync(p->d_small, r->Sk.data(), sizeof(double2) * (size_t)m * kk, hipMemcpyHostToDevice, s));
  NSF_HIP(p, launch_rotate(r->V, r->len, m, kk, p->d_small, r->len, s));
  NSF_HIP(p, launch_rotate(r->AV, r->len, m, kk, p->d_small, r->len, s));
  for (int i = 0; i < r->nev; ++i) {
    NSF_HIP(p, launch_residual_norms(p->geom, p->tabs, r->V + (size_t)i * r->len, r->AV + (size_t)i * r->len,
                                     r->theta[i], p->d_partial, reinterpret_cast<double*>(p->d_res + 64 + i), s));
  }
  NSF_HIP(p, hipMemcpyAsync(p->h_res + 64, p->d_res + 64, sizeof(double2) * r->nev, hipMemcpyDeviceToHost, s));
  // hermitian_eig reads the host copy of the Sk buffer asynchronously: keep it
  // alive in r->Sk until the next synchronisation.
  return NSF_OK;
}

// Inner CG tolerance after a restart.  The solves are inexact applications of
// A_r^{-1} B_r, and the accuracy of the later ones may be lowered in inverse
// proportion to the residual of the wanted Ritz pairs (the relaxation strategy
// of inexact Krylov methods: Simoncini and Szyld, SIAM J. Sci. Comput. 25
// (2003); for eigenproblems, Simoncini, SIAM J. Numer. Anal. 43 (2005)).  A
// new direction enters a wanted Ritz vector with a weight of about that
// pair's residual eta_i, so a solve error of relative size tau adds about
// tau eta_i to it: tau = c res_tol / max_i eta_i keeps that below c res_tol
// for every wanted pair.  The tolerance never drops below cg_rtol and stays at
// most kRelaxCap res_tol.  H = V^* B_r V is formed exactly and A_r V follows V to
// rounding (the image comes from the CG's own residual), so the relaxed
// solves change how fast the basis converges, never the reported pairs, whose
// residuals are recomputed with exact applies.  What the bound leaves out is
// thick restarting: the part of a kept Ritz vector's residual that comes from
// solve errors is not along the last Lanczos vector, so later steps never
// remove it, and it sets a floor under the residuals.  Hence the cap at a
// fraction of res_tol, and the guard: once two restarts in a row fail to halve the largest
// wanted residual, the solve returns to cg_rtol for good.
double relaxed_cg_tol(const Run* r, double eta_max) {
  if (!r->p->opt_cg_relax || !r->relax) return r->cg_rtol;
  const double ref = (eta_max > 0.0 && eta_max < 1.0) ? eta_max : 1.0;
  // A solve error is relative to ||B_r v||, i.e. to the scale of the largest
  // wanted theta, while pair i's residual is relative to theta_i: scale by
  // theta_nev / theta_1 (no relaxation before the first Ritz values exist).
  double spread = 0.0;
  if (r->theta.size() >= (size_t)r->nev) {
    const double t1 = r->theta[0], tn = r->theta[r->nev - 1];
    spread = (t1 > 0.0 && tn > 0.0 && std::isfinite(t1)) ? tn / t1 : 0.0;
  }
  return std::max(r->cg_rtol, spread * std::min(kRelaxCap * r->res_tol, kRelaxC * r->res_tol / ref));
}

// After the restart's synchronisation: residuals, new projected matrix for
// [Ritz vectors, V[m]], move V[m] next to the Ritz vectors.
int restart_finish(Run* r) {
  nsf_plan p = r->p;
  hipStream_t s = p->stream;
  const int m = r->m, kk = r->kkeep;
  bool all = true;
  double eta_max = 0.0;
  for (int i = 0; i < r->nev; ++i) {
    const double2 r2 = p->h_res[64 + i];
    r->eta[i] = std::sqrt(r2.x) / (std::fabs(r->theta[i]) * std::sqrt(r2.y));
    if (!(r->theta[i] > 0.0) || !(r->eta[i] <= r->res_tol)) all = false;
    eta_max = std::isfinite(r->eta[i]) ? std::max(eta_max, r->eta[i]) : 1.0;
  }
  if (r->cg_tol > r->cg_rtol) {  // stagnation guard of the relaxed solves
    r->stalls = eta_max > 0.5 * r->eta_prev ? r->stalls + 1 : 0;
    if (r->stalls >= 2) r->relax = false;
  }
  r->eta_prev = eta_max;
  r->cg_tol = relaxed_cg_tol(r, eta_max);
  std::vector<double2> row(kk);
  for (int c = 0; c < kk; ++c) {
    double2 acc = make_double2(0, 0);
    for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(r->Hat(m, i), r->Sk[(size_t)c * m + i]));
    row[c] = acc;
  }
  const double2 hmm = r->Hat(m, m);
  std::fill(r->H.begin(), r->H.end(), make_double2(0, 0));
  for (int c = 0; c < kk; ++c) {
    r->Hat(c, c) = make_double2(r->theta[c], 0);
    r->Hat(kk, c) = row[c];
    r->Hat(c, kk) = cconj(row[c]);
  }
  r->Hat(kk, kk) = hmm;
  NSF_HIP(p, hipMemcpyAsync(r->V + (size_t)kk * r->len, r->V + (size_t)m * r->len, sizeof(double2) * r->len,
                            hipMemcpyDeviceToDevice, s));
  NSF_HIP(p, hipMemcpyAsync(r->AV + (size_t)kk * r->len, r->AV + (size_t)m * r->len, sizeof(double2) * r->len,
                            hipMemcpyDeviceToDevice, s));
  r->nb = kk + 1;
  if (all) {
    r->converged = true;
    r->finished = true;
  } else {
    r->st.restarts += 1;
    if (r->st.restarts > r->max_restarts) r->finished = true;
  }
  return NSF_OK;
}

// Replace w by a fresh random direction orthogonal to the basis (the Krylov
// space became invariant).  Synchronous; rare.
int refresh_direction(Run* r, hipStream_t s) {
  nsf_plan p = r->p;
  NSF_HIP(p, launch_randn(r->w, r->len, r->seed + 7919ULL * (r->st.lanczos_steps + 1), s));
  int rc = apply_Ar_dev(p, r->w, r->z, nullptr);
  if (rc) return rc;
  r->st.matvecs += 1;
  for (int pass = 0; pass < 2; ++pass) {
    rc = ortho_pass(r);
    if (rc) return rc;
  }
  NSF_HIP(p, hipStreamSynchronize(s));
  return NSF_OK;
}

// H columns of the kept block V[0..nlock) (exact: B_r applied to each vector).
int lock_in(Run* r, hipStream_t s) {
  nsf_plan p = r->p;
  for (int j = 0; j < r->nlock; ++j) {
    NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, r->V + (size_t)j * r->len, r->bv, nullptr, s));
    NSF_HIP(p, launch_multi_dot(r->V, r->len, j + 1, r->bv, r->len, p->d_partial, p->d_coef, s));
    NSF_HIP(p, hipMemcpyAsync(p->h_res + 64, p->d_coef, sizeof(double2) * (j + 1), hipMemcpyDeviceToHost, s));
    NSF_HIP(p, hipStreamSynchronize(s));
    admit_finish(r, j);
  }
  r->nb = r->nlock;
  return NSF_OK;
}

// Instances with at least this many voxels run one per wave in nsf_batch_eigs
// (measured: 12 batched 96^3 instances 5% faster than plain solves, 8 batched
// 128^3 instances 2.6% slower).
constexpr long long kSoloVoxels = 1LL << 21;

// Run every instance to convergence (or its restart cap) in lock step.
int run_engine(std::vector<Run*>& runs, hipStream_t s) {
  // groups of equal grid shape, pass configuration and z-pass kernel (media
  // coupling all six fields cannot share the field-pair launches)
  std::map<std::tuple<int, int, int, double, double, int, int>, int> key;
  std::vector<Group> groups;
  for (Run* r : runs) {
    const Geom& g = r->p->geom;
    auto k = std::make_tuple(g.n1, g.n2, g.n3, g.alpha, g.beta, r->p->opt_fft_path,
                             (six_coupled(r->p->medium_kind) ? 1 << 20 : 0) + r->p->opt_mid_cols * 2048 +
                                 g.mid_pairs * 1024 + g.x_rows * 32 + g.yz_cols);
    if (!key.count(k)) {
      key[k] = (int)groups.size();
      groups.emplace_back();
    }
    groups[key[k]].runs.push_back(r);
  }
  int rc = NSF_OK;
  for (Group& G : groups) {
    nsf_plan p0 = G.runs[0]->p;
    const Geom& g = p0->geom;
    G.fast = p0->opt_fft_path == 0 && fast_axis(g.n1) && fast_axis(g.n2) && fast_axis(g.n3) &&
             cg_fusable(p0) && G.runs.size() > 1;
    G.cap = (int)G.runs.size();
    if (G.fast) {
      NSF_HIP(p0, hipMalloc(&G.d_desc, sizeof(InstDesc) * 2 * G.cap));
      NSF_HIP(p0, hipHostMalloc(&G.h_desc, sizeof(InstDesc) * 2 * G.cap));
    }
  }
  CgGraph cg_graph;
  auto release = [&]() {
    hipStreamSynchronize(s);
    for (Group& G : groups) {
      if (G.d_desc) hipFree(G.d_desc);
      if (G.h_desc) hipHostFree(G.h_desc);
    }
  };
  auto fail = [&](int code) {
    release();
    return code;
  };
  for (Group& G : groups)
    if ((rc = upload_descs(G, s))) return fail(rc);
  for (Run* r : runs) {
    r->nb = 0;
    if (r->nlock > 0 && (rc = lock_in(r, s))) return fail(rc);
  }

  // start vectors: seeded complex normal, A_r-normalised (and A_r-orthogonal to
  // a kept block); with a start block Y0
  // (nsf_eigs_set_start) a seeded combination sum_j c_j Y0_j, c_j complex normal,
  // plus the normal vector at 1e-3 of its size, so that no direction is absent
  for (Run* r : runs) {
    nsf_plan p = r->p;
    NSF_HIP(p, launch_randn(r->w, r->len, r->seed, s));
    if (p->start_Y && p->start_count > 0) {
      const int c = p->start_count;
      // ||Y0_j||_2 is O(1) for A_r-normalised vectors, the normal vector's is sqrt(2 len)
      const double tau = 1e-3 * std::sqrt((double)c / (2.0 * (double)r->len));
      NSF_HIP(p, launch_scale_copy(r->w, r->w, tau, 0.0, r->len, s));
      unsigned long long z = r->seed ^ 0x9e3779b97f4a7c15ULL;
      auto u01 = [&z]() {
        z += 0x9E3779B97F4A7C15ULL;
        unsigned long long t = z;
        t = (t ^ (t >> 30)) * 0xBF58476D1CE4E5B9ULL;
        t = (t ^ (t >> 27)) * 0x94D049BB133111EBULL;
        t ^= t >> 31;
        return ((t >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      };
      double2* hc = p->h_res + 64;
      for (int j = 0; j < c; ++j) {  // -c_j, Box-Muller (multi_axpy subtracts)
        const double a = std::sqrt(-2.0 * std::log(u01())), b = 6.283185307179586 * u01();
        hc[j] = make_double2(-a * std::cos(b), -a * std::sin(b));
      }
      NSF_HIP(p, hipMemcpyAsync(p->d_coef, hc, sizeof(double2) * c, hipMemcpyHostToDevice, s));
      NSF_HIP(p, launch_multi_axpy(p->start_Y, r->len, c, p->d_coef, r->w, r->len, s));
      NSF_HIP(p, hipStreamSynchronize(s));  // hc is reused below
    }
    p->start_Y = nullptr;  // used once
    p->start_count = 0;
  }
  if ((rc = apply_all(groups, s))) return fail(rc);
  for (Run* r : runs) {
    r->st.matvecs += 1;
    for (int pass = 0; pass < (r->nb > 0 ? 2 : 0); ++pass)
      if ((rc = ortho_pass(r))) return fail(rc);
    if ((rc = dot_async(r->p, r->w, r->z, r->len, 0))) return fail(rc);
  }
  NSF_HIP(runs[0]->p, hipStreamSynchronize(s));
  for (Run* r : runs)
    if ((rc = admit_enqueue(r, r->nb, r->p->h_res[0].x))) return fail(rc);
  NSF_HIP(runs[0]->p, hipStreamSynchronize(s));
  for (Run* r : runs) {
    admit_finish(r, r->nb);
    r->nb += 1;
  }

  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); };
  double t_cg = 0, t_orth = 0, t_rst = 0;
  for (;;) {
    std::vector<Run*> act;
    for (Run* r : runs)
      if (!r->finished) act.push_back(r);
    if (act.empty()) break;
    // expand: w = A_r^{-1} B_r V[nb-1], z = A_r w
    auto t0 = clk::now();
    if ((rc = cg_all(groups, act, s, &cg_graph))) return fail(rc);
    t_cg += ms_since(t0);
    t0 = clk::now();
    // z = A_r w from the CG's right-hand side and final residual: CG solved
    // A_r w = bv - (A_r V) h from w = 0 (projected start), so A_r w =
    // bv - (A_r V) h - r, with h and its basis indices still in d_coef.  Then
    // B_r w into bv and one pass over V for both V^* z (the A_r inner products
    // with the basis) and V^* B_r w (the new column of H), and the norms
    // w^* A_r w, w^* B_r w.
    for (Run* r : act) {
      nsf_plan p = r->p;
      // z, B_r w into bv, ||w||_A^2 = w^* z and w^* B_r w into slots 0 and 1
      NSF_HIP(p, launch_step_fused(p->geom, p->tabs, 0, r->w, r->z, r->bv, p->d_cg, nullptr, r->AV, r->len,
                                   r->start_m, p->d_coef, p->d_partial, p->d_res, s));
      NSF_HIP(p, hipMemcpyAsync(p->h_res, p->d_res, sizeof(double2) * 2, hipMemcpyDeviceToHost, s));
      NSF_HIP(p, launch_multi_dot2(r->V, r->len, r->nb, r->z, r->bv, r->len, p->d_partial, p->d_coef, s));
      NSF_HIP(p, hipMemcpyAsync(p->h_res + 64, p->d_coef, sizeof(double2) * 2 * r->nb, hipMemcpyDeviceToHost, s));
    }
    NSF_HIP(act[0]->p, hipStreamSynchronize(s));
    // Sparse Gram-Schmidt: only the coefficients c_i = v_i^* A_r w above
    // ortho_skip_cos ||w||_A are removed (usually none or the few basis columns
    // the projected start left out), reading just those columns of V and A_r V;
    // the H column follows by linearity, V^* B_r (w - V_S c_S) = g - H[:, S] c_S,
    // with H exact on the host.  A second full pass (and the column recomputed)
    // only when the update removes more than half of ||w||_A^2.
    std::vector<Run*> slow, sparse;
    std::vector<std::vector<double2>> cg_host(act.size());
    std::vector<std::vector<int>> sel(act.size());
    std::vector<double> h0s(act.size());
    auto admit_fast = [&](Run* r, const std::vector<double2>& cgv, const std::vector<int>& S, double h1,
                          double wbw) -> int {
      nsf_plan p = r->p;
      const int nb = r->nb;
      const double sc = 1.0 / std::sqrt(h1);
      double2* hc = p->h_res + 64;
      for (int i = 0; i < nb; ++i) {
        double2 gi = cgv[nb + i];
        for (int k : S) gi = csub(gi, cmul(r->Hat(i, k), cgv[k]));
        hc[i] = cscale(gi, sc);
      }
      hc[nb] = make_double2(wbw / h1, 0.0);
      admit_finish(r, nb);
      NSF_HIP(p, launch_scale_copy(r->w, r->V + (size_t)nb * r->len, sc, 0.0, r->len, s));
      NSF_HIP(p, launch_scale_copy(r->z, r->AV + (size_t)nb * r->len, sc, 0.0, r->len, s));
      NSF_HIP(p, launch_scale_copy(r->bv, r->bv, sc, 0.0, r->len, s));  // B_r of the new vector
      r->nb += 1;
      r->st.lanczos_steps += 1;
      r->st.ortho_passes += 1;
      return NSF_OK;
    };
    for (size_t a = 0; a < act.size(); ++a) {
      Run* r = act[a];
      nsf_plan p = r->p;
      const int nb = r->nb;
      const double h0 = p->h_res[0].x, wbw = p->h_res[1].x;
      h0s[a] = h0;
      const double tau = ortho_skip_cos(r);
      cg_host[a].assign(p->h_res + 64, p->h_res + 64 + 2 * nb);
      for (int i = 0; i < nb; ++i)
        if (cabs2(cg_host[a][i]) > tau * tau * h0) sel[a].push_back(i);
      const bool ok = p->opt_ortho_gate && h0 > 0.0 && std::isfinite(h0) && std::isfinite(wbw) &&
                      h0 > 1e-20 * (h0 + r->start_h2) && (int)sel[a].size() <= 64;
      if (!ok) {
        slow.push_back(r);
      } else if (sel[a].empty()) {
        if ((rc = admit_fast(r, cg_host[a], sel[a], h0, wbw))) return fail(rc);
      } else {
        double2* hc = p->h_res + 64;  // staging: coefficients, then indices
        const int ms = (int)sel[a].size();
        for (int k = 0; k < ms; ++k) {
          hc[k] = cg_host[a][sel[a][k]];
          hc[ms + k] = make_double2((double)sel[a][k], 0.0);
        }
        NSF_HIP(p, hipMemcpyAsync(p->d_coef, hc, sizeof(double2) * 2 * ms, hipMemcpyHostToDevice, s));
        // the update, B_r w, and ||w||_A^2, w^* B_r w after it into slots 2 and 3
        NSF_HIP(p, launch_step_fused(p->geom, p->tabs, 1, r->w, r->z, r->bv, nullptr, r->V, r->AV, r->len, ms,
                                     p->d_coef, p->d_partial, p->d_res + 2, s));
        NSF_HIP(p, hipMemcpyAsync(p->h_res + 2, p->d_res + 2, sizeof(double2) * 2, hipMemcpyDeviceToHost, s));
        sparse.push_back(r);
      }
    }
    if (!sparse.empty()) {
      NSF_HIP(sparse[0]->p, hipStreamSynchronize(s));
      for (Run* r : sparse) {
        const size_t a = std::find(act.begin(), act.end(), r) - act.begin();
        nsf_plan p = r->p;
        const double h1 = p->h_res[2].x, wbw1 = p->h_res[3].x;
        if (!(h1 > 0.5 * h0s[a]) || !std::isfinite(h1) || !std::isfinite(wbw1)) {
          p->h_res[0].x = h1;  // the full path below starts from the updated w
          slow.push_back(r);
          continue;
        }
        if ((rc = admit_fast(r, cg_host[a], sel[a], h1, wbw1))) return fail(rc);
      }
    }
    if (!slow.empty()) {
      for (Run* r : slow)
        if ((rc = ortho_pass(r))) return fail(rc);  // norm before: slot 0 above
      NSF_HIP(slow[0]->p, hipStreamSynchronize(s));
      bool again = false;
      for (Run* r : slow) {
        nsf_plan p = r->p;
        if (p->h_res[1].x <= 0.5 * p->h_res[0].x) {  // second pass needed
          if ((rc = ortho_pass(r))) return fail(rc);
          again = true;
        }
      }
      if (again) NSF_HIP(slow[0]->p, hipStreamSynchronize(s));
      for (Run* r : slow) {
        // invariant subspace: nothing of A_r^{-1} B_r v is left outside span(V)
        if (!(r->p->h_res[1].x > 1e-20 * (r->p->h_res[0].x + r->start_h2))) {
          if ((rc = refresh_direction(r, s))) return fail(rc);
        }
        if ((rc = admit_enqueue(r, r->nb, r->p->h_res[1].x))) return fail(rc);
      }
      NSF_HIP(slow[0]->p, hipStreamSynchronize(s));
      for (Run* r : slow) {
        admit_finish(r, r->nb);
        r->nb += 1;
        r->st.lanczos_steps += 1;
      }
    }
    t_orth += ms_since(t0);
    t0 = clk::now();
    bool any_restart = false;
    for (Run* r : act)
      if (r->nb == r->m + 1) {
        if ((rc = restart_enqueue(r))) return fail(rc);
        any_restart = true;
      }
    if (!any_restart) continue;
    NSF_HIP(act[0]->p, hipStreamSynchronize(s));
    bool changed = false;
    for (Run* r : act)
      if (r->nb == r->m + 1) {
        if ((rc = restart_finish(r))) return fail(rc);
        changed |= r->finished;
      }
    if (changed)
      for (Group& G : groups)
        if ((rc = upload_descs(G, s))) return fail(rc);
    t_rst += ms_since(t0);
  }
  for (Run* r : runs) {
    r->st.ms_cg = t_cg;
    r->st.ms_orth = t_orth;
    r->st.ms_restart = t_rst;
  }
  release();
  return NSF_OK;
}

// Prepare one run on plan p (workspace, parameters).
int make_run(nsf_plan p, int nev, double res_tol, double cg_rtol, int max_basis, int max_restarts,
             unsigned long long seed, Run& r) {
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  if (p->medium_kind == kMedNfsep)
    return set_error(p, NSF_E_STATE, "an NFSEP medium has no HHPD pencil; use nsf_eigs_nfsep");
  const long long n = p->geom.n, len = 4 * n;
  if (nev < 1 || nev > 256 || 2LL * nev >= len) return set_error(p, NSF_E_ARG, "nev out of range");
  if (!(res_tol > 0.0) || !(cg_rtol > 0.0)) return set_error(p, NSF_E_ARG, "tolerances must be > 0");
  int m = max_basis > 0 ? max_basis : std::max(3 * nev, nev + 8);
  if (m < nev + 2) m = nev + 2;
  if (m > 510) m = 510;
  if (m >= len) m = (int)len - 1;
  if (m < nev + 2) return set_error(p, NSF_E_ARG, "grid too small for nev");
  int rc = ensure_cg(p);
  if (rc) return rc;
  rc = ensure_ring(p, cg_qfree(p));
  if (rc) return rc;
  rc = ensure_basis(p, (size_t)m + 1);
  if (rc) return rc;
  rc = ensure_small(p, (size_t)m * m);
  if (rc) return rc;
  r.p = p;
  r.nev = nev;
  r.m = m;
  r.kkeep = std::min(m - 1, nev + (m - nev) / 2);
  r.max_restarts = max_restarts > 0 ? max_restarts : 1000;
  r.res_tol = res_tol;
  r.cg_rtol = cg_rtol;
  r.cg_tol = relaxed_cg_tol(&r, 1.0);
  r.seed = seed;
  r.len = len;
  r.V = p->d_basis;
  r.AV = r.V + (size_t)(m + 1) * len;
  r.w = p->d_cg + 3 * len;
  r.z = r.w + len;
  r.bv = r.z + len;
  r.H.assign((size_t)(m + 1) * (m + 1), make_double2(0, 0));
  r.theta.assign(m, 0.0);
  r.eta.assign(nev, INFINITY);
  return NSF_OK;
}

// Final values of the wanted pairs from exact operator applications: for each
// Ritz vector v, A_r v by one apply (replacing the image carried along by the
// CG recurrences), v rescaled to unit A_r-norm, theta = v^* B_r v / v^* A_r v,
// and eta from B_r v - theta A_r v.  The Lanczos values differ from these only
// by the rounding the recurrences accumulate (about 1e-14 relative), but the
// reported omega and residual are then those of the returned vectors exactly.
// Pairs are re-sorted by theta if the refinement swapped neighbours.
int refine_run(Run* r) {
  nsf_plan p = r->p;
  hipStream_t s = p->stream;
  const long long L = r->len;
  for (int i = 0; i < r->nev; ++i) {
    double2* v = r->V + (size_t)i * L;
    double2* av = r->AV + (size_t)i * L;
    int rc = apply_Ar_dev(p, v, av, nullptr);
    if (rc) return rc;
    r->st.matvecs += 1;
    NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, v, r->bv, nullptr, s));
    if ((rc = dot_async(p, v, av, L, 8))) return rc;
    if ((rc = dot_async(p, v, r->bv, L, 9))) return rc;
    NSF_HIP(p, hipStreamSynchronize(s));
    const double a = p->h_res[8].x, b = p->h_res[9].x;
    if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b))
      return set_error(p, NSF_E_BREAKDOWN, "A_r-norm of a Ritz vector is not positive");
    const double sc = 1.0 / std::sqrt(a);
    NSF_HIP(p, launch_scale_copy(v, v, sc, 0.0, L, s));
    NSF_HIP(p, launch_scale_copy(av, av, sc, 0.0, L, s));
    r->theta[i] = b / a;
    NSF_HIP(p, launch_residual_norms(p->geom, p->tabs, v, av, r->theta[i], p->d_partial,
                                     reinterpret_cast<double*>(p->d_res + 64 + i), s));
  }
  NSF_HIP(p, hipMemcpyAsync(p->h_res + 64, p->d_res + 64, sizeof(double2) * r->nev, hipMemcpyDeviceToHost, s));
  NSF_HIP(p, hipStreamSynchronize(s));
  bool all = true;
  for (int i = 0; i < r->nev; ++i) {
    const double2 r2 = p->h_res[64 + i];
    r->eta[i] = std::sqrt(r2.x) / (std::fabs(r->theta[i]) * std::sqrt(r2.y));
    if (!(r->theta[i] > 0.0) || !(r->eta[i] <= r->res_tol)) all = false;
  }
  r->converged = all;
  // insertion sort by descending theta; columns of V and A_r V move through
  // the bv scratch
  for (int i = 1; i < r->nev; ++i)
    for (int j = i; j > 0 && r->theta[j] > r->theta[j - 1]; --j) {
      for (double2* M : {r->V, r->AV}) {
        double2* a0 = M + (size_t)(j - 1) * L;
        double2* a1 = M + (size_t)j * L;
        NSF_HIP(p, hipMemcpyAsync(r->bv, a0, sizeof(double2) * L, hipMemcpyDeviceToDevice, s));
        NSF_HIP(p, hipMemcpyAsync(a0, a1, sizeof(double2) * L, hipMemcpyDeviceToDevice, s));
        NSF_HIP(p, hipMemcpyAsync(a1, r->bv, sizeof(double2) * L, hipMemcpyDeviceToDevice, s));
      }
      std::swap(r->theta[j], r->theta[j - 1]);
      std::swap(r->eta[j], r->eta[j - 1]);
    }
  return NSF_OK;
}

// Multiplicity checks (NSF_OPT_VERIFY) after r has converged and been refined:
// a single start vector cannot see more than one direction of a multiple
// eigenvalue.  Each check keeps the converged vectors, starts a new Lanczos
// sequence from a fresh random vector A_r-orthogonal to them, and takes the
// best nev pairs of the union; it stops once a check changes nothing.  The
// counters of every sequence add up in r.st.
int verify_run(nsf_plan p, Run& r, int max_basis, int max_restarts, unsigned long long seed) {
  const int nev = r.nev;
  for (int v = 0; v < p->opt_verify; ++v) {
    std::vector<double> before(r.theta.begin(), r.theta.begin() + nev);
    Run r2;
    int rc = make_run(p, nev, r.res_tol, r.cg_rtol, max_basis, max_restarts, seed + 7919ULL * (v + 1), r2);
    if (rc) return rc;
    r2.nlock = nev;
    const nsf_stats acc = r.st;
    std::vector<Run*> runs{&r2};
    if ((rc = run_engine(runs, p->stream))) return rc;
    const auto tr = std::chrono::steady_clock::now();
    if ((rc = refine_run(&r2))) return rc;
    r2.st.ms_restart += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tr).count();
    bool changed = false;
    for (int i = 0; i < nev; ++i)
      changed |= std::fabs(r2.theta[i] - before[i]) > 1e-10 * std::fabs(before[0]);
    const nsf_stats add = r2.st;
    r = std::move(r2);
    r.st = acc;
    r.st.matvecs += add.matvecs;
    r.st.cg_iters_total += add.cg_iters_total;
    r.st.cg_solves += add.cg_solves;
    r.st.lanczos_steps += add.lanczos_steps;
    r.st.restarts += add.restarts;
    r.st.ortho_passes += add.ortho_passes;
    r.st.ms_cg += add.ms_cg;
    r.st.ms_orth += add.ms_orth;
    r.st.ms_restart += add.ms_restart;
    if (!changed) break;
  }
  return NSF_OK;
}

void finish_run(Run& r, double* omega, double* resid, nsf_stats* stats, double ms) {
  int nconv = 0;
  for (int i = 0; i < r.nev; ++i) {
    omega[i] = 1.0 / r.theta[i];
    if (resid) resid[i] = r.eta[i];
    if (r.eta[i] <= r.res_tol) ++nconv;
  }
  r.st.converged = nconv;
  r.st.cg_iters_avg = r.st.cg_solves ? (double)r.st.cg_iters_total / r.st.cg_solves : 0.0;
  r.st.bytes_alg = 336.0 * (double)r.p->geom.n * (double)r.st.matvecs;
  r.st.ms_total = ms;
  if (stats) *stats = r.st;
}

}  // namespace
}  // namespace nsf

using namespace nsf;

// The batch: independent plans (grid, k, medium each) on one stream.
struct nsf_batch_s {
  std::vector<nsf_plan> plans;
  hipStream_t stream = nullptr;
  std::string last_error;
};

extern "C" {

int nsf_eigs(nsf_plan p, int nev, double res_tol, double cg_rtol, int max_basis, int max_restarts,
             unsigned long long seed, double* omega_host, nsf_c128* Y_dev, double* resid_host,
             nsf_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p || !omega_host) return set_error(p, NSF_E_ARG, "NULL argument");
  Run r;
  int rc = make_run(p, nev, res_tol, cg_rtol, max_basis, max_restarts, seed, r);
  if (rc) return rc;
  std::vector<Run*> runs{&r};
  rc = run_engine(runs, p->stream);
  if (rc) return rc;
  auto tr = std::chrono::steady_clock::now();
  if ((rc = refine_run(&r))) return rc;
  r.st.ms_restart += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tr).count();
  if ((rc = verify_run(p, r, max_basis, max_restarts, seed))) return rc;
  if (Y_dev)
    NSF_HIP(p, hipMemcpyAsync(Y_dev, r.V, sizeof(double2) * (size_t)nev * r.len, hipMemcpyDeviceToDevice, p->stream));
  NSF_HIP(p, hipStreamSynchronize(p->stream));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  finish_run(r, omega_host, resid_host, stats, ms);
  const int status = r.converged ? NSF_OK : NSF_NOT_CONVERGED;
  trace_solve("nsf_eigs", p, 0, nev, status, r.st, r.eta.data());
  return status;
}

int nsf_batch_create(nsf_batch* out, int count, const int* grids, const double* ks, double a, double alpha,
                     double beta, void* hip_stream) {
  if (!out) return set_error(nullptr, NSF_E_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1 || !grids || !ks) return set_error(nullptr, NSF_E_ARG, "bad batch arguments");
  auto* b = new (std::nothrow) nsf_batch_s();
  if (!b) return set_error(nullptr, NSF_E_NOMEM, "host allocation failed");
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < count; ++i) {
    nsf_plan p = nullptr;
    const int rc = nsf_plan_create(&p, grids[3 * i], grids[3 * i + 1], grids[3 * i + 2], a, ks + 3 * i, alpha,
                                   beta, hip_stream);
    if (rc) {
      const std::string msg = "instance " + std::to_string(i) + ": " + nsf_last_error(nullptr);
      nsf_batch_destroy(b);
      return set_error(nullptr, rc, msg);
    }
    b->plans.push_back(p);
  }
  *out = b;
  return NSF_OK;
}

void nsf_batch_destroy(nsf_batch b) {
  if (!b) return;
  for (nsf_plan p : b->plans) nsf_plan_destroy(p);
  delete b;
}

int nsf_batch_autotune(nsf_batch b, int reps, int* shapes_tuned) {
  if (!b) return set_error(nullptr, NSF_E_ARG, "batch is NULL");
  std::map<std::tuple<int, int, int>, nsf_plan> tuned;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    nsf_plan p = b->plans[i];
    const Geom& g = p->geom;
    const auto key = std::make_tuple(g.n1, g.n2, g.n3);
    auto it = tuned.find(key);
    if (it == tuned.end()) {
      p->stream = b->stream;
      const int rc = nsf_plan_autotune(p, reps, nullptr);
      if (rc) return set_error(nullptr, rc, "instance " + std::to_string(i) + ": " + p->last_error);
      tuned[key] = p;
    } else {
      const nsf_plan q = it->second;
      p->opt_fft_path = q->opt_fft_path;
      p->opt_mid_cols = q->opt_mid_cols;
      p->geom.x_rows = q->geom.x_rows;
      p->geom.yz_cols = q->geom.yz_cols;
      p->geom.mid_pairs = q->geom.mid_pairs;
    }
  }
  if (shapes_tuned) *shapes_tuned = (int)tuned.size();
  return NSF_OK;
}

int nsf_eigs_set_start(nsf_plan p, const nsf_c128* Y0_dev, int count) {
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (count < 0 || count > 512 || (count > 0 && !Y0_dev))
    return set_error(p, NSF_E_ARG, "start block: 0 <= count <= 512 device vectors");
  p->start_Y = count ? reinterpret_cast<const double2*>(Y0_dev) : nullptr;
  p->start_count = count;
  return NSF_OK;
}

int nsf_batch_plan(nsf_batch b, int i, nsf_plan* plan) {
  if (!b || !plan || i < 0 || i >= (int)b->plans.size()) return set_error(nullptr, NSF_E_ARG, "bad batch index");
  *plan = b->plans[i];
  return NSF_OK;
}

int nsf_batch_eigs(nsf_batch b, int nev, double res_tol, double cg_rtol, int max_basis, int max_restarts,
                   unsigned long long seed, double* omega_host, double* resid_host, nsf_stats* stats,
                   nsf_c128* const* Y_dev, int* wave_size) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!b || !omega_host) return set_error(nullptr, NSF_E_ARG, "NULL argument");
  const int B = (int)b->plans.size();
  // Instances of kSoloVoxels or more fill the GPU on their own (every pass
  // streams HBM at 5-6 TB/s), so sharing launches would only add lock-step
  // waits: each runs as a wave of its own, exactly as nsf_eigs.  The others
  // run in shared waves that fit in device memory: fields 6n, CG and Lanczos
  // vectors 6 x 4n, kept CG directions kCgRing x 4n, basis 2 (m+1) x 4n, medium
  // n complex each.
  const int m = max_basis > 0 ? max_basis : std::max(3 * nev, nev + 8);
  size_t free_b = 0, total_b = 0;
  NSF_HIP(b->plans[0], hipMemGetInfo(&free_b, &total_b));
  std::vector<int> shared, solo;
  double need_max = 0;
  for (int i = 0; i < B; ++i) {
    const double n = (double)b->plans[i]->geom.n;
    if (b->plans[i]->geom.n >= kSoloVoxels) {
      solo.push_back(i);
      continue;
    }
    shared.push_back(i);
    need_max = std::max(need_max, 16.0 * n * (6 + 24 + 4.0 * kCgRing + 8.0 * (m + 1) + 1) + (64 << 20));
  }
  int wave = shared.empty() ? 1 : (int)std::max(1.0, std::floor(0.85 * (double)free_b / need_max));
  wave = std::min(wave, std::max((int)shared.size(), 1));
  if (wave_size) *wave_size = wave;
  std::vector<std::vector<int>> waves;
  for (size_t w0 = 0; w0 < shared.size(); w0 += (size_t)wave)
    waves.emplace_back(shared.begin() + w0, shared.begin() + std::min(shared.size(), w0 + (size_t)wave));
  for (int i : solo) waves.push_back({i});
  int worst = NSF_OK;
  // NSF_OPT_WARM_CHAIN: the Ritz vectors of the instance solved last, kept for
  // the next instance when that one asks for them and has the same grid
  double2* chain = nullptr;
  size_t chain_bytes = 0;
  int chain_from = -1;
  auto same_grid = [&](int i, int j) {
    const Geom &a = b->plans[i]->geom, &c = b->plans[j]->geom;
    return a.n1 == c.n1 && a.n2 == c.n2 && a.n3 == c.n3;
  };
  struct ChainFree {
    double2** ptr;
    ~ChainFree() {
      if (*ptr) hipFree(*ptr);
    }
  } chain_free{&chain};
  for (size_t wv = 0; wv < waves.size(); ++wv) {
    const std::vector<int>& ids = waves[wv];
    std::vector<Run> runs(ids.size());
    std::vector<Run*> ptrs;
    for (size_t j = 0; j < ids.size(); ++j) {
      const int i = ids[j];
      nsf_plan p = b->plans[i];
      p->stream = b->stream;
      if (p->opt_warm_chain && chain && chain_from == i - 1 && same_grid(i, i - 1)) {
        p->start_Y = chain;
        p->start_count = nev;
      }
      const int rc = make_run(p, nev, res_tol, cg_rtol, max_basis, max_restarts, seed + 1000003ULL * i, runs[j]);
      if (rc) return set_error(nullptr, rc, "instance " + std::to_string(i) + ": " + p->last_error);
      ptrs.push_back(&runs[j]);
    }
    const int rc = run_engine(ptrs, b->stream);
    if (rc) return set_error(nullptr, rc, std::string("batch: ") + ptrs[0]->p->last_error);
    for (size_t j = 0; j < ids.size(); ++j) {
      const int i = ids[j];
      Run& r = runs[j];
      int rr = refine_run(&r);
      if (!rr) rr = verify_run(r.p, r, max_basis, max_restarts, seed + 1000003ULL * i);
      if (rr) return set_error(nullptr, rr, "instance " + std::to_string(i) + ": " + b->plans[i]->last_error);
      if (Y_dev && Y_dev[i])
        NSF_HIP(r.p, hipMemcpyAsync(Y_dev[i], r.V, sizeof(double2) * (size_t)nev * r.len, hipMemcpyDeviceToDevice,
                                    b->stream));
      // instance i + 1 runs in a later wave (waves keep index order within the
      // shared and the solo instances)
      if (i + 1 < B && b->plans[i + 1]->opt_warm_chain && same_grid(i, i + 1) &&
          std::find(ids.begin(), ids.end(), i + 1) == ids.end()) {
        const size_t bytes = sizeof(double2) * (size_t)nev * r.len;
        if (bytes > chain_bytes) {
          if (chain) NSF_HIP(r.p, hipFree(chain));
          chain = nullptr;
          NSF_HIP(r.p, hipMalloc(&chain, bytes));
          chain_bytes = bytes;
        }
        NSF_HIP(r.p, hipMemcpyAsync(chain, r.V, bytes, hipMemcpyDeviceToDevice, b->stream));
        chain_from = i;
      }
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (size_t j = 0; j < ids.size(); ++j) {
      const int i = ids[j];
      Run& r = runs[j];
      finish_run(r, omega_host + (size_t)i * nev, resid_host ? resid_host + (size_t)i * nev : nullptr,
                 stats ? stats + i : nullptr, ms);
      if (!r.converged) worst = NSF_NOT_CONVERGED;
      trace_solve("nsf_batch_eigs", r.p, i, nev, r.converged ? NSF_OK : NSF_NOT_CONVERGED, r.st, r.eta.data());
    }
    // free this wave's Lanczos storage before the next wave
    if (wv + 1 < waves.size())
      for (int i : ids) {
        nsf_plan p = b->plans[i];
        if (p->ws) continue;  // caller-provided storage stays
        NSF_HIP(p, hipStreamSynchronize(b->stream));
        if (p->d_basis) NSF_HIP(p, hipFree(p->d_basis));
        p->d_basis = nullptr;
        p->basis_vectors = 0;
        if (p->d_cg) NSF_HIP(p, hipFree(p->d_cg));
        p->d_cg = nullptr;
        if (p->d_ring) NSF_HIP(p, hipFree(p->d_ring));
        p->d_ring = nullptr;
      }
  }
  return worst;
}

}  // extern "C"
