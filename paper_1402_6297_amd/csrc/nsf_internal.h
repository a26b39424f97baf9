// Internal declarations shared by the HIP sources of libnsf.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "nsf.h"

namespace nsf {

constexpr int kMaxAxis = 512;    // longest supported axis (six fields of one pencil fit a tile)
constexpr int kMaxStages = 10;   // radix stages per axis
constexpr int kThreads = 256;    // threads per workgroup of the FFT passes
constexpr int kEpt = 16;         // complex elements per thread held in registers

// ---------------------------------------------------------------- complex ops
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i * a
__host__ __device__ inline double2 cmuli(double2 a) { return make_double2(-a.y, a.x); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ FFT plan
// Mixed-radix Stockham factorisation of one axis (radices 8, 4, 2, 3, 5).
struct AxisPlan {
  int N;
  int nst;
  int radix[kMaxStages];
};

// Per-frequency basis data needs the three per-axis lambda tables; the twist
// tables d_l(j) = exp(i 2 pi k_l a j / n_l) are needed only by P_r, Q_r alone.
struct Tables {
  const double2* lam;    // n1 + n2 + n3 values: lambda_1 | lambda_2 | lambda_3
  const double2* twist;  // n1 + n2 + n3 values: d_1 | d_2 | d_3
  const double2* tw;     // n1 + n2 + n3 FFT roots exp(+2 pi i m / n_l) per axis
};

struct Geom {
  int n1, n2, n3;
  long long n;
  double alpha, beta;
  // launch tiling of the two-level passes (tuning only; results do not depend on it)
  int x_rows = 4;    // rows per workgroup of the x passes (1, 2, 4; lowered to fit)
  int yz_cols = 16;  // pencils per workgroup of the y / z passes (1..16, lowered to fit)
  int mid_pairs = 1; // fused z pass: 1 one field pair per workgroup, 0 all six fields
};

enum MediumKind { kMedNone = 0, kMedChiral = 1, kMedPseudo = 2, kMedGeneral = 3, kMedNfsep = 4 };

// Entries of the general per-voxel middle factor kept per voxel: the upper
// triangle of a 6 x 6 Hermitian matrix, row by row.
constexpr int kGenEntries = 21;
// Entries of the NFSEP per-voxel factor i J B^{-1}: a full 6 x 6 matrix, row-major.
constexpr int kFullEntries = 36;

// Algorithmic HBM bytes per voxel of one apply besides the medium: read the 4n
// input (64), write and read six fields (96 + 96), write the 4n output (64).
// The medium adds medium_voxel_bytes (576 for NFSEP factors per voxel, 2 with
// a palette).
constexpr int kNfsepFieldBytesPerVoxel = 320;

// Largest palette of distinct per-voxel factors (general and NFSEP media); a
// medium with more distinct voxels keeps its factors per voxel.
constexpr int kPaletteMax = 4096;

// Media whose per-voxel factor couples all six field components (no pair passes).
inline bool six_coupled(int kind) { return kind == kMedGeneral || kind == kMedNfsep; }

struct MediumView {
  int kind;
  int pa, pb, po;        // pseudochiral coupled axes and the third axis
  const double2* eg;     // per voxel (eps, gamma)
  const double2* mg;     // general media: kGenEntries per voxel (or per palette entry)
  const double2* mf;     // NFSEP media: kFullEntries per voxel (or per palette entry)
  const unsigned short* pidx;  // palette index per voxel, or null (factors stored per voxel)
  // tiles of the field-pair z pass (P columns of one y, index x / P + (n1 / P) y)
  // holding a voxel that is not vacuum, for the plan's current P; used only by
  // a vacuum-skipping launch
  const int* ztiles;
  int nztiles;
  // groups of consecutive x (the y pass's pencils per workgroup, index x / P)
  // holding a voxel that is not vacuum, for a vacuum-skipping y pass
  const int* xgroups;
  int nxgroups;
};

// Which half of the synthesis / projection a pass performs.
enum BasisPart { kPartBoth = 0, kPartP = 1, kPartQ = 2 };

// ------------------------------------------------------------- launch layer
// All launchers enqueue on `s` and return hipError_t of the launch.
// `skip` (nullable, device): when *skip != 0 every workgroup exits at once.

// Synthesis (P_r / Q_r coefficients) fused with the inverse x-FFT.
// y: [y_a; y_b; y_c; y_d] blocks (n each); part selects which blocks are read
// and which fields are written: kPartBoth -> fld[0..5]; kPartP -> fld[0..2]
// from (y_a, y_b) = y[0], y[n]; kPartQ -> fld[0..2] from (y_c, y_d) passed as
// y[0], y[n].
hipError_t launch_x_inv_synth(const Geom& g, const AxisPlan& ax, const Tables& t,
                              int part, const double2* y, double2* fld,
                              const int* skip, hipStream_t s);

// Plain FFT along y (axis 1) or z (axis 2) of nf fields in place.
// dir = +1 inverse (e^{+}), -1 forward (e^{-}).  post_twist: multiply the result
// by D_g / sqrt(n) (inverse z pass of P_r / Q_r).  pre_twist: multiply the input
// by conj(D_g) / sqrt(n) (forward z pass of P_r^* / Q_r^*).
hipError_t launch_yz_pass(const Geom& g, const AxisPlan& ax, const Tables& t, int axis,
                          int dir, int nf, double2* fld, int post_twist, int pre_twist,
                          const int* skip, hipStream_t s);

// Inverse z-FFT, per-voxel constitutive step (times 1/n), forward z-FFT of the
// six fields [E'x E'y E'z H'x H'y H'z] in place.
hipError_t launch_z_mid(const Geom& g, const AxisPlan& ax, const Tables& t,
                        const MediumView& med, double2* fld, const int* skip,
                        hipStream_t s);

// Forward x-FFT fused with the projection P_r^* / Q_r^*.  kPartBoth: fields
// 0..5 -> out blocks a, b, c, d; kPartP: fields 0..2 -> out blocks a, b;
// kPartQ: fields 0..2 -> out blocks c, d (written at out[0], out[n]).
hipError_t launch_x_fwd_proj(const Geom& g, const AxisPlan& ax, const Tables& t,
                             int part, const double2* fld, double2* out,
                             const int* skip, hipStream_t s);

// Register-resident fast path for axis lengths with a two-level split
// (16, 32, 48, 64, 96, 128, 256); same semantics as the generic launchers.
bool fast_axis(int N);
// With insts != nullptr the launch covers ninst instances (grid z) and every
// pointer argument is ignored in favour of the descriptors.
hipError_t launch_fast_x_inv_synth(const Geom& g, const Tables& t, int part, const double2* y,
                                   double2* fld, const int* skip, hipStream_t s,
                                   const struct InstDesc* insts = nullptr, int ninst = 1);
// ysc > 0 (vacuum skipping, axis 1 only): transform only the x groups listed in
// xg (nxg of them; batched: each instance's med.xgroups, nxg the largest
// count) and scale the results by ysc.
hipError_t launch_fast_yz(const Geom& g, const Tables& t, int axis, int dir, int nf, double2* fld,
                          int post_twist, int pre_twist, const int* skip, hipStream_t s,
                          const struct InstDesc* insts = nullptr, int ninst = 1, const int* xg = nullptr,
                          int nxg = -1, double ysc = 0.0);
// Pencils (consecutive x) per workgroup of the two-level y (axis 1) or z pass.
int fast_yz_cols(const Geom& g, int axis);
// With np_mid given and the field-pair kernel in use, also writes per-workgroup
// partials of Re p^* A_r p (the fields' real-space quadratic form) to part_mid
// (batched: to each descriptor's cg.part_mid) and sets *np_mid to their count;
// otherwise *np_mid = 0.
// vac_scale > 0 (vacuum skipping, field-pair kernel only): only the
// med.ztiles tiles are transformed (vac_tiles workgroup triples: the listed
// count, or the largest over a batch), scaled by vac_scale = 1 / n3; the
// partials hold Re f^* (M - I) f / n.  The forward y and x passes must then
// scale by 1 / n2 and 1 / n1 (launch_fast_yz ysc, pscale).
hipError_t launch_fast_z_mid(const Geom& g, const Tables& t, const MediumView& med, double2* fld,
                             int P_want, const int* skip, hipStream_t s,
                             const struct InstDesc* insts = nullptr, int ninst = 1,
                             double* part_mid = nullptr, int* np_mid = nullptr, double vac_scale = 0.0,
                             int vac_tiles = -1);
// Pencil columns per workgroup of the field-pair z pass (0: that kernel is not used).
int fast_z_pair_cols(const Geom& g, int medium_kind, int P_want);
hipError_t launch_fast_x_fwd_proj(const Geom& g, const Tables& t, int part, const double2* fld,
                                  double2* out, const int* skip, hipStream_t s,
                                  const struct InstDesc* insts = nullptr, int ninst = 1, double pscale = 1.0);

// Single-wave passes holding E' / H' components per lane (axis lengths 16,
// 32, 64, 128); same semantics again.
bool wave_axis(int N);
bool wave_mid_ok(const Geom& g);
hipError_t launch_wave_x_inv_synth(const Geom& g, const Tables& t, int part, const double2* y,
                                   double2* fld, const int* skip, hipStream_t s);
hipError_t launch_wave_z_mid(const Geom& g, const Tables& t, const MediumView& med, double2* fld,
                             const int* skip, hipStream_t s);
hipError_t launch_wave_x_fwd_proj(const Geom& g, const Tables& t, int part, const double2* fld,
                                  double2* out, const int* skip, hipStream_t s);

// out = B_r u (Thm 4.2): per frequency 1/sigma_f times i / -i block swaps.
hipError_t launch_apply_Br(const Geom& g, const Tables& t, const double2* u, double2* out,
                           const int* skip, hipStream_t s);

// -------------------------------------------------------------- BLAS layer
constexpr int kRedBlocks = 1024;       // partial-sum slots for one reduction
constexpr int kPartialSlots = 131072;  // partial-sum slots of the multi-vector dot (512 x 256)
constexpr int kCoefSlots = 1024;       // device coefficient vector of the Lanczos steps
constexpr int kResSlots = 1100;        // reduction results (and host copies of coefficients)
constexpr int kMidSlots = 32768;       // doubles x 2: partials of the fused z pass

// Directions kept by the q-free CG in place of updating x every iteration:
// x = x0 + sum_j alpha_j p_j is folded in every kCgRing iterations.
constexpr int kCgRing = 16;

struct CgState {
  double rr;        // r^* r of the current iterate
  double thresh;    // (rtol ||b||)^2
  double bb;        // ||b||^2
  double alpha, beta;
  int iter, maxit;
  int done;         // nonzero: every CG kernel exits at once
  int status;       // NSF_OK / NSF_NOT_CONVERGED / NSF_E_BREAKDOWN
  int ring;         // directions kept (0: x is updated every iteration)
  int bd_step;      // 1: the breakdown happened inside an iteration (its p was written)
  int pad;
  double pap;       // p^* A_r p of the current direction (q-free fused schedule)
  double ahist[kCgRing];  // alpha_j of the kept directions, slot j mod ring
};

// Vectors and device scalars of a CG solve whose recurrences are fused into
// the first and last FFT pass of each A_r apply (see launch_fast_cg_*).
struct CgFuse {
  double2* x;
  double2* r;
  double2* p;
  double2* q;
  double2* ring;     // q-free with kept directions: slot j (4n each) holds p_j, j mod ring
  CgState* st;
  double* part_in;   // per-workgroup |r|^2 of the first pass
  double* part_out;  // per-workgroup (Re p^*q, |q|^2, Re r^*q) of the last pass
  double* part_mid;  // per-workgroup Re p^* A_r p of the fused z pass (field pairs)
  int pnorm;         // q-free: the first pass writes per-workgroup |p|^2 to part_in (vacuum skipping)
};

// Per-instance pointers of a batched launch (instances of one grid shape):
// block index z selects the instance.  Kernels given a descriptor array take
// every pointer below from it instead of from their own arguments.
struct InstDesc {
  Tables t;
  MediumView med;
  double2* fld;         // six-field workspace
  const double2* vin;   // input 4n vector of a plain apply
  double2* vout;        // output 4n vector of a plain apply
  const int* skip;      // nonzero: the instance is finished (CG done flag)
  CgFuse cg;
};

// First pass of a fused CG iteration: for iter > 0 it forms
// r = r - alpha q, x = x + alpha p, p = r + beta p (with alpha, beta of the
// previous iteration), writes them and the per-workgroup |r|^2, then
// synthesises from p exactly like launch_fast_x_inv_synth.  Returns the
// number of workgroups through *nparts.
//
// q-free form (qfree = true), used when the fused z pass sums p^* A_r p: the
// first pass forms x = x + alpha p, p = r + beta p only (r was already updated
// by the last pass) and writes no partial sums.
int fast_x_rows(const Geom& g);
hipError_t launch_fast_cg_first(const Geom& g, const Tables& t, const CgFuse& cg, double2* fld,
                                const int* skip, int* nparts, hipStream_t s,
                                const InstDesc* insts = nullptr, int ninst = 1, bool qfree = false);
// Workgroups of the fused z pass that sum p^* A_r p for this geometry and
// medium kind (0: that pass sums nothing, so the q-free schedule is off).
int fast_z_mid_pq_items(const Geom& g, int medium_kind, int P_want);
// The same decision for a plan's own z pass (pass_z_mid).
int z_mid_pq_items(nsf_plan p);
bool cg_qfree(nsf_plan p);
// Last pass: q = projection of the forward x transform (written to cg.q) and
// the per-workgroup partial sums of p^*q, |q|^2, r^*q.
// pq_done (the q-free form): the fused z pass already produced p^* A_r p and
// launch_cgf_alpha turned it into cg.st->pap; the pass forms q on the fly, sets
// r = r - alpha q with alpha = rr / pap, writes r (not q) and the per-workgroup
// |r|^2.
hipError_t launch_fast_cg_last(const Geom& g, const Tables& t, const CgFuse& cg, const double2* fld,
                               const int* skip, int* nparts, hipStream_t s,
                               const InstDesc* insts = nullptr, int ninst = 1, bool pq_done = false,
                               double pscale = 1.0);
// Scalar steps of the fused CG: check |r|^2 after the first pass, then alpha,
// beta from the last pass (|r - alpha q|^2 by expansion).
// Batched forms (insts != nullptr): one workgroup per instance, partials and
// state taken from insts[i].cg.
hipError_t launch_cgf_check(const double* part_in, int nparts, CgState* st, hipStream_t s,
                            const InstDesc* insts = nullptr, int ninst = 1);
hipError_t launch_cgf_step(const double* part_out, int nparts, CgState* st, hipStream_t s,
                           const InstDesc* insts = nullptr, int ninst = 1,
                           const double* part_mid = nullptr, int np_mid = 0);
// q-free schedule: after the fused z pass, st->pap = sum of its partials; after
// the last pass, |r|^2 from its partials, alpha = rr / pap, beta = |r_new|^2 / rr,
// the convergence test, iter + 1.  launch_cg_finish then applies the pending
// x = x + alpha p of the final iteration once the state is done (not after a
// breakdown).
// With np_in > 0 (vacuum skipping) pap also adds the first pass's |p|^2 partials.
hipError_t launch_cgf_alpha(const double* part_mid, int np_mid, CgState* st, hipStream_t s,
                            const InstDesc* insts = nullptr, int ninst = 1, const double* part_in = nullptr,
                            int np_in = 0);
hipError_t launch_cgf_step_qf(const double* part_out, int nparts, CgState* st, hipStream_t s,
                              const InstDesc* insts = nullptr, int ninst = 1);
hipError_t launch_cg_finish(double2* x, const double2* p, long long len, const CgState* st, hipStream_t s);
// Kept directions (CgState::ring > 0): x += sum alpha_j p_j over the ring.
// final = false, inside an iteration after launch_cgf_alpha: folds all ring
// slots when this iteration fills the ring (its alpha = rr / pap, 0 when pap
// is not positive).  final = true, once the solve has ended: folds the slots
// written since the last fold.  Batched form: x, ring, st from insts[i].cg.
hipError_t launch_cg_fold(double2* x, const double2* ring, long long len, const CgState* st, bool final,
                          hipStream_t s, const InstDesc* insts = nullptr, int ninst = 1);

// partial[blk] = sum conj(x) y over a fixed slice (complex, as double2).
hipError_t launch_dot_partials(const double2* x, const double2* y, long long len,
                               double2* partial, const int* skip, hipStream_t s);
// x = 0 and r = p = b - sum_{j<m} c_j AV_{idx_j} (c on device: m coefficients,
// then the m indices as doubles in .x; m <= 512; plain r = b when m = 0); the
// stopping threshold stays relative to ||b||.  ring > 0: the q-free CG keeps
// that many directions (p is then ring slot 0).
hipError_t launch_cg_init(const double2* b, double2* x, double2* r, double2* p, long long len,
                          double2* partial, CgState* st, double rtol, int maxit, hipStream_t s,
                          const double2* AV = nullptr, long long ld = 0, int m = 0,
                          const double2* c = nullptr, int ring = 0);
hipError_t launch_cg_alpha(const double2* partial, int nparts, CgState* st, hipStream_t s);
hipError_t launch_cg_update(double2* x, double2* r, const double2* p, const double2* q,
                            long long len, double2* partial, CgState* st, hipStream_t s);
hipError_t launch_cg_beta(const double2* partial, int nparts, CgState* st, hipStream_t s);
// Number of partial sums the reductions above write for a vector of length len.
int reduce_parts_for(long long len);
hipError_t launch_cg_p(double2* p, const double2* r, long long len, CgState* st, hipStream_t s);

// Multi-vector kernels for the Lanczos basis (vectors at stride ld).
// c[i] = sum_e conj(V_i[e]) w[e], i < m, written as m complex values to out.
hipError_t launch_multi_dot(const double2* V, long long ld, int m, const double2* w, long long len,
                            double2* partial, double2* out, hipStream_t s);
// out[0..m) = V^* w1 and out[m..2m) = V^* w2 in one pass over V (m <= 256).
hipError_t launch_multi_dot2(const double2* V, long long ld, int m, const double2* w1, const double2* w2,
                             long long len, double2* partial, double2* out, hipStream_t s);
// One pass over the frequencies f of a Lanczos step's 4n vectors (components
// f, f + n, f + 2n, f + 3n; c, idx as for launch_cg_init, m <= 512):
//   mode 0: z = b - r - sum_k c_k AV_{idx_k}, the image A_r x of a CG solution x
//           of A_r x = b started from the projected guess (r its final residual);
//   mode 1: w -= sum_k c_k V_{idx_k}, z -= sum_k c_k AV_{idx_k} (a Gram-Schmidt
//           update over a few basis columns);
// then b = B_r w (b may be the right-hand side read in mode 0: each thread reads
// its frequency before writing it), res2[0] = w^* z and res2[1] = w^* B_r w
// (device; the partial sums use `partial`, 2 x 2048 slots).
hipError_t launch_step_fused(const Geom& g, const Tables& t, int mode, double2* w, double2* z, double2* b,
                             const double2* r, const double2* V, const double2* AV, long long ld, int m,
                             const double2* c, double2* partial, double2* res2, hipStream_t s);
// w = wscale (w - sum_i c[i] V_i) and, if V2 is given, z -= sum_i c[i] V2_i
// (c on device, m <= 512).
hipError_t launch_multi_axpy(const double2* V, long long ld, int m, const double2* c, double2* w,
                             long long len, hipStream_t s, const double2* V2 = nullptr,
                             double2* z = nullptr, double wscale = 1.0);
// V[:, 0:k] = V[:, 0:m] S (S device, m x k column-major complex), in place.
hipError_t launch_rotate(double2* V, long long ld, int m, int k, const double2* S, long long len,
                         hipStream_t s);
// y = a * x  (complex scalar on host)
hipError_t launch_scale_copy(const double2* x, double2* y, double sre, double sim, long long len,
                             hipStream_t s);
// Complex normal vector from a counter-based hash of (seed, index).
hipError_t launch_randn(double2* v, long long len, unsigned long long seed, hipStream_t s);
// out[0] = sum |B u - theta A u|^2, out[1] = sum |A u|^2, with Bu computed on the fly.
hipError_t launch_residual_norms(const Geom& g, const Tables& t, const double2* u,
                                 const double2* Au, double theta, double2* partial,
                                 double* out2, hipStream_t s);
// Reduce kRedBlocks complex partials to one complex value at out.
hipError_t launch_reduce_partials(const double2* partial, int nparts, double2* out, hipStream_t s);

// Gradient accumulation (chiral): after the inverse passes have produced
// E', H' (spatial fields with the 1/sqrt(n) scaling), accumulate
// d_eps += w*omega*(...), d_gamma += w*omega*(...).
hipError_t launch_grad_accum(const Geom& g, const double2* eg, const double2* fld, double wo,
                             double* d_eps, double* d_gamma, int first, hipStream_t s);

}  // namespace nsf

// The opaque plan.
struct nsf_plan_s {
  nsf::Geom geom;
  double a;
  double k[3];
  double delta[3];
  nsf::AxisPlan ax[3];
  hipStream_t stream = nullptr;
  int device = -1;
  bool dev_ready = false;
  double sigma_min = 0, sigma_max = 0;

  // host tables
  std::vector<double2> h_lam, h_twist, h_tw;
  // device tables
  double2* d_tables = nullptr;  // lam | twist | tw
  nsf::Tables tabs{};

  // medium
  int medium_kind = nsf::kMedNone;
  int pa = 0, pb = 1, po = 2;
  double2* d_medium = nullptr;  // (eps, gamma) per voxel
  double2* d_mgen = nullptr;    // general media: 6x6 middle factor per voxel (upper triangle)
  double2* d_mfull = nullptr;   // NFSEP media: 6x6 factor i J B^{-1} per voxel (row-major)
  unsigned short* d_pidx = nullptr;  // palette index per voxel (general / NFSEP media)
  int palette = 0;              // distinct voxel factors in the palette, 0: stored per voxel

  // workspace
  double2* d_fields = nullptr;  // 6 n
  double2* d_cg = nullptr;      // x r p q : 4 x 4n (cg scratch)
  double2* d_partial = nullptr; // kPartialSlots partial sums
  double2* d_coef = nullptr;    // kCoefSlots complex coefficients (multi-dot results)
  double2* d_res = nullptr;     // kResSlots complex reduction results
  double2* h_res = nullptr;     // pinned host mirror of d_res
  double2* d_small = nullptr;   // small dense matrices (Ritz rotations)
  size_t small_cap = 0;
  nsf::CgState* d_state = nullptr;
  nsf::CgState* h_state = nullptr;  // pinned
  int* d_flags = nullptr;           // misc device ints
  int* h_flags = nullptr;           // pinned

  // Lanczos basis storage
  double2* d_basis = nullptr;  // V and AV
  size_t basis_vectors = 0;    // capacity of V (and of AV)

  // start block for the next eigensolve (nsf_eigs_set_start; caller-owned)
  const double2* start_Y = nullptr;
  int start_count = 0;

  // caller-provided workspace (nsf_plan_set_workspace): fields, CG vectors,
  // basis and small matrices are carved from it and never freed by the plan
  char* ws = nullptr;
  size_t ws_bytes = 0;

  // options (nsf_plan_set_option)
  int opt_fft_path = 0;     // 0 auto, 1 generic LDS-staged, 2 two-level without single-wave
  int opt_mid_cols = 16;    // pencils per workgroup of the fused z pass
  int opt_cg_graph = 1;     // CG iterations of the eigensolver replayed from a HIP graph
  int opt_cg_start = 1;     // eigensolver CG starts from the Galerkin solution in span(V)
  int opt_verify = 0;       // multiplicity checks after convergence (nsf_eigs)
  int opt_ortho_gate = 1;   // skip negligible Gram-Schmidt updates on the device
  int opt_gmres_restart = 12;  // GMRES restart length of the NFSEP eigensolver
  int opt_palette = 1;      // general / NFSEP media: palette of distinct voxel factors
  int opt_cg_relax = 0;     // eigensolver inner CG tolerance relaxed with the Ritz residuals
  int opt_warm_chain = 0;   // nsf_batch_eigs: start from the previous instance's Ritz vectors
  int opt_cg_ring = 1;      // q-free CG keeps kCgRing directions instead of updating x
  double2* d_ring = nullptr;  // those directions, kCgRing x 4n
  int opt_vacuum = 1;       // the field-pair z pass leaves out columns of vacuum

  // z-pass tiles that are not all vacuum (chiral and pseudochiral media), one
  // list per P = 1, 2, 4, 8, 16 columns per tile, built when the medium is set
  int* d_ztiles = nullptr;
  int ztile_off[5] = {0, 0, 0, 0, 0};
  int ztile_cnt[5] = {-1, -1, -1, -1, -1};
  int xgrp_off[5] = {0, 0, 0, 0, 0};    // x groups with a voxel other than vacuum, same buffer
  int xgrp_cnt[5] = {-1, -1, -1, -1, -1};
  size_t ztile_cap = 0;     // ints allocated at d_ztiles

  std::string last_error;
};

// Return the library status of a failed HIP call from the enclosing function.
#define NSF_HIP(p, call)                                      \
  do {                                                        \
    const int _rc = ::nsf::hip_check((p), (call), #call);     \
    if (_rc != NSF_OK) return _rc;                            \
  } while (0)

namespace nsf {
// Host helpers (plan.hip)
int ensure_device(nsf_plan p);
int set_error(nsf_plan p, int code, const std::string& msg);
int hip_check(nsf_plan p, hipError_t e, const char* what);
// NSF_SYNC_CHECK set (not "0"): every checked HIP call is followed by a device
// synchronisation and its error check (debugging; graph capture is then off).
bool debug_sync();
// Medium bytes per voxel an apply reads (nsf_plan_medium_info's voxel_bytes).
long long medium_voxel_bytes(nsf_plan p);
// NSF_TRACE set: one JSON line per finished eigensolve (per instance of a
// batch) with the counters and phase times, to stderr ("1" or "stderr") or
// appended to the named file.
void trace_solve(const char* call, nsf_plan p, int instance, int nev, int status, const nsf_stats& st,
                 const double* resid);
MediumView medium_view(nsf_plan p);
int apply_Ar_dev(nsf_plan p, const double2* u, double2* out, const int* skip);
// Vacuum skipping of the plan's A_r passes (opt_vacuum, a chiral or
// pseudochiral medium, every axis on the two-level passes, the field-pair z
// pass): the z pass transforms only the listed tiles, scaled by 1 / n3; both
// y passes only the listed x groups, the forward one scaled by 1 / n2; the
// projection scales by 1 / n1.
struct VacSkip {
  bool on = false;
  double zscale = 0.0, pscale = 1.0, yscale = 0.0;
  int ntiles = -1;  // listed z-pass tiles
  int nxg = -1;     // listed y-pass x groups
};
VacSkip vac_of(nsf_plan p);
// Pass dispatch (fast path when the axis allows it, else generic).
hipError_t pass_x_inv(nsf_plan p, int part, const double2* y, double2* fld, const int* skip);
hipError_t pass_yz(nsf_plan p, int axis, int dir, int nf, double2* fld, int post_twist, int pre_twist,
                   const int* skip, const VacSkip* vac = nullptr);
hipError_t pass_z_mid(nsf_plan p, double2* fld, const int* skip, double* part_mid = nullptr,
                      int* np_mid = nullptr, const VacSkip* vac = nullptr);
hipError_t pass_x_fwd(nsf_plan p, int part, const double2* fld, double2* out, const int* skip,
                      double pscale = 1.0);
// cgv: the three CG vectors r, p, q (4n each, consecutive); nullptr: the plan's own.
int cg_solve_dev(nsf_plan p, const double2* b, double2* x, double rtol, int maxit, int* iters,
                 double* relres, long long* matvecs, double2* cgv = nullptr);
// Bytes of the caller workspace for a basis of m + 1 vectors (fields, CG, V, A_r V, m x m).
size_t workspace_bytes(long long n, int m);
// Part of the caller workspace: 0 fields, 1 CG vectors, 2 basis (capacity in
// vectors to *basis_cap), 3 small matrices; nullptr when the plan has none.
double2* ws_part(nsf_plan p, int which, size_t* basis_cap = nullptr);
int ensure_cg(nsf_plan p);
int ensure_ring(nsf_plan p, bool want);
bool cg_fusable(nsf_plan p);
CgFuse cg_fuse_of(nsf_plan p, double2* x, double2* cgv = nullptr);
int cg_iteration(nsf_plan p, double2* x, bool fused, double2* cgv = nullptr);
int cg_predict(const CgState& h, double rr_prev, int it_prev, bool fused);
int ensure_basis(nsf_plan p, size_t vectors);
int ensure_small(nsf_plan p, size_t count);
int hermitian_eig(int m, const double2* H, double* w, double2* V);
}  // namespace nsf
