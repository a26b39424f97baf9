// The null space free eigenvalue problem for media outside the HHPD
// assumption (Thm 3.2; the else-branch of Algorithm 1; the opening of Sec. 4):
//
//   K y = omega y,   K = diag(S Q_r^*, S P_r^*) B^{-1} diag(P_r S, Q_r S),
//
// S = Sigma_r^{1/2}, B = i [[zeta, mu], [-eps, -xi]] per voxel.  K has no
// Hermitian structure; the paper names a shift-and-invert Arnoldi method at
// zero shift with a GMRES inner solve.
//
// Reformulation used here.  Store per voxel N = i J B^{-1} (J = [[0, I],
// [-I, 0]] on the E / H halves) and let Kern = diag(P_r^*, Q_r^*) N
// diag(P_r, Q_r): the A_r pipeline with N as its middle factor (under the HHPD
// assumption N is exactly A_r's middle factor and Kern = A_r).  Then
//   W = diag(Q_r^*, P_r^*) B^{-1} diag(P_r, Q_r) = (i J4) Kern,
// with (i J4)[a; b] = [i b; -i a] on the 2n halves (an involution), and for
// x = S' y (S' = diag(S, S)) the eigenproblem K y = omega y is
//   Kern^{-1} B_r x = omega^{-1} x,   B_r = i [[0, Sigma_r^{-1}], [-Sigma_r^{-1}, 0]],
// because (i J4) Sigma'^{-1} = B_r.  This is the zero-shift inverted operator;
// for HHPD media it is the invert Lanczos operator A_r^{-1} B_r (Thm 4.2).
// x is the vector Algorithm 1 obtains after its scaling step, so the fields
// of an eigenpair are B^{-1} diag(P_r, Q_r) x (nsf_fields).
//
// Solver: Krylov-Schur restarted Arnoldi (Euclidean inner product) on
// Kern^{-1} B_r, each step one restarted GMRES solve with Kern from zero;
// wanted Ritz values theta = 1/omega: positive real part, largest modulus.
// Each converged pair is finalised with exact applies: omega = y^* K y / y^* y
// and eta = ||K y - omega y|| / (|omega| ||y||), y = S'^{-1} x.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "nsf_internal.h"

namespace nsf {
namespace {

typedef std::complex<double> cd;
typedef std::chrono::steady_clock clk;

double ms_since(clk::time_point t0) {
  return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

inline cd C(double2 v) { return cd(v.x, v.y); }
inline double2 D2(cd v) { return make_double2(v.real(), v.imag()); }

// out = S'^{pw} in (ij = 0) or S'^{pw} (i J4) in (ij = 1), pw = +1/2 (pos) or
// -1/2, per frequency f with sigma(f)^2 = sum_l |lambda_l|^2.  In place is safe.
__global__ void k_sigma_pow(Geom g, Tables t, const double2* in, double2* out, int pos, int ij) {
  const long long n = g.n;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(f % g.n1);
    const int i2 = (int)((f / g.n1) % g.n2);
    const int i3 = (int)(f / ((long long)g.n1 * g.n2));
    const double s2 = cabs2(t.lam[i1]) + cabs2(t.lam[g.n1 + i2]) + cabs2(t.lam[g.n1 + g.n2 + i3]);
    const double q = sqrt(sqrt(s2));  // sigma^{1/2}
    const double w = pos ? q : 1.0 / q;
    const double2 a = in[f], b = in[n + f], c = in[2 * n + f], d = in[3 * n + f];
    if (ij) {
      out[f] = cscale(cmuli(c), w);
      out[n + f] = cscale(cmuli(d), w);
      out[2 * n + f] = cscale(cmuli(a), -w);
      out[3 * n + f] = cscale(cmuli(b), -w);
    } else {
      out[f] = cscale(a, w);
      out[n + f] = cscale(b, w);
      out[2 * n + f] = cscale(c, w);
      out[3 * n + f] = cscale(d, w);
    }
  }
}

// y = a x + b y
__global__ void k_axpby(const double2* __restrict__ x, double2* __restrict__ y, double2 a, double2 b,
                        long long len) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len;
       e += (long long)gridDim.x * blockDim.x)
    y[e] = cadd(cmul(a, x[e]), cmul(b, y[e]));
}

unsigned grid_for(long long len) {
  long long b = (len + 255) / 256;
  return (unsigned)std::min<long long>(std::max<long long>(b, 1), 8192);
}

hipError_t sigma_pow(nsf_plan p, const double2* in, double2* out, bool pos, bool ij) {
  hipLaunchKernelGGL(k_sigma_pow, dim3(grid_for(p->geom.n)), dim3(256), 0, p->stream, p->geom, p->tabs, in,
                     out, pos ? 1 : 0, ij ? 1 : 0);
  return hipGetLastError();
}

hipError_t axpby(nsf_plan p, const double2* x, double2* y, cd a, cd b, long long len) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(len)), dim3(256), 0, p->stream, x, y, D2(a), D2(b), len);
  return hipGetLastError();
}

// Enqueue x^* y into d_res[slot] and its host copy h_res[slot].
int dot_async(nsf_plan p, const double2* x, const double2* y, long long len, int slot) {
  NSF_HIP(p, launch_dot_partials(x, y, len, p->d_partial, nullptr, p->stream));
  NSF_HIP(p, launch_reduce_partials(p->d_partial, reduce_parts_for(len), p->d_res + slot, p->stream));
  NSF_HIP(p, hipMemcpyAsync(p->h_res + slot, p->d_res + slot, sizeof(double2), hipMemcpyDeviceToHost,
                            p->stream));
  return NSF_OK;
}

int sync(nsf_plan p) {
  NSF_HIP(p, hipStreamSynchronize(p->stream));
  return NSF_OK;
}

// Upload host coefficients to d_coef (blocking: the staging area is reused).
int upload_coef(nsf_plan p, const cd* c, int m) {
  double2* h = p->h_res + 64;
  for (int i = 0; i < m; ++i) h[i] = D2(c[i]);
  NSF_HIP(p, hipMemcpyAsync(p->d_coef, h, sizeof(double2) * m, hipMemcpyHostToDevice, p->stream));
  return sync(p);
}

// Second-pass thresholds of gram_schmidt on ||w_after||^2 / ||w_before||^2.
// One classical pass leaves components of about eps ||w_before|| along V, i.e.
// eps / ratio relative to the result.  The Arnoldi basis of the eigensolver
// keeps the Daniel-Gragg-Kaufman-Stewart rule (ratio 1/sqrt 2: orthogonal to
// rounding); the GMRES bases accept 10 eps (ratio 0.1), since their solves are
// checked by an explicitly recomputed residual.
constexpr double kReorthArnoldi = 0.5;
constexpr double kReorthGmres = 0.01;

// Classical Gram-Schmidt of w against V[0..m) where w is stored as V[m] (the
// next slot of the basis): one pass over V[0..m] gives c_i = V_i^* w (i < m)
// and ||w||^2 together; ||w - V c||^2 = ||w||^2 - sum |c_i|^2 (V orthonormal)
// is known on the host before the update, so w -= V c is launched with the
// normalisation folded in (w becomes the next unit basis vector).  A second
// pass when the first leaves no more than reorth of ||w||^2.  cf (host)
// receives c summed over the passes, nrm2 ||w||^2 before the normalisation.
// One host synchronisation per pass.
int gram_schmidt(nsf_plan p, const double2* V, long long len, int m, double2* w, cd* cf, double* nrm2,
                 int* passes, double reorth = kReorthArnoldi) {
  hipStream_t s = p->stream;
  if (w != V + (size_t)m * len) return set_error(p, NSF_E_ARG, "Gram-Schmidt: w must follow the basis");
  for (int i = 0; i < m; ++i) cf[i] = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    NSF_HIP(p, launch_multi_dot(V, len, m + 1, w, len, p->d_partial, p->d_coef, s));
    NSF_HIP(p, hipMemcpyAsync(p->h_res + 64, p->d_coef, sizeof(double2) * (m + 1), hipMemcpyDeviceToHost, s));
    int rc = sync(p);
    if (rc) return rc;
    const double before = p->h_res[64 + m].x;
    double removed = 0;
    for (int i = 0; i < m; ++i) {
      const cd c = C(p->h_res[64 + i]);
      cf[i] += c;
      removed += std::norm(c);
    }
    if (passes) *passes += 1;
    const double after = before - removed;
    const bool done = after > reorth * before || pass == 1;
    const double sc = (done && after > 0.0 && std::isfinite(after)) ? 1.0 / std::sqrt(after) : 1.0;
    NSF_HIP(p, launch_multi_axpy(V, len, m, p->d_coef, w, len, s, nullptr, nullptr, sc));
    *nrm2 = after;
    if (done) break;
  }
  return NSF_OK;
}

// Givens rotation G = [[c, s], [-conj(s), c]] with G [x; y] = [r; 0].
void givens(cd x, cd y, double* c, cd* s, cd* r) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    *c = 1.0;
    *s = 0.0;
    *r = x;
    return;
  }
  if (ax == 0.0) {
    *c = 0.0;
    *s = 1.0;
    *r = y;
    return;
  }
  const double rho = std::hypot(ax, ay);
  const cd ph = x / ax;
  *c = ax / rho;
  *s = ph * std::conj(y) / rho;
  *r = ph * rho;
}

struct Counters {
  long long matvecs = 0, iters = 0;
  int solves = 0, passes = 0;
};

// Solve Kern x = b by GMRES(R) from x = 0 (b and x device, distinct; Vg holds
// R + 1 vectors).  Stops when the explicitly recomputed residual is below
// rtol ||b|| or after maxit iterations.  Returns NSF_OK or NSF_NOT_CONVERGED.
int gmres(nsf_plan p, const double2* b, double2* x, double rtol, int maxit, int R, double2* Vg,
          Counters* cnt, double* relres_out) {
  const long long len = 4 * p->geom.n;
  hipStream_t s = p->stream;
  int rc = dot_async(p, b, b, len, 2);
  if (rc) return rc;
  if ((rc = sync(p))) return rc;
  const double bnorm = std::sqrt(p->h_res[2].x);
  NSF_HIP(p, hipMemsetAsync(x, 0, sizeof(double2) * len, s));
  cnt->solves += 1;
  if (!(bnorm > 0.0)) {
    if (relres_out) *relres_out = 0.0;
    return bnorm == 0.0 ? NSF_OK : set_error(p, NSF_E_ARG, "right-hand side is not finite");
  }
  std::vector<cd> H((size_t)(R + 1) * R), g(R + 1), y(R), h(R + 1), sn(R);
  std::vector<double> cs(R);
  NSF_HIP(p, hipMemcpyAsync(Vg, b, sizeof(double2) * len, hipMemcpyDeviceToDevice, s));
  double beta = bnorm, rel = 1.0;
  int total = 0;
  for (;;) {
    NSF_HIP(p, launch_scale_copy(Vg, Vg, 1.0 / beta, 0.0, len, s));
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    int j = 0;
    for (; j < R && total < maxit;) {
      double2* w = Vg + (size_t)(j + 1) * len;
      if ((rc = apply_Ar_dev(p, Vg + (size_t)j * len, w, nullptr))) return rc;
      cnt->matvecs += 1;
      total += 1;
      double hn2 = 0;
      if ((rc = gram_schmidt(p, Vg, len, j + 1, w, h.data(), &hn2, &cnt->passes, kReorthGmres))) return rc;
      const double hn = std::sqrt(std::max(hn2, 0.0));
      for (int i = 0; i < j; ++i) {  // earlier rotations
        const cd a = h[i], bb = h[i + 1];
        h[i] = cs[i] * a + sn[i] * bb;
        h[i + 1] = -std::conj(sn[i]) * a + cs[i] * bb;
      }
      cd r;
      givens(h[j], cd(hn), &cs[j], &sn[j], &r);
      h[j] = r;
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[(size_t)j * (R + 1) + i] = h[i];
      ++j;
      const bool small = std::abs(g[j]) <= rtol * bnorm;  // (w is already normalised)
      if (small || !(hn > 0.0)) break;
    }
    // x += V_j y with R y = g (upper triangular)
    for (int i = j - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int l = i + 1; l < j; ++l) acc -= H[(size_t)l * (R + 1) + i] * y[l];
      const cd d = H[(size_t)i * (R + 1) + i];
      y[i] = std::abs(d) > 0.0 ? acc / d : cd(0.0);
    }
    for (int i = 0; i < j; ++i) y[i] = -y[i];  // multi_axpy subtracts
    if ((rc = upload_coef(p, y.data(), j))) return rc;
    NSF_HIP(p, launch_multi_axpy(Vg, len, j, p->d_coef, x, len, s));
    // explicit residual r = b - Kern x into Vg[0]
    if ((rc = apply_Ar_dev(p, x, Vg, nullptr))) return rc;
    cnt->matvecs += 1;
    NSF_HIP(p, axpby(p, b, Vg, cd(1.0), cd(-1.0), len));
    if ((rc = dot_async(p, Vg, Vg, len, 3))) return rc;
    if ((rc = sync(p))) return rc;
    beta = std::sqrt(p->h_res[3].x);
    rel = beta / bnorm;
    if (!std::isfinite(rel)) return set_error(p, NSF_E_BREAKDOWN, "GMRES residual is not finite");
    if (rel <= rtol || total >= maxit || !(beta > 0.0)) break;
  }
  cnt->iters += total;
  if (relres_out) *relres_out = rel;
  return rel <= rtol ? NSF_OK : NSF_NOT_CONVERGED;
}

// ---------------------------------------------------------- small dense part
// Column-major m x m complex matrices with leading dimension ld.

// Reduce A to upper Hessenberg form by Householder reflections, A = Z H Z^*.
void hessenberg(int m, cd* A, int ld, cd* Z) {
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Z[(size_t)j * m + i] = i == j ? 1.0 : 0.0;
  std::vector<cd> v(m);
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0;
    for (int i = k + 1; i < m; ++i) xn += std::norm(A[(size_t)k * ld + i]);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cd x0 = A[(size_t)k * ld + k + 1];
    const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
    const cd alpha = -ph * xn;
    double vn = 0;
    for (int i = k + 1; i < m; ++i) {
      v[i] = A[(size_t)k * ld + i];
      if (i == k + 1) v[i] -= alpha;
      vn += std::norm(v[i]);
    }
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < m; ++i) v[i] /= vn;
    // A <- (I - 2 v v^*) A
    for (int j = 0; j < m; ++j) {
      cd d = 0;
      for (int i = k + 1; i < m; ++i) d += std::conj(v[i]) * A[(size_t)j * ld + i];
      for (int i = k + 1; i < m; ++i) A[(size_t)j * ld + i] -= 2.0 * v[i] * d;
    }
    // A <- A (I - 2 v v^*), Z <- Z (I - 2 v v^*)
    for (int i = 0; i < m; ++i) {
      cd d = 0, e = 0;
      for (int j = k + 1; j < m; ++j) {
        d += A[(size_t)j * ld + i] * v[j];
        e += Z[(size_t)j * m + i] * v[j];
      }
      for (int j = k + 1; j < m; ++j) {
        A[(size_t)j * ld + i] -= 2.0 * d * std::conj(v[j]);
        Z[(size_t)j * m + i] -= 2.0 * e * std::conj(v[j]);
      }
    }
    for (int i = k + 2; i < m; ++i) A[(size_t)k * ld + i] = 0.0;
  }
}

// T <- G T on rows (k, k+1), columns j0..m-1; T <- T G^* and Z <- Z G^* on
// columns (k, k+1), rows 0..i1-1 (resp. all of Z).
void rot_rows(int m, cd* T, int ld, int k, int j0, double c, cd s) {
  for (int j = j0; j < m; ++j) {
    const cd a = T[(size_t)j * ld + k], b = T[(size_t)j * ld + k + 1];
    T[(size_t)j * ld + k] = c * a + s * b;
    T[(size_t)j * ld + k + 1] = -std::conj(s) * a + c * b;
  }
}
void rot_cols(cd* A, int ld, int rows, int k, double c, cd s) {
  for (int i = 0; i < rows; ++i) {
    const cd a = A[(size_t)k * ld + i], b = A[(size_t)(k + 1) * ld + i];
    A[(size_t)k * ld + i] = c * a + std::conj(s) * b;
    A[(size_t)(k + 1) * ld + i] = -s * a + c * b;
  }
}

// Complex Schur form A = Z T Z^* (T upper triangular, written over A; Z
// unitary, m x m) by the shifted QR algorithm on the Hessenberg form with
// Wilkinson shifts.  False if it fails to converge.
bool schur(int m, cd* A, int ld, cd* Z) {
  hessenberg(m, A, ld, Z);
  const double eps = 2.220446049250313e-16;
  int hi = m - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double sub = std::abs(A[(size_t)(l - 1) * ld + l]);
      const double dia = std::abs(A[(size_t)(l - 1) * ld + l - 1]) + std::abs(A[(size_t)l * ld + l]);
      if (sub <= eps * (dia > 0 ? dia : 1.0)) {
        A[(size_t)(l - 1) * ld + l] = 0.0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 60 * m) return false;
    ++iter;
    const cd a = A[(size_t)(hi - 1) * ld + hi - 1], b = A[(size_t)hi * ld + hi - 1];
    const cd c = A[(size_t)(hi - 1) * ld + hi], d = A[(size_t)hi * ld + hi];
    cd mu;
    if (iter % 10 == 0) {
      mu = d + 0.75 * std::abs(c);  // exceptional shift
    } else {
      const cd half = 0.5 * (a - d);
      const cd disc = std::sqrt(half * half + b * c);
      const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    cd x = A[(size_t)l * ld + l] - mu, y = A[(size_t)l * ld + l + 1];
    for (int k = l; k < hi; ++k) {
      double cc;
      cd ss, r;
      givens(x, y, &cc, &ss, &r);
      rot_rows(m, A, ld, k, k > l ? k - 1 : l, cc, ss);
      rot_cols(A, ld, std::min(k + 3, hi + 1), k, cc, ss);
      rot_cols(Z, m, m, k, cc, ss);
      if (k > l) A[(size_t)(k - 1) * ld + k + 1] = 0.0;
      if (k + 1 < hi) {
        x = A[(size_t)k * ld + k + 1];
        y = A[(size_t)k * ld + k + 2];
      }
    }
  }
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) A[(size_t)j * ld + i] = 0.0;
  return true;
}

// Swap the diagonal entries k and k+1 of the upper triangular T by one unitary
// rotation, updating Z (T <- G T G^*, Z <- Z G^*).
void swap_diag(int m, cd* T, int ld, cd* Z, int k) {
  const cd t11 = T[(size_t)k * ld + k], t22 = T[(size_t)(k + 1) * ld + k + 1];
  const cd t12 = T[(size_t)(k + 1) * ld + k];
  double c;
  cd s, r;
  givens(t12, t22 - t11, &c, &s, &r);
  rot_rows(m, T, ld, k, k + 2, c, s);
  rot_cols(T, ld, k, k, c, s);
  rot_cols(Z, m, m, k, c, s);
  T[(size_t)k * ld + k] = t22;
  T[(size_t)(k + 1) * ld + k + 1] = t11;
  T[(size_t)k * ld + k + 1] = 0.0;
}

// Eigenvector of the upper triangular T for its diagonal entry i (support 0..i).
void tri_eigvec(const cd* T, int ld, int i, cd* y) {
  const cd lam = T[(size_t)i * ld + i];
  const double tiny = 1e-300 + 2.2e-16 * std::abs(lam);
  y[i] = 1.0;
  for (int j = i - 1; j >= 0; --j) {
    cd acc = 0;
    for (int l = j + 1; l <= i; ++l) acc += T[(size_t)l * ld + j] * y[l];
    cd d = T[(size_t)j * ld + j] - lam;
    if (std::abs(d) < tiny) d = tiny;
    y[j] = -acc / d;
  }
}

// Ritz value order: positive real part first, then descending modulus.
bool before(cd a, cd b) {
  const bool pa = a.real() > 0, pb = b.real() > 0;
  if (pa != pb) return pa;
  return std::abs(a) > std::abs(b);
}

// Schur form (ld = m) with the diagonal in the wanted order (selection by
// adjacent swaps).
bool schur_sorted(int m, cd* T, cd* Z) {
  if (!schur(m, T, m, Z)) return false;
  for (int i = 0; i < m; ++i) {
    int bi = i;
    for (int j = i + 1; j < m; ++j)
      if (before(T[(size_t)j * m + j], T[(size_t)bi * m + bi])) bi = j;
    for (int j = bi; j > i; --j) swap_diag(m, T, m, Z, j - 1);
  }
  return true;
}

struct Out {
  std::vector<cd> omega;
  std::vector<double> eta;
};

}  // namespace
}  // namespace nsf

using namespace nsf;

extern "C" {

int nsf_schur_sorted(int m, const nsf_c128* A, nsf_c128* T, nsf_c128* Z) {
  if (m < 1 || m > 512 || !A || !T || !Z) return set_error(nullptr, NSF_E_ARG, "bad argument");
  std::vector<cd> a((size_t)m * m), z((size_t)m * m);
  for (size_t e = 0; e < a.size(); ++e) a[e] = cd(A[e].re, A[e].im);
  if (!schur_sorted(m, a.data(), z.data())) return set_error(nullptr, NSF_E_BREAKDOWN, "QR iteration failed");
  for (size_t e = 0; e < a.size(); ++e) {
    T[e].re = a[e].real();
    T[e].im = a[e].imag();
    Z[e].re = z[e].real();
    Z[e].im = z[e].imag();
  }
  return NSF_OK;
}

int nsf_apply_nfsep(nsf_plan p, const nsf_c128* y4n, nsf_c128* out4n) {
  if (!p || !y4n || !out4n) return set_error(p, NSF_E_ARG, "NULL argument");
  if (p->medium_kind != kMedNfsep) return set_error(p, NSF_E_STATE, "no NFSEP medium set");
  int rc = ensure_device(p);
  if (rc) return rc;
  if ((rc = ensure_cg(p))) return rc;
  const long long len = 4 * p->geom.n;
  double2* t = p->d_cg;  // scratch: S' y
  double2* out = reinterpret_cast<double2*>(out4n);
  NSF_HIP(p, sigma_pow(p, reinterpret_cast<const double2*>(y4n), t, true, false));
  if ((rc = apply_Ar_dev(p, t, t + len, nullptr))) return rc;
  NSF_HIP(p, sigma_pow(p, t + len, out, true, true));  // S' (i J4) Kern S' y
  return NSF_OK;
}

int nsf_nfsep_solve(nsf_plan p, const nsf_c128* b, nsf_c128* x, double rtol, int maxit, int restart,
                    int* iters, double* relres) {
  if (!p || !b || !x) return set_error(p, NSF_E_ARG, "NULL argument");
  if ((const void*)b == (const void*)x) return set_error(p, NSF_E_ARG, "b and x must be distinct");
  if (!(rtol > 0.0)) return set_error(p, NSF_E_ARG, "rtol must be > 0");
  if (p->medium_kind != kMedNfsep) return set_error(p, NSF_E_STATE, "no NFSEP medium set");
  const int R = restart > 0 ? std::min(restart, 500) : 12;
  if (maxit <= 0) maxit = 2000;
  int rc = ensure_device(p);
  if (rc) return rc;
  if ((rc = ensure_cg(p))) return rc;
  const long long len = 4 * p->geom.n;
  double2* Vg = nullptr;
  if (hipMalloc(&Vg, sizeof(double2) * (size_t)(R + 1) * len) != hipSuccess)
    return set_error(p, NSF_E_NOMEM, "GMRES basis allocation failed");
  double2* t = p->d_cg;
  double2* xx = reinterpret_cast<double2*>(x);
  // K x = b  <=>  Kern (S' x) = (i J4) S'^{-1} b
  rc = hip_check(p, sigma_pow(p, reinterpret_cast<const double2*>(b), t, false, true), "nfsep rhs");
  Counters cnt;
  double rel = 0;
  if (!rc) rc = gmres(p, t, xx, rtol, maxit, R, Vg, &cnt, &rel);
  if (rc >= 0) {
    const int r2 = hip_check(p, sigma_pow(p, xx, xx, false, false), "nfsep scale");
    if (r2) rc = r2;
  }
  hipStreamSynchronize(p->stream);
  hipFree(Vg);
  if (iters) *iters = (int)cnt.iters;
  if (relres) *relres = rel;
  return rc;
}

int nsf_eigs_nfsep(nsf_plan p, int nev, double res_tol, double inner_rtol, int max_basis, int max_restarts,
                   unsigned long long seed, nsf_c128* omega_host, nsf_c128* Y_dev, double* resid_host,
                   nsf_stats* stats) {
  const auto t_start = clk::now();
  if (!p) return set_error(nullptr, NSF_E_ARG, "plan is NULL");
  if (p->medium_kind != kMedNfsep) return set_error(p, NSF_E_STATE, "no NFSEP medium set");
  const long long n = p->geom.n, len = 4 * n;
  if (nev < 1 || nev > 256 || 2LL * nev >= len) return set_error(p, NSF_E_ARG, "nev out of range");
  if (!(res_tol > 0.0) || !(inner_rtol > 0.0)) return set_error(p, NSF_E_ARG, "tolerances must be > 0");
  if (!omega_host) return set_error(p, NSF_E_ARG, "omega_host is NULL");
  int m = max_basis > 0 ? max_basis : std::max(3 * nev, nev + 8);
  if (m < nev + 2) m = nev + 2;
  if (m > 510) m = 510;
  if (m >= len) m = (int)len - 1;
  const int kkeep = std::min(m - 1, nev + (m - nev) / 2);
  const int maxr = max_restarts > 0 ? max_restarts : 1000;
  const int R = p->opt_gmres_restart;
  int rc = ensure_device(p);
  if (rc) return rc;
  if ((rc = ensure_cg(p))) return rc;
  hipStream_t s = p->stream;

  // device buffers: V (m+1), GMRES basis (R+1), rhs, two checks, Ritz vectors
  const size_t nvec = (size_t)(m + 1) + (R + 1) + 3 + (Y_dev ? 0 : nev);
  double2* big = nullptr;
  double2* dS = nullptr;
  if (hipMalloc(&big, sizeof(double2) * nvec * len) != hipSuccess)
    return set_error(p, NSF_E_NOMEM, "NFSEP basis allocation failed");
  if (hipMalloc(&dS, sizeof(double2) * (size_t)m * m) != hipSuccess) {
    hipFree(big);
    return set_error(p, NSF_E_NOMEM, "NFSEP small-matrix allocation failed");
  }
  double2* hS = nullptr;
  if (hipHostMalloc((void**)&hS, sizeof(double2) * (size_t)m * m) != hipSuccess) {
    hipFree(big);
    hipFree(dS);
    return set_error(p, NSF_E_NOMEM, "NFSEP pinned allocation failed");
  }
  double2* V = big;
  double2* Vg = V + (size_t)(m + 1) * len;
  double2* rhs = Vg + (size_t)(R + 1) * len;
  double2* c1 = rhs + len;
  double2* c2 = c1 + len;
  double2* Y = Y_dev ? reinterpret_cast<double2*>(Y_dev) : c2 + len;

  Counters cnt;
  int steps = 0, restarts = 0, status = NSF_NOT_CONVERGED;
  double t_gmres = 0, t_orth = 0, t_rest = 0;
  std::vector<cd> Hm((size_t)(m + 1) * m, cd(0.0));  // Op V_m = V_{m+1} Hm, ld = m + 1
  std::vector<cd> T((size_t)m * m), Z((size_t)m * m), bvec(m), yv(m), hcol(m + 1), S((size_t)m * m);
  Out best;
  double tol_ks = res_tol;

  auto body = [&]() -> int {
    int k = 0;  // columns of the current Krylov-Schur decomposition
    // V_0: seeded complex normal vector, normalised
    NSF_HIP(p, launch_randn(V, len, seed, s));
    int rc2 = dot_async(p, V, V, len, 4);
    if (rc2) return rc2;
    if ((rc2 = sync(p))) return rc2;
    NSF_HIP(p, launch_scale_copy(V, V, 1.0 / std::sqrt(p->h_res[4].x), 0.0, len, s));
    for (;;) {
      for (int j = k; j < m; ++j) {
        auto t0 = clk::now();
        NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, V + (size_t)j * len, rhs, nullptr, s));
        double2* w = V + (size_t)(j + 1) * len;
        double rel = 0;
        rc2 = gmres(p, rhs, w, inner_rtol, 4000, R, Vg, &cnt, &rel);
        if (rc2 < 0) return rc2;
        t_gmres += ms_since(t0);
        t0 = clk::now();
        double nrm2 = 0;
        if ((rc2 = gram_schmidt(p, V, len, j + 1, w, hcol.data(), &nrm2, &cnt.passes))) return rc2;
        double hn = std::sqrt(std::max(nrm2, 0.0));
        double hsz = 0;
        for (int i = 0; i <= j; ++i) hsz += std::norm(hcol[i]);
        if (!(hn > 1e-13 * std::sqrt(hsz))) {
          // invariant subspace: continue from a fresh direction orthogonal to V
          // (two passes, each leaving a unit vector)
          NSF_HIP(p, launch_randn(w, len, seed + 7919ULL * (steps + 1), s));
          std::vector<cd> tmp(j + 1);
          if ((rc2 = gram_schmidt(p, V, len, j + 1, w, tmp.data(), &nrm2, &cnt.passes))) return rc2;
          if ((rc2 = gram_schmidt(p, V, len, j + 1, w, tmp.data(), &nrm2, &cnt.passes))) return rc2;
          hn = 0.0;
        }
        for (int i = 0; i <= j; ++i) Hm[(size_t)j * (m + 1) + i] = hcol[i];
        Hm[(size_t)j * (m + 1) + j + 1] = hn;
        steps += 1;
        t_orth += ms_since(t0);
      }
      auto t0 = clk::now();
      // Schur form of the m x m block, wanted Ritz values first
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) T[(size_t)j * m + i] = Hm[(size_t)j * (m + 1) + i];
      if (!schur_sorted(m, T.data(), Z.data()))
        return set_error(p, NSF_E_BREAKDOWN, "Schur decomposition of the projected matrix failed");
      for (int j = 0; j < m; ++j) {  // b = (last row of Hm) Z
        cd acc = 0;
        for (int i = 0; i < m; ++i) acc += Hm[(size_t)i * (m + 1) + m] * Z[(size_t)j * m + i];
        bvec[j] = acc;
      }
      bool conv = true;
      for (int i = 0; i < nev; ++i) {
        const cd th = T[(size_t)i * m + i];
        std::fill(yv.begin(), yv.end(), cd(0.0));
        tri_eigvec(T.data(), m, i, yv.data());
        double yn = 0;
        cd by = 0;
        for (int l = 0; l <= i; ++l) {
          yn += std::norm(yv[l]);
          by += bvec[l] * yv[l];
        }
        if (!(th.real() > 0) || !(std::abs(by) <= tol_ks * std::abs(th) * std::sqrt(yn))) conv = false;
      }
      const bool last = restarts >= maxr;
      if (conv || last) {
        // Ritz vectors x_i = V_m Z y_i / ||y_i||, then exact residuals
        for (int i = 0; i < nev; ++i) {
          std::fill(yv.begin(), yv.end(), cd(0.0));
          tri_eigvec(T.data(), m, i, yv.data());
          double yn = 0;
          for (int l = 0; l <= i; ++l) yn += std::norm(yv[l]);
          yn = std::sqrt(yn);
          for (int r = 0; r < m; ++r) {
            cd acc = 0;
            for (int l = 0; l <= i; ++l) acc += Z[(size_t)l * m + r] * yv[l];
            S[(size_t)i * m + r] = -acc / yn;  // multi_axpy subtracts
          }
        }
        for (size_t e = 0; e < (size_t)m * nev; ++e) hS[e] = D2(S[e]);
        NSF_HIP(p, hipMemcpyAsync(dS, hS, sizeof(double2) * (size_t)m * nev, hipMemcpyHostToDevice, s));
        Out cur;
        bool all = true;
        for (int i = 0; i < nev; ++i) {
          double2* x = Y + (size_t)i * len;
          NSF_HIP(p, hipMemsetAsync(x, 0, sizeof(double2) * len, s));
          NSF_HIP(p, launch_multi_axpy(V, len, m, dS + (size_t)i * m, x, len, s));
          // q = Kern x, bq = B_r x; y = S' i J4 bq and K y = S' i J4 q
          if ((rc2 = apply_Ar_dev(p, x, c2, nullptr))) return rc2;
          cnt.matvecs += 1;
          NSF_HIP(p, launch_apply_Br(p->geom, p->tabs, x, c1, nullptr, s));
          NSF_HIP(p, sigma_pow(p, c1, c1, true, false));
          NSF_HIP(p, sigma_pow(p, c2, c2, true, false));
          if ((rc2 = dot_async(p, c1, c2, len, 5))) return rc2;
          if ((rc2 = dot_async(p, c1, c1, len, 6))) return rc2;
          if ((rc2 = sync(p))) return rc2;
          const double yy = p->h_res[6].x;
          const cd om = C(p->h_res[5]) / yy;
          NSF_HIP(p, axpby(p, c1, c2, -om, cd(1.0), len));
          if ((rc2 = dot_async(p, c2, c2, len, 7))) return rc2;
          if ((rc2 = sync(p))) return rc2;
          const double eta = std::sqrt(p->h_res[7].x) / (std::abs(om) * std::sqrt(yy));
          cur.omega.push_back(om);
          cur.eta.push_back(eta);
          if (!(eta <= res_tol) || !(om.real() > 0)) all = false;
        }
        // ascending modulus of omega (the wanted order up to the refinement),
        // permuting the Ritz vectors alike through c1
        std::vector<int> ord(nev), at(nev);
        for (int i = 0; i < nev; ++i) ord[i] = at[i] = i;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return std::abs(cur.omega[a]) < std::abs(cur.omega[b]); });
        for (int i = 0; i < nev; ++i) {
          int where = i;
          while (at[where] != ord[i]) ++where;
          if (where == i) continue;
          double2* A = Y + (size_t)i * len;
          double2* B = Y + (size_t)where * len;
          NSF_HIP(p, hipMemcpyAsync(c1, A, sizeof(double2) * len, hipMemcpyDeviceToDevice, s));
          NSF_HIP(p, hipMemcpyAsync(A, B, sizeof(double2) * len, hipMemcpyDeviceToDevice, s));
          NSF_HIP(p, hipMemcpyAsync(B, c1, sizeof(double2) * len, hipMemcpyDeviceToDevice, s));
          std::swap(at[i], at[where]);
        }
        best.omega.clear();
        best.eta.clear();
        for (int i = 0; i < nev; ++i) {
          best.omega.push_back(cur.omega[ord[i]]);
          best.eta.push_back(cur.eta[ord[i]]);
        }
        if (all) {
          status = NSF_OK;
          t_rest += ms_since(t0);
          return NSF_OK;
        }
        if (last) {
          t_rest += ms_since(t0);
          return NSF_OK;
        }
        tol_ks *= 0.1;  // the operator residual was not tight enough
      }
      // restart: keep the leading kkeep Schur vectors and the residual vector
      for (int j = 0; j < kkeep; ++j)
        for (int i = 0; i < m; ++i) hS[(size_t)j * m + i] = D2(Z[(size_t)j * m + i]);
      NSF_HIP(p, hipMemcpyAsync(dS, hS, sizeof(double2) * (size_t)m * kkeep, hipMemcpyHostToDevice, s));
      NSF_HIP(p, launch_rotate(V, len, m, kkeep, dS, len, s));
      NSF_HIP(p, hipMemcpyAsync(V + (size_t)kkeep * len, V + (size_t)m * len, sizeof(double2) * len,
                                hipMemcpyDeviceToDevice, s));
      if ((rc2 = sync(p))) return rc2;  // hS is reused
      std::fill(Hm.begin(), Hm.end(), cd(0.0));
      for (int j = 0; j < kkeep; ++j) {
        for (int i = 0; i <= j; ++i) Hm[(size_t)j * (m + 1) + i] = T[(size_t)j * m + i];
        Hm[(size_t)j * (m + 1) + kkeep] = bvec[j];
      }
      k = kkeep;
      restarts += 1;
      t_rest += ms_since(t0);
    }
  };
  rc = body();
  hipStreamSynchronize(s);
  hipFree(big);
  hipFree(dS);
  hipHostFree(hS);
  if (rc < 0) return rc;
  int nconv = 0;
  for (size_t i = 0; i < best.omega.size(); ++i) {
    omega_host[i].re = best.omega[i].real();
    omega_host[i].im = best.omega[i].imag();
    if (resid_host) resid_host[i] = best.eta[i];
    if (best.eta[i] <= res_tol) ++nconv;
  }
  nsf_stats st{};
  st.matvecs = cnt.matvecs;
  st.cg_iters_total = cnt.iters;
  st.cg_solves = cnt.solves;
  st.lanczos_steps = steps;
  st.restarts = restarts;
  st.converged = nconv;
  st.ortho_passes = cnt.passes;
  st.cg_iters_avg = cnt.solves ? (double)cnt.iters / cnt.solves : 0.0;
  st.bytes_alg = (double)(kNfsepFieldBytesPerVoxel + medium_voxel_bytes(p)) * (double)n * (double)cnt.matvecs;
  st.ms_cg = t_gmres;
  st.ms_orth = t_orth;
  st.ms_restart = t_rest;
  st.ms_total = ms_since(t_start);
  if (stats) *stats = st;
  trace_solve("nsf_eigs_nfsep", p, 0, nev, status, st, best.eta.data());
  return status;
}

}  // extern "C"
