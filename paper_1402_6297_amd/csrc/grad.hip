// Eigenvalue gradients w.r.t. per-voxel eps and gamma of a chiral medium.
//
// For the HHPD pencil B_r y = theta A_r y (Thm 4.2) with B_r independent of
// the medium and y^* A_r y = 1, first-order perturbation gives
// d theta = -theta y^* dA_r y, i.e. d omega = omega y^* dA_r y.  Writing the
// factors of A_r out for mu = 1, xi = i gamma, zeta = -i gamma,
//   y^* A_r y = sum_g sum_c [ |i gamma_g E'_gc + H'_gc|^2 / Phi_g + |E'_gc|^2 ],
// with E' = P_r y_P, H' = Q_r y_Q and Phi = eps - gamma^2.  Differentiating:
//   d omega/d eps_g   = -omega sum_c |s_c|^2 / Phi^2,          s = i gamma E' + H'
//   d omega/d gamma_g =  omega sum_c [ 2 Re(conj(s_c) i E'_c) / Phi + 2 gamma |s_c|^2 / Phi^2 ].
// Each eigenvector costs the three inverse passes of P_r, Q_r plus one
// pointwise accumulation.
#include "nsf_internal.h"

namespace nsf {
namespace {

__global__ void k_grad_accum(long long n, const double2* __restrict__ eg,
                             const double2* __restrict__ fld, double wo, double* __restrict__ d_eps,
                             double* __restrict__ d_gam, int first) {
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x) {
    const double eps = eg[g].x, gam = eg[g].y;
    const double phi = eps - gam * gam;
    double A = 0, Bv = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 e = fld[c * n + g], h = fld[(3 + c) * n + g];
      const double2 sc = cadd(cmuli(cscale(e, gam)), h);
      A += cabs2(sc);
      const double2 ie = cmuli(e);
      Bv += sc.x * ie.x + sc.y * ie.y;  // Re(conj(s) i E')
    }
    const double de = -wo * A / (phi * phi);
    const double dg = wo * (2.0 * Bv / phi + 2.0 * gam * A / (phi * phi));
    if (first) {
      d_eps[g] = de;
      d_gam[g] = dg;
    } else {
      d_eps[g] += de;
      d_gam[g] += dg;
    }
  }
}

}  // namespace

hipError_t launch_grad_accum(const Geom& g, const double2* eg, const double2* fld, double wo,
                             double* d_eps, double* d_gamma, int first, hipStream_t s) {
  long long blocks = (g.n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_grad_accum, dim3((unsigned)blocks), dim3(256), 0, s, g.n, eg, fld, wo, d_eps,
                     d_gamma, first);
  return hipGetLastError();
}

}  // namespace nsf

using namespace nsf;

extern "C" int nsf_eig_grad(nsf_plan p, int nev, const double* omega_host, const nsf_c128* Y_dev,
                            const double* weights_host, double* d_eps_dev, double* d_gamma_dev) {
  if (!p || !omega_host || !Y_dev || !weights_host || !d_eps_dev || !d_gamma_dev)
    return set_error(p, NSF_E_ARG, "NULL argument");
  if (nev < 1) return set_error(p, NSF_E_ARG, "nev must be >= 1");
  if (p->medium_kind != kMedChiral) return set_error(p, NSF_E_STATE, "gradient needs a chiral medium");
  int rc = ensure_device(p);
  if (rc) return rc;
  const Geom& g = p->geom;
  const long long len = 4 * g.n;
  hipStream_t s = p->stream;
  double2* F = p->d_fields;
  for (int j = 0; j < nev; ++j) {
    const double2* y = reinterpret_cast<const double2*>(Y_dev) + (size_t)j * len;
    NSF_HIP(p, pass_x_inv(p, kPartBoth, y, F, nullptr));
    NSF_HIP(p, pass_yz(p, 1, +1, 6, F, 0, 0, nullptr));
    NSF_HIP(p, pass_yz(p, 2, +1, 6, F, 1, 0, nullptr));
    NSF_HIP(p, launch_grad_accum(g, p->d_medium, F, weights_host[j] * omega_host[j], d_eps_dev,
                                 d_gamma_dev, j == 0, s));
  }
  return NSF_OK;
}
