// Electric and magnetic fields of an eigenvector (Algorithm 1, last step):
// x = [E; H] = B^{-1} diag(P_r, Q_r) y.
//
// With J = [[0, I], [-I, 0]], the factorisation in the proof of Thm 4.2 reads
// i J B^{-1} = M, the Hermitian per-voxel middle factor of A_r, so
// B^{-1} = (i J)^{-1} M = i J M.  Hence, with [E'; H'] = [P_r y_P; Q_r y_Q] the
// twisted spatial fields and [o1; o2] = M [E'; H'] voxel by voxel,
//   E = i o2,  H = -i o1.
// The twist D is a per-voxel phase and commutes with M, so the fields carry the
// Bloch phase of k exactly as P_r and Q_r produce it.
#include "nsf_internal.h"
#include "fft_common.h"

namespace nsf {
namespace {

__global__ void k_fields(MediumView med, double2* __restrict__ EH, long long n) {
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < n;
       g += (long long)gridDim.x * blockDim.x) {
    double2 E[3], H[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[c] = EH[c * n + g];
      H[c] = EH[(3 + c) * n + g];
    }
    medium_apply_at(med, g, 1.0, E, H);  // E <- o1, H <- o2
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      EH[c * n + g] = cmuli(H[c]);                           // i o2
      EH[(3 + c) * n + g] = cscale(cmuli(E[c]), -1.0);       // -i o1
    }
  }
}

}  // namespace
}  // namespace nsf

using namespace nsf;

extern "C" {

int nsf_fields(nsf_plan p, const nsf_c128* y4n, nsf_c128* eh6n) {
  if (!p || !y4n || !eh6n) return set_error(p, NSF_E_ARG, "NULL argument");
  if (p->medium_kind == kMedNone) return set_error(p, NSF_E_STATE, "no medium set");
  int rc = ensure_device(p);
  if (rc) return rc;
  const Geom& g = p->geom;
  const long long n = g.n;
  const double2* y = reinterpret_cast<const double2*>(y4n);
  double2* EH = reinterpret_cast<double2*>(eh6n);
  // E' = P_r y_P into the first 3n, H' = Q_r y_Q into the second 3n
  NSF_HIP(p, pass_x_inv(p, kPartP, y, EH, nullptr));
  NSF_HIP(p, pass_x_inv(p, kPartQ, y + 2 * n, EH + 3 * n, nullptr));
  NSF_HIP(p, pass_yz(p, 1, +1, 6, EH, 0, 0, nullptr));
  NSF_HIP(p, pass_yz(p, 2, +1, 6, EH, 1, 0, nullptr));
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fields, dim3((unsigned)blocks), dim3(256), 0, p->stream, medium_view(p), EH, n);
  NSF_HIP(p, hipGetLastError());
  return NSF_OK;
}

}  // extern "C"
