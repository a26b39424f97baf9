// Pencil passes of the twisted 3-D FFTs that apply P_r, Q_r and A_r.
//
// T = n^{-1/2} (D3 (x) D2 (x) D1)(U3 (x) U2 (x) U1) (Sec. 2); U_m is the
// unnormalised DFT with kernel e^{+2 pi i j k / m}.  A_r applies T, a
// per-voxel 6x6 step and T^* (Thm 4.2); the twist D is a per-voxel phase and
// cancels around that step, so the A_r passes run untwisted transforms and
// scale by 1/n once.  P_r and Q_r alone apply D / sqrt(n) after the last
// inverse pass, P_r^* and Q_r^* apply conj(D) / sqrt(n) before the first
// forward pass.
//
// Every pass stages a tile of P pencils x N points x F fields in LDS and runs
// mixed-radix Stockham stages (radix 8, 4, 2, 3, 5) on it: each stage reads R
// points per butterfly into registers, multiplies by the stage twiddles from
// an LDS copy of exp(+2 pi i m / N), does the radix-R DFT and writes the
// results back in autosorted order.
#include "nsf_internal.h"
#include "fft_common.h"

namespace nsf {
namespace {

// One Stockham stage over a tile laid out as tile[(f*N + j)*P + p].
// Butterfly b of a pencil reads points b + r*N/R; after the DFT its outputs
// land at (b / Ns) * Ns * R + (b mod Ns) + r * Ns.
template <int R, int S>
__device__ __forceinline__ void stage(double2* tile, const double2* tw, int F, int P, int N, int Ns) {
  constexpr int MB = (kEpt + R - 1) / R;
  const int nb = N / R;
  const int total = F * P * nb;
  const int step = N / (Ns * R);
  double2 v[MB][R];
  int jout[MB], pp[MB];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const int w = threadIdx.x + i * kThreads;
    jout[i] = -1;
    if (w < total) {
      const int p = w % P;
      const int rest = w / P;
      const int b = rest % nb;
      const int f = rest / nb;
      const int kk = b % Ns;
      const int fb = f * N;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 x = tile[(fb + b + r * nb) * P + p];
        if (r > 0 && kk > 0) {
          double2 t = tw[kk * r * step];
          if (S < 0) t = cconj(t);
          x = cmul(x, t);
        }
        v[i][r] = x;
      }
      dft<R, S>(v[i]);
      jout[i] = fb + (b / Ns) * Ns * R + kk;
      pp[i] = p;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (jout[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) tile[(jout[i] + r * Ns) * P + pp[i]] = v[i][r];
    }
  }
  __syncthreads();
}

template <int S>
__device__ void tile_fft(double2* tile, const double2* tw, int F, int P, const AxisPlan& ax) {
  int Ns = 1;
  for (int s = 0; s < ax.nst; ++s) {
    const int R = ax.radix[s];
    switch (R) {
      case 8: stage<8, S>(tile, tw, F, P, ax.N, Ns); break;
      case 4: stage<4, S>(tile, tw, F, P, ax.N, Ns); break;
      case 2: stage<2, S>(tile, tw, F, P, ax.N, Ns); break;
      case 3: stage<3, S>(tile, tw, F, P, ax.N, Ns); break;
      default: stage<5, S>(tile, tw, F, P, ax.N, Ns); break;
    }
    Ns *= R;
  }
}

// ------------------------------------------------------------- x passes
template <int PART>
__global__ __launch_bounds__(kThreads) void k_x_inv_synth(Geom g, AxisPlan ax, Tables t,
                                                          const double2* __restrict__ y,
                                                          double2* __restrict__ fld, int P,
                                                          const int* skip) {
  if (skip && *skip) return;
  extern __shared__ double2 sm[];
  const int N = g.n1;
  double2* tw = sm;
  double2* tile = sm + N;
  for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = t.tw[i];
  constexpr int F = (PART == kPartBoth) ? 6 : 3;
  const long long rows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * P;
  const long long n = g.n;
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int p = e / N;
    const int i1 = e - p * N;
    const long long row = row0 + p;
    if (row >= rows) continue;
    const int i2 = (int)(row % g.n2);
    const int i3 = (int)(row / g.n2);
    const long long f = row * N + i1;
    Basis B;
    basis_at(t.lam, g, i1, i2, i3, B);
    if (PART == kPartBoth || PART == kPartP) {
      const double2 ya = y[f], yb = y[n + f];
#pragma unroll
      for (int c = 0; c < 3; ++c)  // e = -conj(pi2) y_a + conj(pi1) y_b
        tile[(c * N + i1) * P + p] = csub(cmulc(B.pi1[c], yb), cmulc(B.pi2[c], ya));
    }
    if (PART == kPartBoth || PART == kPartQ) {
      const long long o = (PART == kPartBoth) ? 2 * n : 0;
      const int cb = (PART == kPartBoth) ? 3 : 0;
      const double2 yc = y[o + f], yd = y[o + n + f];
#pragma unroll
      for (int c = 0; c < 3; ++c)  // h = pi1 y_c + pi2 y_d
        tile[((cb + c) * N + i1) * P + p] = cadd(cmul(B.pi1[c], yc), cmul(B.pi2[c], yd));
    }
  }
  __syncthreads();
  tile_fft<+1>(tile, tw, F, P, ax);
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int p = e / N;
    const int i1 = e - p * N;
    const long long row = row0 + p;
    if (row >= rows) continue;
    const long long gi = row * N + i1;
#pragma unroll
    for (int c = 0; c < F; ++c) fld[c * n + gi] = tile[(c * N + i1) * P + p];
  }
}

template <int PART>
__global__ __launch_bounds__(kThreads) void k_x_fwd_proj(Geom g, AxisPlan ax, Tables t,
                                                         const double2* __restrict__ fld,
                                                         double2* __restrict__ out, int P,
                                                         const int* skip) {
  if (skip && *skip) return;
  extern __shared__ double2 sm[];
  const int N = g.n1;
  double2* tw = sm;
  double2* tile = sm + N;
  for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = t.tw[i];
  constexpr int F = (PART == kPartBoth) ? 6 : 3;
  const long long rows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * P;
  const long long n = g.n;
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int p = e / N;
    const int i1 = e - p * N;
    const long long row = row0 + p;
    if (row >= rows) continue;
    const long long gi = row * N + i1;
#pragma unroll
    for (int c = 0; c < F; ++c) tile[(c * N + i1) * P + p] = fld[c * n + gi];
  }
  __syncthreads();
  tile_fft<-1>(tile, tw, F, P, ax);
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int p = e / N;
    const int i1 = e - p * N;
    const long long row = row0 + p;
    if (row >= rows) continue;
    const int i2 = (int)(row % g.n2);
    const int i3 = (int)(row / g.n2);
    const long long f = row * N + i1;
    Basis B;
    basis_at(t.lam, g, i1, i2, i3, B);
    if (PART == kPartBoth || PART == kPartP) {
      double2 oa = make_double2(0, 0), ob = make_double2(0, 0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {  // a = -pi2^T o1, b = pi1^T o1
        const double2 o = tile[(c * N + i1) * P + p];
        oa = csub(oa, cmul(B.pi2[c], o));
        ob = cadd(ob, cmul(B.pi1[c], o));
      }
      out[f] = oa;
      out[n + f] = ob;
    }
    if (PART == kPartBoth || PART == kPartQ) {
      const long long o0 = (PART == kPartBoth) ? 2 * n : 0;
      const int cb = (PART == kPartBoth) ? 3 : 0;
      double2 oc = make_double2(0, 0), od = make_double2(0, 0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {  // c = pi1^* o2, d = pi2^* o2
        const double2 o = tile[((cb + c) * N + i1) * P + p];
        oc = cadd(oc, cmulc(B.pi1[c], o));
        od = cadd(od, cmulc(B.pi2[c], o));
      }
      out[o0 + f] = oc;
      out[o0 + n + f] = od;
    }
  }
}

// --------------------------------------------------------- y / z passes
// Pencil group gid covers P consecutive i1 at one (i3) for axis 1 or one (i2)
// for axis 2.  Element (j, p) of the group sits at base + j*stride + p.
__device__ inline void yz_group(const Geom& g, int axis, int P, long long gid, long long& base,
                                long long& stride, int& i1_0, int& io) {
  const int groups1 = g.n1 / P;
  i1_0 = (int)(gid % groups1) * P;
  io = (int)(gid / groups1);
  if (axis == 1) {
    base = (long long)io * g.n1 * g.n2 + i1_0;
    stride = g.n1;
  } else {
    base = (long long)io * g.n1 + i1_0;
    stride = (long long)g.n1 * g.n2;
  }
}

template <int S>
__global__ __launch_bounds__(kThreads) void k_yz_pass(Geom g, AxisPlan ax, Tables t, int axis,
                                                      double2* __restrict__ fld, int P,
                                                      int post_twist, int pre_twist,
                                                      const int* skip) {
  if (skip && *skip) return;
  extern __shared__ double2 sm[];
  const int N = ax.N;
  const int twoff = (axis == 1) ? g.n1 : g.n1 + g.n2;
  double2* tw = sm;
  double2* tile = sm + N;
  for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = t.tw[twoff + i];
  long long base, stride;
  int i1_0, io;
  yz_group(g, axis, P, blockIdx.x, base, stride, i1_0, io);
  double2* F = fld + (long long)blockIdx.y * g.n;
  const double rs = 1.0 / sqrt((double)g.n);
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int j = e / P;
    const int p = e - j * P;
    double2 v = F[base + j * stride + p];
    if (pre_twist) {  // axis 2 only: conj(D_g)/sqrt(n)
      const double2 d = twist_at(t.twist, g, i1_0 + p, io, j);
      v = cscale(cmulc(d, v), rs);
    }
    tile[j * P + p] = v;
  }
  __syncthreads();
  tile_fft<S>(tile, tw, 1, P, ax);
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int j = e / P;
    const int p = e - j * P;
    double2 v = tile[j * P + p];
    if (post_twist) {  // axis 2 only: D_g/sqrt(n)
      const double2 d = twist_at(t.twist, g, i1_0 + p, io, j);
      v = cscale(cmul(d, v), rs);
    }
    F[base + j * stride + p] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_z_mid(Geom g, AxisPlan ax, Tables t, MediumView med,
                                                    double2* __restrict__ fld, int P,
                                                    const int* skip) {
  if (skip && *skip) return;
  extern __shared__ double2 sm[];
  const int N = ax.N;
  double2* tw = sm;
  double2* tile = sm + N;
  for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = t.tw[g.n1 + g.n2 + i];
  long long base, stride;
  int i1_0, io;
  yz_group(g, 2, P, blockIdx.x, base, stride, i1_0, io);
  const long long n = g.n;
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int j = e / P;
    const int p = e - j * P;
    const long long gi = base + j * stride + p;
#pragma unroll
    for (int c = 0; c < 6; ++c) tile[(c * N + j) * P + p] = fld[c * n + gi];
  }
  __syncthreads();
  tile_fft<+1>(tile, tw, 6, P, ax);
  const double inv_n = 1.0 / (double)n;
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int j = e / P;
    const int p = e - j * P;
    const long long gi = base + j * stride + p;
    double2 E[3], H[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[c] = tile[(c * N + j) * P + p];
      H[c] = tile[((3 + c) * N + j) * P + p];
    }
    medium_apply_at(med, gi, inv_n, E, H);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tile[(c * N + j) * P + p] = E[c];
      tile[((3 + c) * N + j) * P + p] = H[c];
    }
  }
  __syncthreads();
  tile_fft<-1>(tile, tw, 6, P, ax);
  for (int e = threadIdx.x; e < P * N; e += kThreads) {
    const int j = e / P;
    const int p = e - j * P;
    const long long gi = base + j * stride + p;
#pragma unroll
    for (int c = 0; c < 6; ++c) fld[c * n + gi] = tile[(c * N + j) * P + p];
  }
}

// -------------------------------------------------------------- B_r
__global__ void k_apply_Br(Geom g, Tables t, const double2* u, double2* out, const int* skip) {
  if (skip && *skip) return;
  const long long n = g.n;
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    const int i1 = (int)(f % g.n1);
    const int i2 = (int)((f / g.n1) % g.n2);
    const int i3 = (int)(f / ((long long)g.n1 * g.n2));
    const double s2 = cabs2(t.lam[i1]) + cabs2(t.lam[g.n1 + i2]) + cabs2(t.lam[g.n1 + g.n2 + i3]);
    const double is = 1.0 / sqrt(s2);
    const double2 a = u[f], b = u[n + f], c = u[2 * n + f], d = u[3 * n + f];
    out[f] = cscale(cmuli(c), is);              // i y_c / sigma
    out[n + f] = cscale(cmuli(d), is);          // i y_d / sigma
    out[2 * n + f] = cscale(cmuli(a), -is);     // -i y_a / sigma
    out[3 * n + f] = cscale(cmuli(b), -is);     // -i y_b / sigma
  }
}

// Tile width P: pencils per workgroup.  x passes take whole rows; y/z passes
// take P consecutive x positions (P divides n1) for coalesced access.
int pick_P_rows(int N, int F, long long rows) {
  int P = 1;
  while (2 * P * F * N + N <= kEpt * kThreads && 2 * P <= rows) P *= 2;
  return P;
}

int pick_P_cols(int N, int F, int n1) {
  int P = 1;
  while (2 * P * F * N + N <= kEpt * kThreads && n1 % (2 * P) == 0 && 2 * P <= 16) P *= 2;
  return P;
}

size_t lds_bytes(int N, int F, int P) { return sizeof(double2) * (size_t)(N + F * P * N); }

}  // namespace

hipError_t launch_x_inv_synth(const Geom& g, const AxisPlan& ax, const Tables& t, int part,
                              const double2* y, double2* fld, const int* skip, hipStream_t s) {
  const int F = part == kPartBoth ? 6 : 3;
  const long long rows = (long long)g.n2 * g.n3;
  const int P = pick_P_rows(g.n1, F, rows);
  const dim3 grid((unsigned)((rows + P - 1) / P));
  const size_t lds = lds_bytes(g.n1, F, P);
  if (part == kPartBoth)
    hipLaunchKernelGGL(k_x_inv_synth<kPartBoth>, grid, dim3(kThreads), lds, s, g, ax, t, y, fld, P, skip);
  else if (part == kPartP)
    hipLaunchKernelGGL(k_x_inv_synth<kPartP>, grid, dim3(kThreads), lds, s, g, ax, t, y, fld, P, skip);
  else
    hipLaunchKernelGGL(k_x_inv_synth<kPartQ>, grid, dim3(kThreads), lds, s, g, ax, t, y, fld, P, skip);
  return hipGetLastError();
}

hipError_t launch_x_fwd_proj(const Geom& g, const AxisPlan& ax, const Tables& t, int part,
                             const double2* fld, double2* out, const int* skip, hipStream_t s) {
  const int F = part == kPartBoth ? 6 : 3;
  const long long rows = (long long)g.n2 * g.n3;
  const int P = pick_P_rows(g.n1, F, rows);
  const dim3 grid((unsigned)((rows + P - 1) / P));
  const size_t lds = lds_bytes(g.n1, F, P);
  if (part == kPartBoth)
    hipLaunchKernelGGL(k_x_fwd_proj<kPartBoth>, grid, dim3(kThreads), lds, s, g, ax, t, fld, out, P, skip);
  else if (part == kPartP)
    hipLaunchKernelGGL(k_x_fwd_proj<kPartP>, grid, dim3(kThreads), lds, s, g, ax, t, fld, out, P, skip);
  else
    hipLaunchKernelGGL(k_x_fwd_proj<kPartQ>, grid, dim3(kThreads), lds, s, g, ax, t, fld, out, P, skip);
  return hipGetLastError();
}

hipError_t launch_yz_pass(const Geom& g, const AxisPlan& ax, const Tables& t, int axis, int dir,
                          int nf, double2* fld, int post_twist, int pre_twist, const int* skip,
                          hipStream_t s) {
  const int P = pick_P_cols(ax.N, 1, g.n1);
  const long long other = (axis == 1) ? g.n3 : g.n2;
  const dim3 grid((unsigned)((g.n1 / P) * other), (unsigned)nf);
  const size_t lds = lds_bytes(ax.N, 1, P);
  if (dir > 0)
    hipLaunchKernelGGL(k_yz_pass<+1>, grid, dim3(kThreads), lds, s, g, ax, t, axis, fld, P,
                       post_twist, pre_twist, skip);
  else
    hipLaunchKernelGGL(k_yz_pass<-1>, grid, dim3(kThreads), lds, s, g, ax, t, axis, fld, P,
                       post_twist, pre_twist, skip);
  return hipGetLastError();
}

hipError_t launch_z_mid(const Geom& g, const AxisPlan& ax, const Tables& t, const MediumView& med,
                        double2* fld, const int* skip, hipStream_t s) {
  const int P = pick_P_cols(ax.N, 6, g.n1);
  const dim3 grid((unsigned)((g.n1 / P) * g.n2));
  const size_t lds = lds_bytes(ax.N, 6, P);
  hipLaunchKernelGGL(k_z_mid, grid, dim3(kThreads), lds, s, g, ax, t, med, fld, P, skip);
  return hipGetLastError();
}

hipError_t launch_apply_Br(const Geom& g, const Tables& t, const double2* u, double2* out,
                           const int* skip, hipStream_t s) {
  long long blocks = (g.n + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(k_apply_Br, dim3((unsigned)blocks), dim3(256), 0, s, g, t, u, out, skip);
  return hipGetLastError();
}

}  // namespace nsf
