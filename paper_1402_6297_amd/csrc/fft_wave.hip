// Single-wave passes that keep the coupled field components of a pencil in
// registers (the default path for axis lengths N = N1 * N2 with N2 | N1).
//
// A workgroup is one 64-lane wave.  When all six components are involved the
// wave is split in halves: lanes 0..31 hold E' (three components), lanes
// 32..63 hold H' of the same pencils, so a half holds P = 32 / N2 pencils (or
// rows) with N2 lanes each; with three components the whole wave is one half.
// A lane holds, for each of its three components, the N1 points of its pencil
// that the two-level split assigns to it:
//   X[k1 + N1 k2] = sum_{n2} W_N^{n2 k1} [sum_{n1} x[n2 + N2 n1] W_{N1}^{n1 k1}] W_{N2}^{n2 k2}.
// After the N2-point DFTs lane t owns the outputs k1 + N1 k2 with
// k1 = t + d N2, i.e. exactly the positions t + N2 m, m = d + (N1/N2) k2,
// that its next N1-point DFT consumes.  So:
//  * the per-voxel middle factor of A_r (Thm 4.2) needs E' and H' of a voxel:
//    lane l and lane l ^ 32 trade their three components with cross-lane
//    shuffles and each keeps its half of the result, between the inverse and
//    the forward z transform, with no LDS traffic;
//  * the basis synthesis (Thm 2.5) computes pi_1, pi_2 per frequency and
//    writes the lane's components in registers before the inverse x
//    transform, and the projection consumes the forward x transform the same
//    way (E' lanes give y_a, y_b; H' lanes give y_c, y_d).
// LDS is used only for the one exchange inside each transform.  Every lane
// keeps many independent loads in flight, which is what hides HBM latency
// here (one wave per SIMD).
#include "nsf_internal.h"
#include "fft_common.h"

namespace nsf {
namespace {

template <int N1, int N2, int S>
__device__ __forceinline__ void w_step1(double2 (&v)[N1], int n2, const double2* twl) {
  reg_dft<N1, S>(v);
  if (n2 > 0) {
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      double2 t = twl[n2 * k1];
      if (S < 0) t = cconj(t);
      v[k1] = cmul(v[k1], t);
    }
  }
}

// Exchange through tile (element e of this lane's pencil at tile[e * ES + eo])
// and the N2-point DFTs.  On return v[d + (N1/N2) k2] = X[t + d N2 + N1 k2].
template <int N1, int N2, int S>
__device__ __forceinline__ void w_step2(double2 (&v)[N1], int t, double2* tile, int ES, int eo) {
  constexpr int D = N1 / N2;
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) tile[(t + N2 * k1) * ES + eo] = v[k1];
  __syncthreads();
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = t + d * N2;
    double2 u[N2];
#pragma unroll
    for (int m = 0; m < N2; ++m) u[m] = tile[(m + N2 * k1) * ES + eo];
    reg_dft<N2, S>(u);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) v[d + D * k2] = u[k2];
  }
  __syncthreads();
}

// ------------------------------------------------------- z pass with medium
// Blocks are remapped so that the two workgroups sharing a 128-byte line of
// every pencil row (adjacent x groups) run on the same XCD (workgroups are
// dispatched to the 8 XCDs round robin) and meet in its L2.
__device__ __forceinline__ long long xcd_pair_remap(long long b, long long nblk) {
  const long long span = nblk & ~15LL;  // the tail keeps the identity map
  if (b >= span) return b;
  const long long xcd = b & 7, slot = b >> 3;
  return (((slot >> 1) << 3) + xcd) * 2 + (slot & 1);
}

template <int N1, int N2>
__global__ __launch_bounds__(64) void k_wz_mid(Geom g, Tables t, MediumView med, double2* __restrict__ fld,
                                               const int* skip) {
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int P = 32 / N2;
  constexpr int D = N1 / N2;
  __shared__ double2 twl[N];
  __shared__ double2 tile[2 * N * P];
  const int twoff = g.n1 + g.n2;
  for (int i = threadIdx.x; i < N; i += 64) twl[i] = t.tw[twoff + i];
  const int h = threadIdx.x >> 5;
  const int q = threadIdx.x & 31;
  const int p = q % P;
  const int ln = q / P;
  const int groups1 = g.n1 / P;
  const long long blk = xcd_pair_remap(blockIdx.x, gridDim.x);
  const int i1_0 = (int)(blk % groups1) * P;
  const int i2 = (int)(blk / groups1);
  const unsigned n = (unsigned)g.n;
  const unsigned stride = (unsigned)(g.n1 * g.n2);
  double2* Fb = fld + (long long)i2 * g.n1 + i1_0;            // workgroup-uniform
  const double2* Mb = med.eg + (long long)i2 * g.n1 + i1_0;
  const unsigned lo = 3u * h * n + p + ln * stride;            // lane offset of position ln
  double2* T = tile + h * N * P;
  double2 v[3][N1];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[c][n1] = ld_off(Fb, lo + c * n + N2 * n1 * stride);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w_step1<N1, N2, +1>(v[c], ln, twl);
    w_step2<N1, N2, +1>(v[c], ln, T, P, p);
  }
  // lane holds z positions j = ln + N2 m of E' (h = 0) or H' (h = 1)
  const double inv_n = 1.0 / (double)g.n;
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    double2 mine[3], other[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mine[c] = v[c][m];
      other[c] = make_double2(__shfl_xor(mine[c].x, 32, 64), __shfl_xor(mine[c].y, 32, 64));
    }
    double2 E[3], H[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E[c] = h ? other[c] : mine[c];
      H[c] = h ? mine[c] : other[c];
    }
    medium_apply(med, ld_off(Mb, p + (ln + N2 * m) * stride), inv_n, E, H);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][m] = h ? H[c] : E[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w_step1<N1, N2, -1>(v[c], ln, twl);
    w_step2<N1, N2, -1>(v[c], ln, T, P, p);
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) st_off(Fb, lo + c * n + (d * N2 + N1 * k2) * stride, v[c][d + D * k2]);
  }
}

// ---------------------------------------------------------- x passes
// Halves: HV = 2 when all six components are involved (h = 0: E', h = 1: H'),
// else 1.  R = 64 / (HV N2) rows per wave; lane (h, r, t) with t fastest; the
// exchange tile of (h, r) is tile[(h R + r) (N + 1) + e].
template <int N1, int N2, int PART>
__global__ __launch_bounds__(64) void k_wx_inv_synth(Geom g, Tables t, const double2* __restrict__ y,
                                                     double2* __restrict__ fld, const int* skip) {
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int HV = (PART == kPartBoth) ? 2 : 1;
  constexpr int R = 64 / (HV * N2);
  constexpr int D = N1 / N2;
  __shared__ double2 twl[N];
  __shared__ double2 tile[HV * R * (N + 1)];
  for (int i = threadIdx.x; i < N; i += 64) twl[i] = t.tw[i];
  const int ln = threadIdx.x % N2;
  const int r = (threadIdx.x / N2) % R;
  const int h = threadIdx.x / (N2 * R);
  const long long rows = (long long)g.n2 * g.n3;
  const long long row = (long long)blockIdx.x * R + r;
  const bool live = row < rows;
  const long long rr = live ? row : rows - 1;  // dead lanes compute a valid row and store nothing
  const int i2 = (int)(rr % g.n2), i3 = (int)(rr / g.n2);
  const unsigned n = (unsigned)g.n;
  // which coefficient pair feeds this lane: (y_a, y_b) -> E', (y_c, y_d) -> H'
  const bool isH = (PART == kPartQ) || (PART == kPartBoth && h == 1);
  const unsigned in0 = (PART == kPartBoth && h == 1) ? 2u * n : 0u;
  const long long row_first = (long long)blockIdx.x * R;
  const double2* Yb = y + row_first * N;                      // workgroup-uniform
  const unsigned lrow = (unsigned)(rr - row_first) * N;      // lane row offset
  double2 v[3][N1];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) {
    const int i1 = ln + N2 * n1;
    Basis B;
    basis_at(t.lam, g, i1, i2, i3, B);
    const double2 y0 = ld_off(Yb, in0 + lrow + i1), y1 = ld_off(Yb, in0 + n + lrow + i1);
#pragma unroll
    for (int c = 0; c < 3; ++c)
      v[c][n1] = isH ? cadd(cmul(B.pi1[c], y0), cmul(B.pi2[c], y1))    // h = pi1 y_c + pi2 y_d
                     : csub(cmulc(B.pi1[c], y1), cmulc(B.pi2[c], y0));  // e = -conj(pi2) y_a + conj(pi1) y_b
  }
  __syncthreads();
  double2* T = tile + (h * R + r) * (N + 1);
  double2* Ob = fld + row_first * N;
  const unsigned lo = 3u * h * n + lrow + ln;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w_step1<N1, N2, +1>(v[c], ln, twl);
    w_step2<N1, N2, +1>(v[c], ln, T, 1, 0);
    if (live) {
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) st_off(Ob, lo + c * n + d * N2 + N1 * k2, v[c][d + D * k2]);
    }
  }
}

template <int N1, int N2, int PART>
__global__ __launch_bounds__(64) void k_wx_fwd_proj(Geom g, Tables t, const double2* __restrict__ fld,
                                                    double2* __restrict__ out, const int* skip) {
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int HV = (PART == kPartBoth) ? 2 : 1;
  constexpr int R = 64 / (HV * N2);
  constexpr int D = N1 / N2;
  __shared__ double2 twl[N];
  __shared__ double2 tile[HV * R * (N + 1)];
  for (int i = threadIdx.x; i < N; i += 64) twl[i] = t.tw[i];
  const int ln = threadIdx.x % N2;
  const int r = (threadIdx.x / N2) % R;
  const int h = threadIdx.x / (N2 * R);
  const long long rows = (long long)g.n2 * g.n3;
  const long long row = (long long)blockIdx.x * R + r;
  const bool live = row < rows;
  const long long rr = live ? row : rows - 1;
  const int i2 = (int)(rr % g.n2), i3 = (int)(rr / g.n2);
  const unsigned n = (unsigned)g.n;
  const bool isH = (PART == kPartQ) || (PART == kPartBoth && h == 1);
  const long long row_first = (long long)blockIdx.x * R;
  const double2* Fb = fld + row_first * N;                    // workgroup-uniform
  const unsigned lrow = (unsigned)(rr - row_first) * N;
  const unsigned lo = 3u * h * n + lrow + ln;
  double2 v[3][N1];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[c][n1] = ld_off(Fb, lo + c * n + N2 * n1);
  __syncthreads();
  double2* T = tile + (h * R + r) * (N + 1);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    w_step1<N1, N2, -1>(v[c], ln, twl);
    w_step2<N1, N2, -1>(v[c], ln, T, 1, 0);
  }
  if (!live) return;
  // E' lanes give (a, b) = (-pi2^T o1, pi1^T o1); H' lanes give
  // (c, d) = (pi1^* o2, pi2^* o2).  Output block pair at out + o0.
  const unsigned o0 = (PART == kPartBoth && h == 1) ? 2u * n : 0u;
  double2* Ob = out + row_first * N;
#pragma unroll
  for (int d = 0; d < D; ++d)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) {
      const int m = d + D * k2;
      const int i1 = ln + d * N2 + N1 * k2;
      const unsigned f = lrow + i1;
      Basis B;
      basis_at(t.lam, g, i1, i2, i3, B);
      double2 r0 = make_double2(0, 0), r1 = make_double2(0, 0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (isH) {
          r0 = cadd(r0, cmulc(B.pi1[c], v[c][m]));
          r1 = cadd(r1, cmulc(B.pi2[c], v[c][m]));
        } else {
          r0 = csub(r0, cmul(B.pi2[c], v[c][m]));
          r1 = cadd(r1, cmul(B.pi1[c], v[c][m]));
        }
      }
      st_off(Ob, o0 + f, r0);
      st_off(Ob, o0 + n + f, r1);
    }
}

#define NSF_WAVE_SWITCH(N, MACRO) \
  switch (N) {                    \
    case 128: MACRO(16, 8); break; \
    case 64: MACRO(8, 8); break;   \
    case 32: MACRO(8, 4); break;   \
    case 16: MACRO(4, 4); break;   \
    default: return hipErrorInvalidValue; \
  }

int wave_n2(int N) {
  switch (N) {
    case 128: return 8;
    case 64: return 8;
    case 32: return 4;
    case 16: return 4;
    default: return 0;
  }
}

}  // namespace

// The lane offsets are 32-bit byte offsets: six fields of n elements must stay
// below 2^32 bytes.
static bool wave_size_ok(const Geom& g) { return g.n <= (1LL << 32) / (16 * 6); }

bool wave_axis(int N) { return wave_n2(N) > 0; }

bool wave_mid_ok(const Geom& g) {
  const int n2w = wave_n2(g.n3);
  return n2w > 0 && g.n1 % (32 / n2w) == 0 && wave_size_ok(g);
}

hipError_t launch_wave_z_mid(const Geom& g, const Tables& t, const MediumView& med, double2* fld,
                             const int* skip, hipStream_t s) {
  if (!wave_mid_ok(g)) return hipErrorInvalidValue;
  const int P = 32 / wave_n2(g.n3);
  const dim3 grid((unsigned)((g.n1 / P) * g.n2));
#define L_WM(A, B) hipLaunchKernelGGL((k_wz_mid<A, B>), grid, dim3(64), 0, s, g, t, med, fld, skip);
  NSF_WAVE_SWITCH(g.n3, L_WM)
#undef L_WM
  return hipGetLastError();
}

hipError_t launch_wave_x_inv_synth(const Geom& g, const Tables& t, int part, const double2* y,
                                   double2* fld, const int* skip, hipStream_t s) {
  const int n2w = wave_n2(g.n1);
  if (!n2w || !wave_size_ok(g)) return hipErrorInvalidValue;
  const int R = 64 / ((part == kPartBoth ? 2 : 1) * n2w);
  const long long rows = (long long)g.n2 * g.n3;
  const dim3 grid((unsigned)((rows + R - 1) / R));
#define L_WXI(A, B)                                                                                     \
  if (part == kPartBoth)                                                                                \
    hipLaunchKernelGGL((k_wx_inv_synth<A, B, kPartBoth>), grid, dim3(64), 0, s, g, t, y, fld, skip);    \
  else if (part == kPartP)                                                                              \
    hipLaunchKernelGGL((k_wx_inv_synth<A, B, kPartP>), grid, dim3(64), 0, s, g, t, y, fld, skip);       \
  else                                                                                                  \
    hipLaunchKernelGGL((k_wx_inv_synth<A, B, kPartQ>), grid, dim3(64), 0, s, g, t, y, fld, skip);
  NSF_WAVE_SWITCH(g.n1, L_WXI)
#undef L_WXI
  return hipGetLastError();
}

hipError_t launch_wave_x_fwd_proj(const Geom& g, const Tables& t, int part, const double2* fld,
                                  double2* out, const int* skip, hipStream_t s) {
  const int n2w = wave_n2(g.n1);
  if (!n2w || !wave_size_ok(g)) return hipErrorInvalidValue;
  const int R = 64 / ((part == kPartBoth ? 2 : 1) * n2w);
  const long long rows = (long long)g.n2 * g.n3;
  const dim3 grid((unsigned)((rows + R - 1) / R));
#define L_WXF(A, B)                                                                                      \
  if (part == kPartBoth)                                                                                 \
    hipLaunchKernelGGL((k_wx_fwd_proj<A, B, kPartBoth>), grid, dim3(64), 0, s, g, t, fld, out, skip);    \
  else if (part == kPartP)                                                                               \
    hipLaunchKernelGGL((k_wx_fwd_proj<A, B, kPartP>), grid, dim3(64), 0, s, g, t, fld, out, skip);       \
  else                                                                                                   \
    hipLaunchKernelGGL((k_wx_fwd_proj<A, B, kPartQ>), grid, dim3(64), 0, s, g, t, fld, out, skip);
  NSF_WAVE_SWITCH(g.n1, L_WXF)
#undef L_WXF
  return hipGetLastError();
}

}  // namespace nsf
