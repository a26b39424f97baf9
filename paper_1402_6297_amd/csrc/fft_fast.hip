// Register-resident pencil passes for axis lengths N = N1 * N2 (the fast path).
//
// Each length-N transform of a pencil is split as
//   X[k1 + N1 k2] = sum_{n2} W_N^{n2 k1} [ sum_{n1} x[n2 + N2 n1] W_{N1}^{n1 k1} ] W_{N2}^{n2 k2}:
// N2 threads per pencil; thread n2 loads its N1 points straight from global
// memory, does the N1-point DFT in registers and the twiddle, one LDS
// exchange hands every thread the N2 values of its k1's, and the N2-point
// DFTs write natural-order results straight back to global memory.  Compared
// with staging every radix stage through LDS this needs one exchange per
// transform and few registers, so several workgroups share a CU and hide HBM
// latency.  The fused steps (basis synthesis, per-voxel middle factor,
// projection, twist) are the same as in the generic passes.
#include "nsf_internal.h"
#include "fft_common.h"

namespace nsf {
namespace {

// ----------------------------------------------------------- two-level core
// Step 1 for one thread: v[n1] = x[n2 + N2 n1] -> B[k1] * W_N^{S n2 k1}.
template <int N1, int N2, int S>
__device__ __forceinline__ void step1(double2 (&v)[N1], int n2, const double2* twl) {
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

template <int N1, int N2>
struct Split {
  static constexpr int N = N1 * N2;
  static constexpr int D = (N1 + N2 - 1) / N2;  // step-2 transforms per thread
};

// The y/z passes exchange between the two steps in PH phases of up to RP rows
// k1 (each of N2 elements), so that their LDS tile holds RP rows, not N1.  The
// forward passes (S < 0) take two phases when a thread has two or more step-2
// transforms: half the LDS per pencil, twice the workgroups per CU (LDS, not
// registers, limits them), measured faster; the inverse passes ran slower so
// and keep one.
struct YzPhases {
  int PH, DP, RP, rows;
};
__host__ __device__ constexpr YzPhases yz_phases(int N1, int N2, int S) {
  const int D = (N1 + N2 - 1) / N2;
  const int PH = D > 1 && S < 0 ? 2 : 1;
  const int DP = (D + PH - 1) / PH;
  const int RP = DP * N2;
  return YzPhases{PH, DP, RP, RP < N1 ? RP : N1};
}

// ------------------------------------------------------------ y / z passes
// P pencils (consecutive x) per workgroup, N2 threads per pencil, lane order
// p fastest.  LDS tile[(e) * P + p], e = n2 + N2 k1.
// ysc > 0 (vacuum skipping, y axis): the grid covers nxg groups of P x columns
// per z, taken from the list xg (batched: each instance's med.xgroups, nxg the
// largest count); the results are scaled by ysc.  A group left out has no
// voxel other than vacuum, so the y transforms around the z pass cancel there.
template <int N1, int N2, int S, bool BT = false>
__global__ __launch_bounds__(256) void k_fyz(Geom g, Tables t, int axis, double2* __restrict__ fld,
                                             int P, int post_twist, int pre_twist, const int* skip,
                                             const InstDesc* __restrict__ insts, const int* xg, int nxg,
                                             double ysc) {
  int mine = nxg;
  if constexpr (BT) {
    const InstDesc& d = insts[blockIdx.z];
    t = d.t;
    fld = d.fld;
    skip = d.skip;
    xg = d.med.xgroups;
    mine = d.med.nxgroups;
  }
  if (skip && *skip) return;
  const int groups1 = g.n1 / P;
  const int ng = ysc > 0.0 ? nxg : groups1;
  const int gsel = (int)(blockIdx.x % (unsigned)ng);
  if (ysc > 0.0 && gsel >= mine) return;  // batched: this instance lists fewer groups
  constexpr int N = N1 * N2;
  constexpr int D = Split<N1, N2>::D;
  extern __shared__ double2 sm[];
  double2* twl = sm;
  double2* tile = sm + N;
  const int twoff = (axis == 1) ? g.n1 : g.n1 + g.n2;
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = t.tw[twoff + i];
  const int p = threadIdx.x % P;
  const int n2 = threadIdx.x / P;
  const int i1_0 = (ysc > 0.0 ? xg[gsel] : gsel) * P;
  const int io = (int)(blockIdx.x / (unsigned)ng);
  long long base, stride;
  if (axis == 1) {
    base = (long long)io * g.n1 * g.n2 + i1_0;
    stride = g.n1;
  } else {
    base = (long long)io * g.n1 + i1_0;
    stride = (long long)g.n1 * g.n2;
  }
  double2* F = fld + (long long)blockIdx.y * g.n + base + p;
  const double rs = 1.0 / sqrt((double)g.n);
  double2 v[N1];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) {
    const int j = n2 + N2 * n1;
    double2 x = F[j * stride];
    if (pre_twist) x = cscale(cmulc(twist_at(t.twist, g, i1_0 + p, io, j), x), rs);
    v[n1] = x;
  }
  __syncthreads();  // twiddle table ready
  step1<N1, N2, S>(v, n2, twl);
  constexpr YzPhases Y = yz_phases(N1, N2, S);
#pragma unroll
  for (int ph = 0; ph < Y.PH; ++ph) {
    if (ph > 0) __syncthreads();  // the previous phase's rows have been read
#pragma unroll
    for (int kl = 0; kl < Y.RP; ++kl) {
      const int k1 = ph * Y.RP + kl;
      if (k1 < N1) tile[(n2 + N2 * kl) * P + p] = v[k1];
    }
    __syncthreads();
#pragma unroll
    for (int dd = 0; dd < Y.DP; ++dd) {
      const int k1 = n2 + (ph * Y.DP + dd) * N2;
      if (ph * Y.DP + dd < D && k1 < N1) {
        const int kl = n2 + dd * N2;  // k1's row in this phase
        double2 u[N2];
#pragma unroll
        for (int m = 0; m < N2; ++m) u[m] = tile[(m + N2 * kl) * P + p];
        reg_dft<N2, S>(u);
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
          const int j = k1 + N1 * k2;
          double2 x = u[k2];
          if (post_twist) x = cscale(cmul(twist_at(t.twist, g, i1_0 + p, io, j), x), rs);
          if (ysc > 0.0) x = cscale(x, ysc);
          F[j * stride] = x;
        }
      }
    }
  }
}

// ------------------------------------------------------ z pass with medium
template <int N1, int N2, bool BT = false>
__global__ __launch_bounds__(384) void k_fz_mid(Geom g, Tables t, MediumView med,
                                                double2* __restrict__ fld, int P, const int* skip,
                                                const InstDesc* __restrict__ insts) {
  if constexpr (BT) {
    const InstDesc& d = insts[blockIdx.z];
    t = d.t;
    med = d.med;
    fld = d.fld;
    skip = d.skip;
  }
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int D = Split<N1, N2>::D;
  extern __shared__ double2 sm[];
  double2* twl = sm;
  double2* tile = sm + N;  // [(c * N + e) * P + p]
  const int twoff = g.n1 + g.n2;
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = t.tw[twoff + i];
  const int p = threadIdx.x % P;
  const int n2 = (threadIdx.x / P) % N2;
  const int c = threadIdx.x / (P * N2);
  const int groups1 = g.n1 / P;
  const int i1_0 = (int)(blockIdx.x % groups1) * P;
  const int i2 = (int)(blockIdx.x / groups1);
  const long long base = (long long)i2 * g.n1 + i1_0;
  const long long stride = (long long)g.n1 * g.n2;
  const long long n = g.n;
  double2* F = fld + c * n + base + p;
  double2* T = tile + c * N * P + p;
  double2 v[N1];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) v[n1] = F[(n2 + N2 * n1) * stride];
  __syncthreads();
  // inverse z
  step1<N1, N2, +1>(v, n2, twl);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) T[(n2 + N2 * k1) * P] = v[k1];
  __syncthreads();
  double2 out[D][N2];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
#pragma unroll
      for (int m = 0; m < N2; ++m) out[d][m] = T[(m + N2 * k1) * P];
      reg_dft<N2, +1>(out[d]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) T[(k1 + N1 * k2) * P] = out[d][k2];
    }
  }
  __syncthreads();
  // per-voxel middle factor (times 1/n)
  const double inv_n = 1.0 / (double)n;
  for (int vx = threadIdx.x; vx < P * N; vx += blockDim.x) {
    const int pp = vx % P, j = vx / P;
    double2 E[3], H[3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      E[cc] = tile[(cc * N + j) * P + pp];
      H[cc] = tile[((3 + cc) * N + j) * P + pp];
    }
    medium_apply_at(med, base + j * stride + pp, inv_n, E, H);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      tile[(cc * N + j) * P + pp] = E[cc];
      tile[((3 + cc) * N + j) * P + pp] = H[cc];
    }
  }
  __syncthreads();
  // forward z
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) v[n1] = T[(n2 + N2 * n1) * P];
  __syncthreads();
  step1<N1, N2, -1>(v, n2, twl);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) T[(n2 + N2 * k1) * P] = v[k1];
  __syncthreads();
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
      double2 u[N2];
#pragma unroll
      for (int m = 0; m < N2; ++m) u[m] = T[(m + N2 * k1) * P];
      reg_dft<N2, -1>(u);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) F[(k1 + N1 * k2) * stride] = u[k2];
    }
  }
}

// ------------------------------------------- z pass with medium, field pairs
// The constitutive step couples the six fields only in pairs: chiral media pair
// E'_c with H'_c; pseudochiral media with coupled axes (a, b) pair E'_a with
// H'_b and E'_b with H'_a, and leave E'_o, H'_o (o the third axis) uncoupled.
// In every pair the step is e' = (eps e - i g h) s, h' = (i g e + h) s with
// s = 1/(n (eps - g^2)), where g = gamma for a coupled pair and g = 0 for the
// uncoupled one.  One workgroup transforms one pair of P z-pencil columns, so
// its LDS tile is a third of the six-field tile; the three pairs of a tile go
// to the same XCD one after another (when the tile count is a multiple of 8),
// so the medium they all read is served from that XCD's L2.
//
// With z = n2 + N2 n1 and frequency k = k1 + N1 k2, the inverse transform
// leaves each thread with its field at the positions k1 + N1 k2 of its k1 and
// every k2.  The constitutive step runs there (the partner field comes through
// LDS), and the forward transform starts from the same distribution: a radix-N2
// transform over k2 in registers, the twiddle w^-(k1 m2), one LDS exchange, and
// a radix-N1 transform over k1 that yields the outputs m2 + N2 m1 at exactly the
// addresses the thread loaded.
// vs > 0 (vacuum skipping): the workgroups cover only the tiles listed in
// med.ztiles (a tile is P columns of one y; listed when one of its voxels is
// not vacuum), the constitutive step scales by vs = 1 / n3 instead of 1 / n
// (the forward y and x passes apply 1 / n2 and 1 / n1), and a column left out
// keeps its input, which is what the inverse z, identity, forward z sequence
// scaled by 1 / n3 returns there.  The partial sums then hold Re f^* (M - I) f / n; the
// first CG pass adds |p|^2 = sum |f|^2 / n.
template <int N1, int N2, bool BT = false, bool PQ = false>
__global__ __launch_bounds__(256) void k_fz_pair(Geom g, Tables t, MediumView med,
                                                 double2* __restrict__ fld, int P, const int* skip,
                                                 const InstDesc* __restrict__ insts, double* part_mid, double vs) {
  if constexpr (BT) {
    const InstDesc& d = insts[blockIdx.z];
    t = d.t;
    med = d.med;
    fld = d.fld;
    skip = d.skip;
    part_mid = d.cg.part_mid;
  }
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int D = Split<N1, N2>::D;
  const int groups1 = g.n1 / P;
  const unsigned tiles = vs > 0.0 ? (unsigned)med.nztiles : (unsigned)groups1 * (unsigned)g.n2;
  if (blockIdx.x >= 3u * tiles) {  // batched: this instance has fewer listed tiles
    if (PQ && threadIdx.x == 0) part_mid[blockIdx.x] = 0.0;
    return;
  }
  extern __shared__ double2 sm[];
  double2* twl = sm;
  double2* tile = sm + N;  // [(h * N + e) * P + p], h = 0 (E field), 1 (H field)
  const int twoff = g.n1 + g.n2;
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = t.tw[twoff + i];
  unsigned tix, q;
  if ((tiles & 7u) == 0) {
    const unsigned sq = blockIdx.x >> 3;
    q = sq % 3u;
    tix = (blockIdx.x & 7u) + 8u * (sq / 3u);
  } else {
    q = blockIdx.x % 3u;
    tix = blockIdx.x / 3u;
  }
  if (vs > 0.0) tix = (unsigned)med.ztiles[tix];
  int fe, fh;
  bool coupled = true;
  if (med.kind == kMedChiral) {
    fe = (int)q;
    fh = 3 + (int)q;
  } else if (q == 0) {
    fe = med.pa;
    fh = 3 + med.pb;
  } else if (q == 1) {
    fe = med.pb;
    fh = 3 + med.pa;
  } else {
    fe = med.po;
    fh = 3 + med.po;
    coupled = false;
  }
  const int p = threadIdx.x % P;
  const int n2 = (threadIdx.x / P) % N2;
  const int h = threadIdx.x / (P * N2);
  const int i1_0 = (int)(tix % (unsigned)groups1) * P;
  const int i2 = (int)(tix / (unsigned)groups1);
  const long long base = (long long)i2 * g.n1 + i1_0;
  const long long stride = (long long)g.n1 * g.n2;
  const long long n = g.n;
  double2* F = fld + (h == 0 ? fe : fh) * n + base + p;
  double2* T = tile + h * N * P + p;
  const double2* Tq = tile + (1 - h) * N * P + p;  // the partner field
  const double2* eg = med.eg + base + p;
  double2 v[N1];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1) v[n1] = F[(n2 + N2 * n1) * stride];
  __syncthreads();  // twiddles ready
  // inverse z
  step1<N1, N2, +1>(v, n2, twl);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) T[(n2 + N2 * k1) * P] = v[k1];
  __syncthreads();
  // the medium at this thread's positions k1 + N1 k2, in flight during the
  // second radix
  double2 mv[D][N2];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) mv[d][k2] = eg[(k1 + N1 * k2) * stride];
    }
  }
  double2 out[D][N2];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
#pragma unroll
      for (int m = 0; m < N2; ++m) out[d][m] = T[(m + N2 * k1) * P];
      reg_dft<N2, +1>(out[d]);
    }
  }
  __syncthreads();
  // constitutive step at this thread's positions k1 + N1 k2 (times 1/n)
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) T[(k1 + N1 * k2) * P] = out[d][k2];
    }
  }
  __syncthreads();
  const double inv_n = 1.0 / (double)n;
  const double zs = vs > 0.0 ? vs : inv_n;  // scale of the constitutive step
  const double pq_s = inv_n / zs;
  double pq[1] = {0.0};  // Re f^* (M f) / n (vs > 0: Re f^* (M - I) f / n): this thread's share of p^* A_r p
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        const int z = k1 + N1 * k2;
        const double2 m = mv[d][k2];
        const double eps = m.x, gm = coupled ? m.y : 0.0;
        const double sc = zs / (eps - gm * gm);
        const double2 other = Tq[z * P];
        const double2 own = out[d][k2];
        out[d][k2] = (h == 0) ? cscale(csub(cscale(own, eps), cmuli(cscale(other, gm))), sc)
                              : cscale(cadd(cmuli(cscale(other, gm)), own), sc);
        if (PQ) {
          pq[0] += (own.x * out[d][k2].x + own.y * out[d][k2].y) * pq_s;
          if (vs > 0.0) pq[0] -= cabs2(own) * inv_n;
        }
      }
    }
  }
  if (PQ) {
    block_sum_k<1>(pq);  // synchronises the workgroup
    if (threadIdx.x == 0) part_mid[blockIdx.x] = pq[0];
  }
  __syncthreads();  // partner values read before the tile is reused
  // forward z: radix N2 over k2, twiddle, exchange, radix N1 over k1
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
      reg_dft<N2, -1>(out[d]);
#pragma unroll
      for (int m2 = 0; m2 < N2; ++m2) {
        double2 x = out[d][m2];
        if (k1 > 0 && m2 > 0) x = cmul(x, cconj(twl[k1 * m2]));
        T[(m2 * N1 + k1) * P] = x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) v[k1] = T[(n2 * N1 + k1) * P];
  reg_dft<N1, -1>(v);
#pragma unroll
  for (int m1 = 0; m1 < N1; ++m1) F[(n2 + N2 * m1) * stride] = v[m1];
}

// ------------------------------------------------------------- x passes
// LDS rows of the x passes hold N elements each, row after row, with element e
// of row r (r = row within the workgroup) at e ^ ((a (e >> s) + b r) & 15): an
// XOR swizzle of the 16-element (256-byte) bank groups, chosen per split N1 x N2
// so that the 16-lane groups of the strided second-radix reads, the first-radix
// accesses and the synthesis / projection sweeps hit distinct 16-byte slots
// (found by enumerating (s, a, b) against those access patterns).  Measured, the
// swizzle pays in the forward projection pass and not in the inverse synthesis
// pass (whose index arithmetic it lengthens), so only the former uses it.
template <int N1, int N2>
struct XSwz {
  static constexpr int s = 3, a = 0, b = 0;
};
template <> struct XSwz<16, 8> { static constexpr int s = 3, a = 1, b = 8; };
template <> struct XSwz<8, 8> { static constexpr int s = 3, a = 1, b = 8; };
template <> struct XSwz<16, 16> { static constexpr int s = 4, a = 1, b = 0; };
template <> struct XSwz<16, 6> { static constexpr int s = 5, a = 9, b = 7; };
template <> struct XSwz<16, 3> { static constexpr int s = 3, a = 0, b = 12; };
template <> struct XSwz<8, 4> { static constexpr int s = 3, a = 0, b = 5; };
template <> struct XSwz<4, 4> { static constexpr int s = 3, a = 0, b = 5; };
template <int N1, int N2, bool SW>
__device__ __forceinline__ int xpos(int e, int r) {
  using W = XSwz<N1, N2>;
  return SW ? e ^ ((((e >> W::s) * W::a) + r * W::b) & 15) : e;
}

// R rows per workgroup; LDS tile[(c * R + r) * N + xpos(e, r)].
// QF (with CG): the q-free schedule, whose last pass has already updated r.
template <int N1, int N2, int PART, bool CG = false, bool BT = false, bool QF = false, bool PF = false>
__global__ __launch_bounds__(384) void k_fx_inv_synth(Geom g, Tables t, const double2* __restrict__ y,
                                                      double2* __restrict__ fld, int R,
                                                      const int* skip, CgFuse cg,
                                                      const InstDesc* __restrict__ insts) {
  if constexpr (BT) {
    const InstDesc& d = insts[blockIdx.z];
    t = d.t;
    y = d.vin;
    fld = d.fld;
    skip = d.skip;
    cg = d.cg;
  }
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int NP = N;
  constexpr int D = Split<N1, N2>::D;
  constexpr int F = (PART == kPartBoth) ? 6 : 3;
  extern __shared__ double2 sm[];
  double2* twl = sm;
  double2* tile = sm + N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = t.tw[i];
  const long long rows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * R;
  const long long n = g.n;
  double rr_acc[1] = {0.0};
  double pn_acc[1] = {0.0};  // |p|^2 of this workgroup's frequencies (cg.pnorm, q-free)
  int cg_iter = 0;
  double cg_al = 0, cg_be = 0;
  // p of the previous iteration is read from pin and the new p written to
  // pout: the same vector, or (q-free with kept directions) ring slots
  // (k - 1) mod K and k mod K, in which case x is not updated here
  const double2* pin = nullptr;
  double2* pout = nullptr;
  bool ring = false;
  if (CG) {
    cg_iter = cg.st->iter;
    cg_al = cg.st->alpha;
    cg_be = cg.st->beta;
    pin = cg.p;
    pout = cg.p;
    const int K = QF && cg.ring ? cg.st->ring : 0;
    if (K > 0) {
      ring = true;
      pin = cg.ring + (long long)((cg_iter > 0 ? cg_iter - 1 : 0) % K) * 4 * g.n;
      pout = cg.ring + (long long)(cg_iter % K) * 4 * g.n;
    }
  }
  // synthesis of the coefficient fields at frequency slot e of the workgroup
  auto synth = [&](int e) {
    const int r = e / N, i1 = e - r * N;
    const long long row = row0 + r;
    if (row >= rows) return;
    const int i2 = (int)(row % g.n2), i3 = (int)(row / g.n2);
    const long long f = row * N + i1;
    double2 yv[4];
    if (CG) {
      // CG recurrences of the previous iteration, then this iteration's p;
      // every load is issued before the stores (which may alias them)
      double2 po[4], qo[4], ro[4], xo[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) po[b] = pin[b * n + f];
      if (QF && cg_iter > 0) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          ro[b] = cg.r[b * n + f];
          if (!ring) xo[b] = cg.x[b * n + f];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const long long o = b * n + f;
          const double2 pn = make_double2(ro[b].x + cg_be * po[b].x, ro[b].y + cg_be * po[b].y);
          if (!ring) st_stream(cg.x + o, make_double2(xo[b].x + cg_al * po[b].x, xo[b].y + cg_al * po[b].y));
          st_stream(pout + o, pn);
          yv[b] = pn;
          pn_acc[0] += cabs2(pn);
        }
      } else if (cg_iter > 0) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          qo[b] = cg.q[b * n + f];
          ro[b] = cg.r[b * n + f];
          xo[b] = cg.x[b * n + f];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const long long o = b * n + f;
          const double2 rv = make_double2(ro[b].x - cg_al * qo[b].x, ro[b].y - cg_al * qo[b].y);
          const double2 xv = make_double2(xo[b].x + cg_al * po[b].x, xo[b].y + cg_al * po[b].y);
          const double2 pn = make_double2(rv.x + cg_be * po[b].x, rv.y + cg_be * po[b].y);
          st_stream(cg.r + o, rv);
          st_stream(cg.x + o, xv);
          st_stream(cg.p + o, pn);
          rr_acc[0] += cabs2(rv);
          yv[b] = pn;
        }
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          yv[b] = po[b];
          pn_acc[0] += cabs2(po[b]);
        }
      }
    }
    Basis B;
    basis_at(t.lam, g, i1, i2, i3, B);
    if (PART == kPartBoth || PART == kPartP) {
      const double2 ya = CG ? yv[0] : y[f], yb = CG ? yv[1] : y[n + f];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        tile[(cc * R + r) * NP + xpos<N1, N2, false>(i1, r)] = csub(cmulc(B.pi1[cc], yb), cmulc(B.pi2[cc], ya));
    }
    if (PART == kPartBoth || PART == kPartQ) {
      const long long o = (PART == kPartBoth) ? 2 * n : 0;
      const int cb = (PART == kPartBoth) ? 3 : 0;
      const double2 yc = CG ? yv[2] : y[o + f], yd = CG ? yv[3] : y[o + n + f];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        tile[((cb + cc) * R + r) * NP + xpos<N1, N2, false>(i1, r)] = cadd(cmul(B.pi1[cc], yc), cmul(B.pi2[cc], yd));
    }
  };
  // this thread's slots are e = threadIdx.x + it * blockDim.x (blockDim = F R N2
  // for R N frequencies); with the CG update the loop is unrolled so that each
  // slot's loads are issued together
  if constexpr (PF && PART == kPartBoth && (!CG || QF)) {
    // every global load of every slot first, then the updates, stores and
    // synthesis slot by slot (the stores of one slot cannot hold up the loads
    // of the next).  Used by the q-free CG first pass: measured 1.2% off the
    // 128^3 eigensolve (180 registers); the plain apply keeps the loop below,
    // which ran as fast.
    constexpr int IT = (N1 + F - 1) / F;
    double2 a0[IT][4], a1[IT][4], a2[IT][4];
    long long fo[IT];
    int i1v[IT], rv_[IT];
    bool ok[IT];
    const bool upd = CG && cg_iter > 0;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + it * blockDim.x;
      const int r = e / N, i1 = e - r * N;
      ok[it] = e < R * N && row0 + r < rows;
      rv_[it] = r;
      i1v[it] = i1;
      fo[it] = (row0 + r) * N + i1;
      if (ok[it]) {
#pragma unroll
        for (int b = 0; b < 4; ++b) a0[it][b] = CG ? pin[b * n + fo[it]] : y[b * n + fo[it]];
        if (upd) {
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            a1[it][b] = cg.r[b * n + fo[it]];
            if (!ring) a2[it][b] = cg.x[b * n + fo[it]];
          }
        }
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      if (!ok[it]) continue;
      const long long f = fo[it];
      const int r = rv_[it], i1 = i1v[it];
      const long long row = row0 + r;
      const int i2 = (int)(row % g.n2), i3 = (int)(row / g.n2);
      double2 yv[4];
      if (upd) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const long long o = b * n + f;
          const double2 po = a0[it][b];
          const double2 pn = make_double2(a1[it][b].x + cg_be * po.x, a1[it][b].y + cg_be * po.y);
          if (!ring)
            st_stream(cg.x + o, make_double2(a2[it][b].x + cg_al * po.x, a2[it][b].y + cg_al * po.y));
          st_stream(pout + o, pn);
          yv[b] = pn;
        }
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) yv[b] = a0[it][b];
      }
      if (CG) {
#pragma unroll
        for (int b = 0; b < 4; ++b) pn_acc[0] += cabs2(yv[b]);
      }
      Basis B;
      basis_at(t.lam, g, i1, i2, i3, B);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        tile[(cc * R + r) * NP + i1] = csub(cmulc(B.pi1[cc], yv[1]), cmulc(B.pi2[cc], yv[0]));
        tile[((3 + cc) * R + r) * NP + i1] = cadd(cmul(B.pi1[cc], yv[2]), cmul(B.pi2[cc], yv[3]));
      }
    }
  } else if constexpr (CG) {
    constexpr int IT = (N1 + F - 1) / F;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + it * blockDim.x;
      if (e < R * N) synth(e);
    }
  } else {
    for (int e = threadIdx.x; e < R * N; e += blockDim.x) synth(e);
  }
  if (CG && !QF) {
    block_sum_k<1>(rr_acc);
    if (threadIdx.x == 0) cg.part_in[blockIdx.x] = rr_acc[0];
  } else if (CG && cg.pnorm) {
    block_sum_k<1>(pn_acc);
    if (threadIdx.x == 0) cg.part_in[blockIdx.x] = pn_acc[0];
  }
  __syncthreads();
  const int n2 = threadIdx.x % N2;
  const int r = (threadIdx.x / N2) % R;
  const int c = threadIdx.x / (N2 * R);
  const bool active = c < F && row0 + r < rows;
  double2* T = tile + (c * R + r) * NP;
  double2 v[N1];
  if (active) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = T[xpos<N1, N2, false>(n2 + N2 * n1, r)];
    step1<N1, N2, +1>(v, n2, twl);
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) T[xpos<N1, N2, false>(n2 + N2 * k1, r)] = v[k1];
  }
  __syncthreads();
  if (!active) return;
  double2* out = fld + c * n + (row0 + r) * N;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int k1 = n2 + d * N2;
    if (k1 < N1) {
      double2 u[N2];
#pragma unroll
      for (int m = 0; m < N2; ++m) u[m] = T[xpos<N1, N2, false>(m + N2 * k1, r)];
      reg_dft<N2, +1>(u);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) out[k1 + N1 * k2] = u[k2];
    }
  }
}

// NOPQ (with CG): the q-free schedule; r = r - alpha q in place of q, with
// alpha = rr / pap from the CG state (0 when pap is not positive: the step
// kernel then stops the solve with a breakdown).
// ps scales the projected result (1 / n1 after vacuum-skipping y and z passes, else 1).
template <int N1, int N2, int PART, bool CG = false, bool BT = false, bool NOPQ = false>
__global__ __launch_bounds__(384) void k_fx_fwd_proj(Geom g, Tables t, const double2* __restrict__ fld,
                                                     double2* __restrict__ out, int R,
                                                     const int* skip, CgFuse cg,
                                                     const InstDesc* __restrict__ insts, double ps) {
  if constexpr (BT) {
    const InstDesc& d = insts[blockIdx.z];
    t = d.t;
    fld = d.fld;
    out = CG ? d.cg.q : d.vout;
    skip = d.skip;
    cg = d.cg;
  }
  if (skip && *skip) return;
  constexpr int N = N1 * N2;
  constexpr int NP = N;
  constexpr int D = Split<N1, N2>::D;
  constexpr int F = (PART == kPartBoth) ? 6 : 3;
  constexpr bool QF = CG && NOPQ;
  extern __shared__ double2 sm[];
  double2* twl = sm;
  double2* tile = sm + N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) twl[i] = t.tw[i];
  const long long rows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * R;
  const long long n = g.n;
  double qf_al = 0.0;
  if (QF) {
    const double pap = cg.st->pap;
    if (pap > 0.0 && isfinite(pap)) qf_al = cg.st->rr / pap;
  }
  const int n2 = threadIdx.x % N2;
  const int r = (threadIdx.x / N2) % R;
  const int c = threadIdx.x / (N2 * R);
  const bool active = c < F && row0 + r < rows;
  double2* T = tile + (c * R + r) * NP;
  double2 v[N1];
  if (active) {
    const double2* src = fld + c * n + (row0 + r) * N;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) v[n1] = src[n2 + N2 * n1];
  }
  __syncthreads();
  if (active) {
    step1<N1, N2, -1>(v, n2, twl);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) T[xpos<N1, N2, true>(n2 + N2 * k1, r)] = v[k1];
  }
  __syncthreads();
  double2 res[D][N2];
  if (active) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int k1 = n2 + d * N2;
      if (k1 < N1) {
#pragma unroll
        for (int m = 0; m < N2; ++m) res[d][m] = T[xpos<N1, N2, true>(m + N2 * k1, r)];
        reg_dft<N2, -1>(res[d]);
      }
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int k1 = n2 + d * N2;
      if (k1 < N1) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) T[xpos<N1, N2, true>(k1 + N1 * k2, r)] = res[d][k2];
      }
    }
  }
  __syncthreads();
  double acc[3] = {0.0, 0.0, 0.0};  // Re p^*q, |q|^2, Re r^*q (fused CG)
  // projection: this thread's frequencies e = threadIdx.x + it * blockDim.x
  constexpr int IT = (N1 + F - 1) / F;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * blockDim.x;
    if (e >= R * N) break;
    const int rr = e / N, i1 = e - rr * N;
    const long long row = row0 + rr;
    if (row >= rows) continue;
    const int i2 = (int)(row % g.n2), i3 = (int)(row / g.n2);
    const long long f = row * N + i1;
    double2 pv[4], rv[4];  // fused CG: loaded before the stores of q (which may alias them)
    if (CG) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (!NOPQ) pv[b] = cg.p[b * n + f];
        rv[b] = cg.r[b * n + f];
      }
    }
    Basis B;
    basis_at(t.lam, g, i1, i2, i3, B);
    double2 oa = make_double2(0, 0), ob = make_double2(0, 0);
    if (PART == kPartBoth || PART == kPartP) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const double2 o = tile[(cc * R + rr) * NP + xpos<N1, N2, true>(i1, rr)];
        oa = csub(oa, cmul(B.pi2[cc], o));
        ob = cadd(ob, cmul(B.pi1[cc], o));
      }
      oa = cscale(oa, ps);
      ob = cscale(ob, ps);
      if (!QF) {
        out[f] = oa;
        out[n + f] = ob;
      }
    }
    if (PART == kPartBoth || PART == kPartQ) {
      const long long o0 = (PART == kPartBoth) ? 2 * n : 0;
      const int cb = (PART == kPartBoth) ? 3 : 0;
      double2 oc = make_double2(0, 0), od = make_double2(0, 0);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const double2 o = tile[((cb + cc) * R + rr) * NP + xpos<N1, N2, true>(i1, rr)];
        oc = cadd(oc, cmulc(B.pi1[cc], o));
        od = cadd(od, cmulc(B.pi2[cc], o));
      }
      oc = cscale(oc, ps);
      od = cscale(od, ps);
      if (!QF) {
        out[o0 + f] = oc;
        out[o0 + n + f] = od;
      }
      if (QF) {
        const double2 qv[4] = {oa, ob, oc, od};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double2 rn = make_double2(rv[b].x - qf_al * qv[b].x, rv[b].y - qf_al * qv[b].y);
          st_stream(cg.r + b * n + f, rn);
          acc[0] += cabs2(rn);
        }
      } else if (CG) {
        const double2 qv[4] = {oa, ob, oc, od};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (!NOPQ) acc[0] += pv[b].x * qv[b].x + pv[b].y * qv[b].y;
          acc[1] += cabs2(qv[b]);
          acc[2] += rv[b].x * qv[b].x + rv[b].y * qv[b].y;
        }
      }
    }
  }
  if (QF) {
    double a1[1] = {acc[0]};
    block_sum_k<1>(a1);
    if (threadIdx.x == 0) cg.part_out[blockIdx.x] = a1[0];
  } else if (CG) {
    block_sum_k<3>(acc);
    if (threadIdx.x == 0) {
      cg.part_out[3 * blockIdx.x + 0] = acc[0];
      cg.part_out[3 * blockIdx.x + 1] = acc[1];
      cg.part_out[3 * blockIdx.x + 2] = acc[2];
    }
  }
}

// ------------------------------------------------------------- dispatch
struct FastCfg {
  int N1, N2;
};

bool fast_cfg(int N, FastCfg& c) {
  switch (N) {
    case 128: c = {16, 8}; return true;
    case 64: c = {8, 8}; return true;
    case 32: c = {8, 4}; return true;
    case 16: c = {4, 4}; return true;
    case 256: c = {16, 16}; return true;
    case 96: c = {16, 6}; return true;
    case 48: c = {16, 3}; return true;
    default: return false;
  }
}

#define NSF_FAST_SWITCH(N, MACRO) \
  switch (N) {                    \
    case 128: MACRO(16, 8); break; \
    case 64: MACRO(8, 8); break;   \
    case 32: MACRO(8, 4); break;   \
    case 16: MACRO(4, 4); break;   \
    case 256: MACRO(16, 16); break; \
    case 96: MACRO(16, 6); break;  \
    case 48: MACRO(16, 3); break;  \
    default: return hipErrorInvalidValue; \
  }

// Largest LDS allocation one workgroup may make on the current device.
size_t lds_limit() {
  static size_t cached = 0;
  if (!cached) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      cached = (size_t)v;
    else
      cached = 65536;
  }
  return cached;
}

int pick_cols(int n1, int want) {
  int P = 1;
  while (P * 2 <= want && n1 % (P * 2) == 0) P *= 2;
  return P;
}

// Rows per workgroup of an x pass over F fields: the plan's choice, halved
// until the workgroup fits 384 lanes and 64 KB of LDS; 0 if one row does not.
int x_rows_for(const Geom& g, const FastCfg& cfg, int F) {
  const int N = g.n1;
  int R = g.x_rows >= 4 ? 4 : (g.x_rows >= 2 ? 2 : 1);
  while (R > 1 && (F * R * cfg.N2 > 384 || (size_t)(N + F * R * N) * 16 > 64 * 1024)) R /= 2;
  return F * R * cfg.N2 > 384 ? 0 : R;
}

}  // namespace

bool fast_axis(int N) {
  FastCfg c;
  return fast_cfg(N, c);
}

int fast_yz_cols(const Geom& g, int axis) {
  FastCfg cfg;
  if (!fast_cfg(axis == 1 ? g.n2 : g.n3, cfg)) return 0;
  return pick_cols(g.n1, std::min(std::min(256 / cfg.N2, 16), std::max(g.yz_cols, 1)));
}

hipError_t launch_fast_yz(const Geom& g, const Tables& t, int axis, int dir, int nf, double2* fld,
                          int post_twist, int pre_twist, const int* skip, hipStream_t s,
                          const InstDesc* insts, int ninst, const int* xg, int nxg, double ysc) {
  const int N = axis == 1 ? g.n2 : g.n3;
  FastCfg cfg;
  if (!fast_cfg(N, cfg)) return hipErrorInvalidValue;
  const int P = fast_yz_cols(g, axis);
  const long long other = (axis == 1) ? g.n3 : g.n2;
  if (ysc > 0.0 && (axis != 1 || nxg < 0 || (!insts && !xg))) return hipErrorInvalidValue;
  if (ysc > 0.0 && nxg == 0) return hipSuccess;  // every x group is vacuum
  const long long groups = ysc > 0.0 ? nxg : g.n1 / P;
  const dim3 grid((unsigned)(groups * other), (unsigned)nf, (unsigned)ninst);
  const dim3 block(P * cfg.N2);
  const size_t lds = sizeof(double2) * (size_t)(N + yz_phases(cfg.N1, cfg.N2, dir).rows * cfg.N2 * P);
#define L_YZ(A, B)                                                                                   \
  if (insts && dir > 0)                                                                              \
    hipLaunchKernelGGL((k_fyz<A, B, +1, true>), grid, block, lds, s, g, t, axis, fld, P, post_twist, \
                       pre_twist, skip, insts, xg, nxg, ysc);                                       \
  else if (insts)                                                                                    \
    hipLaunchKernelGGL((k_fyz<A, B, -1, true>), grid, block, lds, s, g, t, axis, fld, P, post_twist, \
                       pre_twist, skip, insts, xg, nxg, ysc);                                       \
  else if (dir > 0)                                                                                  \
    hipLaunchKernelGGL((k_fyz<A, B, +1>), grid, block, lds, s, g, t, axis, fld, P, post_twist,       \
                       pre_twist, skip, insts, xg, nxg, ysc);                                       \
  else                                                                                               \
    hipLaunchKernelGGL((k_fyz<A, B, -1>), grid, block, lds, s, g, t, axis, fld, P, post_twist,       \
                       pre_twist, skip, insts, xg, nxg, ysc);
  NSF_FAST_SWITCH(N, L_YZ)
#undef L_YZ
  return hipGetLastError();
}

int fast_z_pair_cols(const Geom& g, int medium_kind, int P_want) {
  const int N = g.n3;
  FastCfg cfg;
  if (!fast_cfg(N, cfg) || !g.mid_pairs || six_coupled(medium_kind)) return 0;
  const size_t lmax = lds_limit() - 1024;  // room for the kernel's static LDS (reductions)
  int P = pick_cols(g.n1, P_want);
  while (P > 1 && (2 * P * cfg.N2 > 256 || (size_t)(N + 2 * N * P) * 16 > lmax)) P /= 2;
  if (2 * P * cfg.N2 > 256 || (size_t)(N + 2 * N * P) * 16 > lmax) return 0;
  return P;
}

int fast_z_mid_pq_items(const Geom& g, int medium_kind, int P_want) {
  const int P = fast_z_pair_cols(g, medium_kind, P_want);
  if (!P) return 0;
  const unsigned items = (unsigned)(3 * (g.n1 / P) * g.n2);
  return items <= 2u * kMidSlots ? (int)items : 0;
}

hipError_t launch_fast_z_mid(const Geom& g, const Tables& t, const MediumView& med, double2* fld,
                             int P_want, const int* skip, hipStream_t s, const InstDesc* insts,
                             int ninst, double* part_mid, int* np_mid, double vac_scale, int vac_tiles) {
  const int N = g.n3;
  if (np_mid) *np_mid = 0;
  FastCfg cfg;
  if (!fast_cfg(N, cfg)) return hipErrorInvalidValue;
  if (g.mid_pairs && !six_coupled(med.kind)) {  // general media couple all six fields
    const int P = fast_z_pair_cols(g, med.kind, P_want);
    if (!P) return hipErrorInvalidValue;
    const bool vac = vac_scale > 0.0;
    if (vac && vac_tiles < 0) return hipErrorInvalidValue;
    const unsigned items = (unsigned)(3 * (vac ? vac_tiles : (g.n1 / P) * g.n2));
    if (items == 0) return hipSuccess;  // every listed column is vacuum: nothing to do
    const dim3 block(2 * P * cfg.N2);
    const size_t lds = sizeof(double2) * (size_t)(N + 2 * N * P);
    const dim3 grid(items, 1, (unsigned)ninst);
    const bool pq = np_mid && (insts || part_mid) && items <= 2u * kMidSlots;
    if (pq) *np_mid = (int)items;
#define L_PAIR(A, B)                                                                                 \
  if (lds > 65536) { /* opt in once per kernel, to the device limit (not a stream operation) */     \
    const void* ks[4] = {reinterpret_cast<const void*>(&k_fz_pair<A, B, false, false>),              \
                         reinterpret_cast<const void*>(&k_fz_pair<A, B, true, false>),               \
                         reinterpret_cast<const void*>(&k_fz_pair<A, B, false, true>),               \
                         reinterpret_cast<const void*>(&k_fz_pair<A, B, true, true>)};              \
    static const hipError_t e0 = [&]() { /* dynamic LDS up to the limit less the static part */    \
      for (const void* k : ks) {                                                                     \
        hipFuncAttributes fa;                                                                        \
        hipError_t e = hipFuncGetAttributes(&fa, k);                                                 \
        if (e == hipSuccess)                                                                         \
          e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,                     \
                                  (int)(lds_limit() - fa.sharedSizeBytes));                          \
        if (e != hipSuccess) return e;                                                               \
      }                                                                                              \
      return hipSuccess;                                                                             \
    }();                                                                                             \
    if (e0 != hipSuccess) return e0;                                                                 \
  }                                                                                                  \
  if (insts && pq)                                                                                   \
    hipLaunchKernelGGL((k_fz_pair<A, B, true, true>), grid, block, lds, s, g, t, med, fld, P, skip,  \
                       insts, part_mid, vac_scale);                                                  \
  else if (insts)                                                                                    \
    hipLaunchKernelGGL((k_fz_pair<A, B, true>), grid, block, lds, s, g, t, med, fld, P, skip, insts, \
                       part_mid, vac_scale);                                                         \
  else if (pq)                                                                                       \
    hipLaunchKernelGGL((k_fz_pair<A, B, false, true>), grid, block, lds, s, g, t, med, fld, P, skip, \
                       insts, part_mid, vac_scale);                                                  \
  else                                                                                               \
    hipLaunchKernelGGL((k_fz_pair<A, B>), grid, block, lds, s, g, t, med, fld, P, skip, insts,       \
                       part_mid, vac_scale);
    NSF_FAST_SWITCH(N, L_PAIR)
#undef L_PAIR
    return hipGetLastError();
  }
  int P = pick_cols(g.n1, P_want);
  while (P > 1 && (6 * P * cfg.N2 > 384 || (size_t)(N + 6 * N * P) * 16 > lds_limit())) P /= 2;
  if (6 * P * cfg.N2 > 384) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.n1 / P) * g.n2), 1, (unsigned)ninst);
  const dim3 block(6 * P * cfg.N2);
  const size_t lds = sizeof(double2) * (size_t)(N + 6 * N * P);
  // Workgroups above 64 KiB of LDS opt in once per kernel.
#define L_MID(A, B)                                                                                 \
  if (lds > 65536) { /* opt in once per kernel, to the device limit (not a stream operation) */    \
    static const hipError_t e0 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fz_mid<A, B>), \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit()); \
    static const hipError_t e1 = hipFuncSetAttribute(                                               \
        reinterpret_cast<const void*>(&k_fz_mid<A, B, true>),                                       \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_limit());                              \
    if (e0 != hipSuccess) return e0;                                                                \
    if (e1 != hipSuccess) return e1;                                                                \
  }                                                                                                 \
  if (insts)                                                                                        \
    hipLaunchKernelGGL((k_fz_mid<A, B, true>), grid, block, lds, s, g, t, med, fld, P, skip, insts); \
  else                                                                                              \
    hipLaunchKernelGGL((k_fz_mid<A, B>), grid, block, lds, s, g, t, med, fld, P, skip, insts);
  NSF_FAST_SWITCH(N, L_MID)
#undef L_MID
  return hipGetLastError();
}

hipError_t launch_fast_x_inv_synth(const Geom& g, const Tables& t, int part, const double2* y, double2* fld,
                                   const int* skip, hipStream_t s, const InstDesc* insts, int ninst) {
  const int N = g.n1;
  FastCfg cfg;
  if (!fast_cfg(N, cfg)) return hipErrorInvalidValue;
  const int F = part == kPartBoth ? 6 : 3;
  const int R = x_rows_for(g, cfg, F);
  if (R == 0) return hipErrorInvalidValue;
  const long long rows = (long long)g.n2 * g.n3;
  const dim3 grid((unsigned)((rows + R - 1) / R), 1, (unsigned)ninst);
  const dim3 block(F * R * cfg.N2);
  const size_t lds = sizeof(double2) * (size_t)(N + F * R * N);
  if (insts && part != kPartBoth) return hipErrorInvalidValue;  // batched form covers both halves only
  const CgFuse none{};
#define L_XI(A, B)                                                                                    \
  if (part == kPartBoth && insts)                                                                     \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartBoth, false, true>), grid, block, lds, s, g, t, y,    \
                       fld, R, skip, none, insts);                                                    \
  else if (part == kPartBoth)                                                                         \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartBoth>), grid, block, lds, s, g, t, y, fld, R, skip,  \
                       none, insts);                                                                  \
  else if (part == kPartP)                                                                            \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartP>), grid, block, lds, s, g, t, y, fld, R, skip,     \
                       none, insts);                                                                  \
  else                                                                                                \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartQ>), grid, block, lds, s, g, t, y, fld, R, skip,     \
                       none, insts);
  NSF_FAST_SWITCH(N, L_XI)
#undef L_XI
  return hipGetLastError();
}

hipError_t launch_fast_x_fwd_proj(const Geom& g, const Tables& t, int part, const double2* fld, double2* out,
                                  const int* skip, hipStream_t s, const InstDesc* insts, int ninst, double pscale) {
  const int N = g.n1;
  FastCfg cfg;
  if (!fast_cfg(N, cfg)) return hipErrorInvalidValue;
  const int F = part == kPartBoth ? 6 : 3;
  const int R = x_rows_for(g, cfg, F);
  if (R == 0) return hipErrorInvalidValue;
  const long long rows = (long long)g.n2 * g.n3;
  const dim3 grid((unsigned)((rows + R - 1) / R), 1, (unsigned)ninst);
  const dim3 block(F * R * cfg.N2);
  const size_t lds = sizeof(double2) * (size_t)(N + F * R * N);
  if (insts && part != kPartBoth) return hipErrorInvalidValue;  // batched form covers both halves only
  const CgFuse none{};
#define L_XF(A, B)                                                                                     \
  if (part == kPartBoth && insts)                                                                      \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartBoth, false, true>), grid, block, lds, s, g, t, fld,    \
                       out, R, skip, none, insts, pscale);                                                     \
  else if (part == kPartBoth)                                                                          \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartBoth>), grid, block, lds, s, g, t, fld, out, R, skip,  \
                       none, insts, pscale);                                                                   \
  else if (part == kPartP)                                                                             \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartP>), grid, block, lds, s, g, t, fld, out, R, skip,     \
                       none, insts, pscale);                                                                   \
  else                                                                                                 \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartQ>), grid, block, lds, s, g, t, fld, out, R, skip,     \
                       none, insts, pscale);
  NSF_FAST_SWITCH(N, L_XF)
#undef L_XF
  return hipGetLastError();
}

// Rows per workgroup of the six-field x passes (0: no two-level pass).
int fast_x_rows(const Geom& g) {
  FastCfg cfg;
  if (!fast_cfg(g.n1, cfg)) return 0;
  return x_rows_for(g, cfg, 6);
}

hipError_t launch_fast_cg_first(const Geom& g, const Tables& t, const CgFuse& cg, double2* fld,
                                const int* skip, int* nparts, hipStream_t s, const InstDesc* insts,
                                int ninst, bool qfree) {
  const int N = g.n1;
  FastCfg cfg;
  if (!fast_cfg(N, cfg)) return hipErrorInvalidValue;
  const int R = x_rows_for(g, cfg, 6);
  if (R == 0) return hipErrorInvalidValue;
  const long long rows = (long long)g.n2 * g.n3;
  const dim3 grid((unsigned)((rows + R - 1) / R), 1, (unsigned)ninst);
  *nparts = (int)grid.x;
  const dim3 block(6 * R * cfg.N2);
  const size_t lds = sizeof(double2) * (size_t)(N + 6 * R * N);
#define L_CGI(A, B)                                                                                  \
  if (insts && qfree)                                                                                \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartBoth, true, true, true, true>), grid, block, lds, s, \
                       g, t, (const double2*)nullptr, fld, R, skip, cg, insts);                      \
  else if (insts)                                                                                    \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartBoth, true, true>), grid, block, lds, s, g, t,     \
                       (const double2*)nullptr, fld, R, skip, cg, insts);                            \
  else if (qfree)                                                                                    \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartBoth, true, false, true, true>), grid, block, lds, s, \
                       g, t, (const double2*)nullptr, fld, R, skip, cg, insts);                      \
  else                                                                                               \
    hipLaunchKernelGGL((k_fx_inv_synth<A, B, kPartBoth, true>), grid, block, lds, s, g, t,           \
                       (const double2*)nullptr, fld, R, skip, cg, insts);
  NSF_FAST_SWITCH(N, L_CGI)
#undef L_CGI
  return hipGetLastError();
}

hipError_t launch_fast_cg_last(const Geom& g, const Tables& t, const CgFuse& cg, const double2* fld,
                               const int* skip, int* nparts, hipStream_t s, const InstDesc* insts,
                               int ninst, bool pq_done, double pscale) {
  const int N = g.n1;
  FastCfg cfg;
  if (!fast_cfg(N, cfg)) return hipErrorInvalidValue;
  const int R = x_rows_for(g, cfg, 6);
  if (R == 0) return hipErrorInvalidValue;
  const long long rows = (long long)g.n2 * g.n3;
  const dim3 grid((unsigned)((rows + R - 1) / R), 1, (unsigned)ninst);
  *nparts = (int)grid.x;
  const dim3 block(6 * R * cfg.N2);
  const size_t lds = sizeof(double2) * (size_t)(N + 6 * R * N);
#define L_CGL(A, B)                                                                                  \
  if (insts && pq_done)                                                                              \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartBoth, true, true, true>), grid, block, lds, s, g, t,  \
                       fld, cg.q, R, skip, cg, insts, pscale);                                               \
  else if (insts)                                                                                    \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartBoth, true, true>), grid, block, lds, s, g, t, fld,  \
                       cg.q, R, skip, cg, insts, pscale);                                                    \
  else if (pq_done)                                                                                  \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartBoth, true, false, true>), grid, block, lds, s, g, t, \
                       fld, cg.q, R, skip, cg, insts, pscale);                                               \
  else                                                                                               \
    hipLaunchKernelGGL((k_fx_fwd_proj<A, B, kPartBoth, true>), grid, block, lds, s, g, t, fld, cg.q, \
                       R, skip, cg, insts, pscale);
  NSF_FAST_SWITCH(N, L_CGL)
#undef L_CGL
  return hipGetLastError();
}

}  // namespace nsf
