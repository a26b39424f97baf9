// Device helpers shared by the FFT pass kernels: small register DFTs, the
// per-frequency singular-vector blocks of C and the per-voxel middle factor.
#pragma once

#include "nsf_internal.h"

namespace nsf {

// ----------------------------------------------------------- small DFTs
template <int S>
__device__ inline double2 mul_si(double2 a) {  // (S i) * a
  return S > 0 ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

template <int S>
__device__ inline void dft2(double2* v) {
  const double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int S>
__device__ inline void dft4(double2* v) {
  const double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const double2 t2 = cadd(v[1], v[3]), t3 = mul_si<S>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <int S>
__device__ inline void dft8(double2* v) {
  double2 e[4] = {v[0], v[2], v[4], v[6]};
  double2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<S>(e);
  dft4<S>(o);
  constexpr double h = 0.70710678118654752440;
  const double2 o1 = cmul(o[1], make_double2(h, S * h));
  const double2 o2 = mul_si<S>(o[2]);
  const double2 o3 = cmul(o[3], make_double2(-h, S * h));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <int S>
__device__ inline void dft3(double2* v) {
  constexpr double c = 0.86602540378443864676;  // sin(2 pi / 3)
  const double2 t = cadd(v[1], v[2]);
  const double2 m = csub(v[0], cscale(t, 0.5));
  const double2 d = mul_si<S>(cscale(csub(v[1], v[2]), c));
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, d);
  v[2] = csub(m, d);
}

template <int S>
__device__ inline void dft5(double2* v) {
  constexpr double c1 = 0.30901699437494742410;   // cos(2 pi / 5)
  constexpr double c2 = -0.80901699437494742410;  // cos(4 pi / 5)
  constexpr double s1 = 0.95105651629515357212;   // sin(2 pi / 5)
  constexpr double s2 = 0.58778525229247312917;   // sin(4 pi / 5)
  const double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const double2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  const double2 m1 = cadd(v[0], cadd(cscale(t1, c1), cscale(t2, c2)));
  const double2 m2 = cadd(v[0], cadd(cscale(t1, c2), cscale(t2, c1)));
  const double2 n1 = mul_si<S>(cadd(cscale(t3, s1), cscale(t4, s2)));
  const double2 n2 = mul_si<S>(csub(cscale(t3, s2), cscale(t4, s1)));
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(m1, n1);
  v[4] = csub(m1, n1);
  v[2] = cadd(m2, n2);
  v[3] = csub(m2, n2);
}

template <int R, int S>
__device__ inline void dft(double2* v) {
  if constexpr (R == 2) dft2<S>(v);
  else if constexpr (R == 3) dft3<S>(v);
  else if constexpr (R == 4) dft4<S>(v);
  else if constexpr (R == 5) dft5<S>(v);
  else dft8<S>(v);
}


// dft6 = 3 x 2 split: X[k1 + 3 k2] = sum_{n2<2} W6^{n2 k1} [sum_{n1<3} x[n2 + 2 n1] W3^{n1 k1}] W2^{n2 k2}
template <int S>
__device__ inline void dft6(double2* v) {
  double2 a[3] = {v[0], v[2], v[4]};
  double2 b[3] = {v[1], v[3], v[5]};
  dft3<S>(a);
  dft3<S>(b);
  constexpr double c = 0.86602540378443864676;  // sin(pi/3)
  b[1] = cmul(b[1], make_double2(0.5, S * c));   // W6^1
  b[2] = cmul(b[2], make_double2(-0.5, S * c));  // W6^2
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    const double2 x0 = a[k1], x1 = b[k1];
    v[k1] = cadd(x0, x1);
    v[k1 + 3] = csub(x0, x1);
  }
}

// cos and sin of 2 pi j / 16, j = 0..15
__device__ constexpr double kC16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kS16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// dft16 = 4 x 4 split with the twiddles W16^{n2 k1} as constants.
template <int S>
__device__ inline void dft16(double2* v) {
  double2 a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[n2 + 4 * n1];
    dft4<S>(a[n2]);
  }
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      const int j = n2 * k1;
      a[n2][k1] = cmul(a[n2][k1], make_double2(kC16[j], S * kS16[j]));
    }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    double2 u[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4<S>(u);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = u[k2];
  }
}

template <int N, int S>
__device__ inline void reg_dft(double2* v) {
  if constexpr (N == 1) return;
  else if constexpr (N == 2) dft2<S>(v);
  else if constexpr (N == 3) dft3<S>(v);
  else if constexpr (N == 4) dft4<S>(v);
  else if constexpr (N == 5) dft5<S>(v);
  else if constexpr (N == 6) dft6<S>(v);
  else if constexpr (N == 8) dft8<S>(v);
  else if constexpr (N == 16) dft16<S>(v);
  else static_assert(N == 16, "unsupported register DFT size");
}

// ---------------------------------------------------------------- basis
// Per-frequency singular-vector blocks (Thm 2.5): with lambda = (l1,l2,l3),
// p = a x lambda (a column of Lambda_p, Lemma 2.2), sigma = ||lambda||:
//   pi2 = conj(p)/||p||,  pi1 = (conj(lambda) x p)/(sigma ||p||),
// the unit-norm columns of Pi_2 and Pi_1 (Pi_1 is the projection of
// (alpha, beta, 1) off lambda/sigma, normalised).
struct Basis {
  double2 pi1[3], pi2[3];
};

// Sum of up to four doubles over a workgroup of at most 1024 threads; the
// result is valid in thread 0.  Fixed order: wave butterflies, then waves in
// index order.
template <int K>
__device__ __forceinline__ void block_sum_k(double (&v)[K]) {
  __shared__ double red[16][K];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = 0;
      for (int w = 0; w < nw; ++w) a += red[w][k];
      v[k] = a;
    }
  }
}

// Loads and stores at a workgroup-uniform base plus a 32-bit lane offset (in
// elements), so the compiler can use SGPR-base addressing instead of holding
// a 64-bit address per load in VGPRs.  Offsets times 16 must stay below 2^32.
__device__ __forceinline__ double2 ld_off(const double2* __restrict__ base, unsigned off) {
  return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(base) + (off << 4));
}
__device__ __forceinline__ void st_off(double2* __restrict__ base, unsigned off, double2 v) {
  *reinterpret_cast<double2*>(reinterpret_cast<char*>(base) + (off << 4)) = v;
}

// Nontemporal store, for the CG vectors x, p, r: each is read back only in the
// next CG iteration, after gigabytes of other traffic, so keeping it in the
// caches gains nothing.  (The fields between passes keep plain stores: the
// next pass finds part of them in the Infinity Cache.)
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  const v2d t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<v2d*>(p));
}

// 1 / sqrt(x) for positive normal x: the hardware estimate (v_rsq_f64) refined by
// two Newton-Raphson steps y <- y (3 - x y^2) / 2, each of which roughly doubles
// the number of correct bits (to within an ulp or two in double precision).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

__device__ __forceinline__ void basis_at(const double2* __restrict__ lam, const Geom& g, int i1, int i2,
                                int i3, Basis& B) {
  const double2 l1 = lam[i1], l2 = lam[g.n1 + i2], l3 = lam[g.n1 + g.n2 + i3];
  const double al = g.alpha, be = g.beta;
  // p = (beta l3 - l2, l1 - alpha l3, alpha l2 - beta l1)
  const double2 p1 = csub(cscale(l3, be), l2);
  const double2 p2 = csub(l1, cscale(l3, al));
  const double2 p3 = csub(cscale(l2, al), cscale(l1, be));
  const double pn2 = cabs2(p1) + cabs2(p2) + cabs2(p3);
  const double s2 = cabs2(l1) + cabs2(l2) + cabs2(l3);
  const double ip = rsqrt_nr(pn2);
  const double iq = ip * rsqrt_nr(s2);
  B.pi2[0] = cscale(cconj(p1), ip);
  B.pi2[1] = cscale(cconj(p2), ip);
  B.pi2[2] = cscale(cconj(p3), ip);
  // conj(l) x p
  const double2 q1 = csub(cmulc(l2, p3), cmulc(l3, p2));
  const double2 q2 = csub(cmulc(l3, p1), cmulc(l1, p3));
  const double2 q3 = csub(cmulc(l1, p2), cmulc(l2, p1));
  B.pi1[0] = cscale(q1, iq);
  B.pi1[1] = cscale(q2, iq);
  B.pi1[2] = cscale(q3, iq);
}

__device__ inline double2 twist_at(const double2* __restrict__ tws, const Geom& g, int i1, int i2,
                                   int i3) {
  return cmul(cmul(tws[i1], tws[g.n1 + i2]), tws[g.n1 + g.n2 + i3]);
}


// ---------------------------------------------------- z pass with medium
// Per voxel, with E', H' the untwisted inverse transforms (times n) and the
// 1/n normalisation folded in, the middle factor of A_r (Thm 4.2) maps
//   o2 = Phi^{-1} (xi E' + H'),  o1 = zeta o2 + E'   (mu = 1).
// Chiral (xi = i gamma, zeta = -i gamma, Phi = eps - gamma^2):
//   o1 = (eps E' - i gamma H')/Phi,  o2 = (i gamma E' + H')/Phi.
// Pseudochiral on axes (a, b): xi = i gamma (e_a e_b^T + e_b e_a^T),
//   Phi = eps - gamma^2 on a and b, eps on the third axis o.
// Pseudochiral coupling of axes (A, B), third axis O (compile-time indices
// keep the six components in registers).
template <int A, int B>
__device__ __forceinline__ void pseudo_apply(double eps, double gam, double inv_n, double2* E, double2* H) {
  constexpr int O = 3 - A - B;
  const double ip = inv_n / (eps - gam * gam);
  const double2 o2a = cscale(cadd(cmuli(cscale(E[B], gam)), H[A]), ip);
  const double2 o2b = cscale(cadd(cmuli(cscale(E[A], gam)), H[B]), ip);
  const double2 o1a = csub(cscale(E[A], inv_n), cmuli(cscale(o2b, gam)));
  const double2 o1b = csub(cscale(E[B], inv_n), cmuli(cscale(o2a, gam)));
  H[O] = cscale(H[O], inv_n / eps);
  E[O] = cscale(E[O], inv_n);
  H[A] = o2a;
  H[B] = o2b;
  E[A] = o1a;
  E[B] = o1b;
}

__device__ __forceinline__ void medium_apply(const MediumView& m, double2 eg, double inv_n, double2* E,
                                             double2* H) {
  const double eps = eg.x, gam = eg.y;
  if (m.kind == kMedChiral) {
    const double ip = inv_n / (eps - gam * gam);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 e = E[c], h = H[c];
      const double2 ige = cmuli(cscale(e, gam));
      const double2 igh = cmuli(cscale(h, gam));
      E[c] = cscale(csub(cscale(e, eps), igh), ip);
      H[c] = cscale(cadd(ige, h), ip);
    }
  } else if (m.pa == 0 && m.pb == 1) {
    pseudo_apply<0, 1>(eps, gam, inv_n, E, H);
  } else if (m.pa == 0) {
    pseudo_apply<0, 2>(eps, gam, inv_n, E, H);
  } else {
    pseudo_apply<1, 2>(eps, gam, inv_n, E, H);
  }
}

// General (HHPD) media: [E; H] <- M [E; H] / n with M the voxel's 6 x 6
// Hermitian middle factor [[mu^-1 zeta Phi^-1 xi mu^-1 + mu^-1, mu^-1 zeta Phi^-1],
// [Phi^-1 xi mu^-1, Phi^-1]] (Thm 4.2), stored as its upper triangle.
__device__ __forceinline__ void general_apply(const double2* __restrict__ Mu, double inv_n, double2* E,
                                              double2* H) {
  double2 v[6] = {E[0], E[1], E[2], H[0], H[1], H[2]};
  double2 o[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) o[i] = make_double2(0, 0);
  int k = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = i; j < 6; ++j, ++k) {
      const double2 m = Mu[k];
      o[i] = cadd(o[i], cmul(m, v[j]));
      if (j != i) o[j] = cadd(o[j], cmulc(m, v[i]));  // M_ji = conj(M_ij)
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    E[c] = cscale(o[c], inv_n);
    H[c] = cscale(o[3 + c], inv_n);
  }
}

// NFSEP media: [E; H] <- N [E; H] / n with N = i J B^{-1} the voxel's full 6 x 6
// factor, J = [[0, I], [-I, 0]] (Thm 3.2; N is the Hermitian middle factor of
// A_r when the medium meets the assumption of Sec. 4.1), row-major.
__device__ __forceinline__ void full_apply(const double2* __restrict__ N, double inv_n, double2* E,
                                           double2* H) {
  const double2 v[6] = {E[0], E[1], E[2], H[0], H[1], H[2]};
  double2 o[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double2 acc = make_double2(0, 0);
#pragma unroll
    for (int j = 0; j < 6; ++j) acc = cadd(acc, cmul(N[6 * i + j], v[j]));
    o[i] = cscale(acc, inv_n);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    E[c] = o[c];
    H[c] = o[3 + c];
  }
}

// The constitutive step of voxel gi for any medium kind.
__device__ __forceinline__ void medium_apply_at(const MediumView& m, long long gi, double inv_n, double2* E,
                                                double2* H) {
  const long long slot = m.pidx ? (long long)m.pidx[gi] : gi;
  if (m.kind == kMedGeneral)
    general_apply(m.mg + slot * kGenEntries, inv_n, E, H);
  else if (m.kind == kMedNfsep)
    full_apply(m.mf + slot * kFullEntries, inv_n, E, H);
  else
    medium_apply(m, m.eg[gi], inv_n, E, H);
}

}  // namespace nsf
