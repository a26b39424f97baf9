// Vector kernels: fixed-order reductions, the CG recurrences (Sec. 4.2) and
// the multi-vector products of the Lanczos basis.
//
// Reductions are deterministic: every launch uses the same grid, every thread
// sums a fixed strided slice, waves reduce with butterfly shuffles and a
// single workgroup folds the per-workgroup partials in a fixed order.  No
// floating-point atomics are used.
#include <algorithm>

#include "nsf_internal.h"

namespace nsf {
namespace {

constexpr int kRedThreads = 256;

__device__ inline double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Sum over the workgroup; the result is valid in thread 0.
__device__ inline double2 block_sum(double2 v) {
  __shared__ double2 red[kRedThreads / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double2 s = make_double2(0, 0);
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = cadd(s, red[i]);
  }
  __syncthreads();
  return s;
}

// Four independent accumulators per thread, so four loads are in flight at once
// (the fold is latency-bound otherwise); fixed order, hence reproducible.
__device__ inline double2 fold_partials(const double2* partial, int nparts) {
  double2 v0 = make_double2(0, 0), v1 = v0, v2 = v0, v3 = v0;
  const int bd = blockDim.x;
  int i = threadIdx.x;
  for (; i + 3 * bd < nparts; i += 4 * bd) {
    v0 = cadd(v0, partial[i]);
    v1 = cadd(v1, partial[i + bd]);
    v2 = cadd(v2, partial[i + 2 * bd]);
    v3 = cadd(v3, partial[i + 3 * bd]);
  }
  for (; i < nparts; i += bd) v0 = cadd(v0, partial[i]);
  return block_sum(cadd(cadd(v0, v1), cadd(v2, v3)));
}

// sum of part[0..n) (strided by `stride` doubles from `part`), four accumulators per thread
__device__ inline double fold_doubles(const double* part, int n, int stride) {
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  const int bd = blockDim.x;
  int i = threadIdx.x;
  for (; i + 3 * bd < n; i += 4 * bd) {
    a0 += part[(long long)i * stride];
    a1 += part[(long long)(i + bd) * stride];
    a2 += part[(long long)(i + 2 * bd) * stride];
    a3 += part[(long long)(i + 3 * bd) * stride];
  }
  for (; i < n; i += bd) a0 += part[(long long)i * stride];
  return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(kRedThreads) void k_dot(const double2* __restrict__ x,
                                                     const double2* __restrict__ y, long long len,
                                                     double2* partial, const int* skip) {
  if (skip && *skip) return;
  double2 acc = make_double2(0, 0);
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < len;
       i += (long long)gridDim.x * kRedThreads)
    acc = cadd(acc, cmulc(x[i], y[i]));
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const double2* partial, int nparts,
                                                        double2* out) {
  const double2 s = fold_partials(partial, nparts);
  if (threadIdx.x == 0) out[0] = s;
}

// ------------------------------------------------------------------ CG
// x = 0, r = p = b - sum_j c_j AV_{idx_j} (the residual of the start
// x0 = sum_j c_j V_{idx_j} when AV_i = A V_i; no sum when m = 0); partials of
// (|b|^2, |r|^2).  c holds m coefficients followed by the m indices (in .x).
__global__ __launch_bounds__(kRedThreads) void k_cg_init(const double2* __restrict__ b,
                                                         double2* __restrict__ x,
                                                         double2* __restrict__ r,
                                                         double2* __restrict__ p, long long len,
                                                         double2* partial,
                                                         const double2* __restrict__ AV, long long ld,
                                                         int m, const double2* __restrict__ c) {
  __shared__ double2 cs[512];
  __shared__ int ix[512];
  for (int i = threadIdx.x; i < m; i += kRedThreads) {
    cs[i] = c[i];
    ix[i] = (int)c[m + i].x;
  }
  __syncthreads();
  double2 acc = make_double2(0, 0);
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < len;
       i += (long long)gridDim.x * kRedThreads) {
    const double2 v = b[i];
    double2 rv = v;
#pragma unroll 4
    for (int j = 0; j < m; ++j) rv = csub(rv, cmul(cs[j], AV[ix[j] * ld + i]));
    x[i] = make_double2(0, 0);
    r[i] = rv;
    p[i] = rv;
    acc.x += cabs2(v);
    acc.y += cabs2(rv);
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kRedThreads) void k_cg_init_final(const double2* partial, int nparts,
                                                               CgState* st, double rtol,
                                                               int maxit, int ring) {
  const double2 s = fold_partials(partial, nparts);
  if (threadIdx.x == 0) {
    const double bb = s.x;
    st->ring = ring;
    st->bd_step = 0;
    st->bb = bb;
    st->rr = s.y;
    st->thresh = rtol * rtol * bb;
    st->alpha = 0;
    st->beta = 0;
    st->iter = 0;
    st->maxit = maxit;
    st->status = NSF_OK;
    st->done = 0;
    if (!(bb > 0.0) || !(s.y == s.y)) {
      st->done = 1;
      st->status = (bb == 0.0) ? NSF_OK : NSF_E_BREAKDOWN;  // zero rhs, or NaN
    } else if (s.y <= st->thresh) {
      st->done = 1;  // the start already solves the system to the tolerance
    } else if (maxit <= 0) {
      st->done = 1;
      st->status = NSF_NOT_CONVERGED;
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_alpha(const double2* partial, int nparts,
                                                          CgState* st) {
  if (st->done) return;
  const double2 s = fold_partials(partial, nparts);
  if (threadIdx.x == 0) {
    const double pq = s.x;  // p^* A_r p is real for Hermitian A_r
    if (!(pq > 0.0) || !isfinite(pq)) {
      st->status = NSF_E_BREAKDOWN;
      st->done = 1;
    } else {
      st->alpha = st->rr / pq;
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_update(double2* __restrict__ x,
                                                           double2* __restrict__ r,
                                                           const double2* __restrict__ p,
                                                           const double2* __restrict__ q,
                                                           long long len, double2* partial,
                                                           const CgState* st) {
  if (st->done) return;
  const double al = st->alpha;
  double2 acc = make_double2(0, 0);
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < len;
       i += (long long)gridDim.x * kRedThreads) {
    const double2 pi = p[i], qi = q[i];
    double2 xi = x[i], ri = r[i];
    xi = make_double2(xi.x + al * pi.x, xi.y + al * pi.y);
    ri = make_double2(ri.x - al * qi.x, ri.y - al * qi.y);
    x[i] = xi;
    r[i] = ri;
    acc.x += cabs2(ri);
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kRedThreads) void k_cg_beta(const double2* partial, int nparts,
                                                         CgState* st) {
  if (st->done) return;
  const double2 s = fold_partials(partial, nparts);
  if (threadIdx.x == 0) {
    const double rr_new = s.x;
    st->iter += 1;
    st->beta = rr_new / st->rr;
    st->rr = rr_new;
    if (!isfinite(rr_new)) {
      st->status = NSF_E_BREAKDOWN;
      st->done = 1;
    } else if (rr_new <= st->thresh) {
      st->status = NSF_OK;
      st->done = 1;
    } else if (st->iter >= st->maxit) {
      st->status = NSF_NOT_CONVERGED;
      st->done = 1;
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_cg_p(double2* __restrict__ p,
                                                      const double2* __restrict__ r, long long len,
                                                      const CgState* st) {
  if (st->done) return;
  const double be = st->beta;
  for (long long i = blockIdx.x * (long long)kRedThreads + threadIdx.x; i < len;
       i += (long long)gridDim.x * kRedThreads) {
    const double2 pi = p[i], ri = r[i];
    p[i] = make_double2(ri.x + be * pi.x, ri.y + be * pi.y);
  }
}

// ----------------------------------------------------- fused CG scalars
// After the first pass of round k (k > 0) the workgroups have written
// |r_k|^2 partials: decide convergence on the recurrence residual r_k.
__global__ __launch_bounds__(kRedThreads) void k_cgf_check(const double* part, int nparts, CgState* st,
                                                           const InstDesc* insts) {
  if (insts) {
    part = insts[blockIdx.x].cg.part_in;
    st = insts[blockIdx.x].cg.st;
  }
  if (st->done || st->iter == 0) return;
  double2 v = make_double2(fold_doubles(part, nparts, 1), 0);
  v = block_sum(v);
  if (threadIdx.x == 0) {
    const double rr = v.x;
    st->rr = rr;
    if (!isfinite(rr)) {
      st->status = NSF_E_BREAKDOWN;
      st->done = 1;
    } else if (rr <= st->thresh) {
      st->status = NSF_OK;
      st->done = 1;
    } else if (st->iter >= st->maxit) {
      st->status = NSF_NOT_CONVERGED;
      st->done = 1;
    }
  }
}

// After the last pass: alpha = |r|^2 / p^*A p and beta = |r - alpha q|^2 / |r|^2,
// the new residual norm expanded as |r|^2 - 2 alpha Re r^*q + alpha^2 |q|^2.
// With np_mid > 0, p^*A p comes from the fused z pass's partials instead.
__global__ __launch_bounds__(kRedThreads) void k_cgf_step(const double* part, int nparts, CgState* st,
                                                          const InstDesc* insts, const double* part_mid,
                                                          int np_mid) {
  if (insts) {
    part = insts[blockIdx.x].cg.part_out;
    st = insts[blockIdx.x].cg.st;
    part_mid = insts[blockIdx.x].cg.part_mid;
  }
  if (st->done) return;
  double2 a, b;
  a.x = np_mid > 0 ? fold_doubles(part_mid, np_mid, 1) : fold_doubles(part, nparts, 3);
  a.y = fold_doubles(part + 1, nparts, 3);
  b = make_double2(fold_doubles(part + 2, nparts, 3), 0);
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    const double pq = a.x, qq = a.y, rq = b.x, rr = st->rr;
    if (!(pq > 0.0) || !isfinite(pq)) {
      st->status = NSF_E_BREAKDOWN;
      st->done = 1;
      return;
    }
    const double al = rr / pq;
    double rn = rr - 2.0 * al * rq + al * al * qq;
    if (rn < 0.0) rn = 0.0;
    st->alpha = al;
    st->beta = rn / rr;
    st->iter += 1;
  }
}

// q-free schedule, after the fused z pass: st->pap = sum of its partials.
// With np_in > 0 (vacuum skipping) the z pass summed Re f^* (M - I) f / n only
// and the first pass's |p|^2 partials complete p^* A_r p.
__global__ __launch_bounds__(kRedThreads) void k_cgf_alpha(const double* part_mid, int np_mid, CgState* st,
                                                           const InstDesc* insts, const double* part_in,
                                                           int np_in) {
  if (insts) {
    part_mid = insts[blockIdx.x].cg.part_mid;
    st = insts[blockIdx.x].cg.st;
    part_in = insts[blockIdx.x].cg.part_in;
  }
  if (st->done) return;
  double2 a = make_double2(fold_doubles(part_mid, np_mid, 1) + (np_in > 0 ? fold_doubles(part_in, np_in, 1) : 0.0),
                           0);
  a = block_sum(a);
  if (threadIdx.x == 0) st->pap = a.x;
}

// q-free schedule, after the last pass (which set r = r - alpha q): the new
// |r|^2, alpha and beta of this iteration, and the convergence test.
__global__ __launch_bounds__(kRedThreads) void k_cgf_step_qf(const double* part, int nparts, CgState* st,
                                                             const InstDesc* insts) {
  if (insts) {
    part = insts[blockIdx.x].cg.part_out;
    st = insts[blockIdx.x].cg.st;
  }
  if (st->done) return;
  double2 v = make_double2(fold_doubles(part, nparts, 1), 0);
  v = block_sum(v);
  if (threadIdx.x == 0) {
    const double pap = st->pap, rr = st->rr, rn = v.x;
    if (!(pap > 0.0) || !isfinite(pap)) {  // the last pass left r unchanged
      if (st->ring > 0) st->ahist[st->iter % st->ring] = 0.0;  // its p is not folded in
      st->bd_step = 1;
      st->status = NSF_E_BREAKDOWN;
      st->done = 1;
      return;
    }
    st->alpha = rr / pap;
    if (st->ring > 0) st->ahist[st->iter % st->ring] = st->alpha;
    st->beta = rn / rr;
    st->rr = rn;
    st->iter += 1;
    if (!isfinite(rn)) {
      st->status = NSF_E_BREAKDOWN;
      st->done = 1;
    } else if (rn <= st->thresh) {
      st->status = NSF_OK;
      st->done = 1;
    } else if (st->iter >= st->maxit) {
      st->status = NSF_NOT_CONVERGED;
      st->done = 1;
    }
  }
}

// x = x + alpha p: the update the q-free schedule leaves for the next first
// pass, applied once when the solve has ended (not after a breakdown).
__global__ void k_cg_finish(double2* __restrict__ x, const double2* __restrict__ p, long long len,
                            const CgState* st) {
  if (st->status == NSF_E_BREAKDOWN || st->iter == 0) return;
  const double al = st->alpha;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x) {
    const double2 pv = p[i];
    const double2 xv = x[i];
    x[i] = make_double2(xv.x + al * pv.x, xv.y + al * pv.y);
  }
}

// Kept directions of the q-free CG: x += sum_j alpha_j p_j over ring slots
// [0, cnt).  final = false runs inside iteration k = st->iter, after its alpha
// is known (rr / pap), and folds the whole ring when k + 1 fills it; final =
// true runs once after the solve and folds the slots written since the last
// fold (an iteration that broke down has alpha 0 in the history).
__global__ __launch_bounds__(256) void k_cg_fold(double2* __restrict__ x, const double2* __restrict__ ring,
                                                 long long len, const CgState* st, int final,
                                                 const InstDesc* __restrict__ insts) {
  if (insts) {
    const CgFuse& cg = insts[blockIdx.z].cg;
    x = cg.x;
    ring = cg.ring;
    st = cg.st;
  }
  const int K = st->ring;
  if (K <= 0) return;
  double a[kCgRing];
  int cnt;
  if (!final) {
    if (st->done) return;
    const int k = st->iter;
    if ((k + 1) % K != 0) return;
    const double pap = st->pap;
    const double ak = (pap > 0.0 && isfinite(pap)) ? st->rr / pap : 0.0;  // this iteration's alpha
#pragma unroll
    for (int j = 0; j < kCgRing; ++j) a[j] = j < K - 1 ? st->ahist[j] : (j == K - 1 ? ak : 0.0);
    cnt = K;
  } else {
    const int nit = st->iter + (st->status == NSF_E_BREAKDOWN ? st->bd_step : 0);
    cnt = nit % K;
    if (cnt == 0) return;
#pragma unroll
    for (int j = 0; j < kCgRing; ++j) a[j] = j < cnt ? st->ahist[j] : 0.0;
  }
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x) {
    double2 acc = x[i];
#pragma unroll
    for (int j = 0; j < kCgRing; ++j) {
      if (j < cnt) {
        const double2 pv = ring[(long long)j * len + i];
        acc.x += a[j] * pv.x;
        acc.y += a[j] * pv.y;
      }
    }
    x[i] = acc;
  }
}

// ------------------------------------------------------- multi-vector ops
// Partial sums of V[i]^* w for the kDotChunk basis vectors of one workgroup
// row: each element of w is read once per chunk, and the loads of one element
// for every vector of the chunk are issued together.
constexpr int kDotChunk = 4;

__global__ __launch_bounds__(kRedThreads) void k_multi_dot(const double2* __restrict__ V,
                                                           long long ld, int m,
                                                           const double2* __restrict__ w,
                                                           long long len, double2* partial) {
  const int i0 = blockIdx.y * kDotChunk;
  const int cnt = min(kDotChunk, m - i0);
  double2 acc[kDotChunk];
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) acc[c] = make_double2(0, 0);
  const double2* Vc = V + (long long)i0 * ld;
  for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < len;
       e += (long long)gridDim.x * kRedThreads) {
    const double2 we = w[e];
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c)
      if (c < cnt) acc[c] = cadd(acc[c], cmulc(Vc[c * ld + e], we));
  }
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) {
    const double2 s = block_sum(acc[c]);
    if (threadIdx.x == 0 && c < cnt) partial[(long long)(i0 + c) * gridDim.x + blockIdx.x] = s;
  }
}

// The same for two right-hand sides: partials of V[i]^* w1 (rows 0..m) and
// V[i]^* w2 (rows m..2m), each basis element read once for both.
__global__ __launch_bounds__(kRedThreads) void k_multi_dot2(const double2* __restrict__ V, long long ld,
                                                            int m, const double2* __restrict__ w1,
                                                            const double2* __restrict__ w2, long long len,
                                                            double2* partial) {
  const int i0 = blockIdx.y * kDotChunk;
  const int cnt = min(kDotChunk, m - i0);
  double2 a1[kDotChunk], a2[kDotChunk];
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) a1[c] = a2[c] = make_double2(0, 0);
  const double2* Vc = V + (long long)i0 * ld;
  for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < len;
       e += (long long)gridDim.x * kRedThreads) {
    const double2 x1 = w1[e], x2 = w2[e];
#pragma unroll
    for (int c = 0; c < kDotChunk; ++c)
      if (c < cnt) {
        const double2 v = Vc[c * ld + e];
        a1[c] = cadd(a1[c], cmulc(v, x1));
        a2[c] = cadd(a2[c], cmulc(v, x2));
      }
  }
#pragma unroll
  for (int c = 0; c < kDotChunk; ++c) {
    const double2 s1 = block_sum(a1[c]);
    const double2 s2 = block_sum(a2[c]);
    if (threadIdx.x == 0 && c < cnt) {
      partial[(long long)(i0 + c) * gridDim.x + blockIdx.x] = s1;
      partial[(long long)(m + i0 + c) * gridDim.x + blockIdx.x] = s2;
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_multi_dot_final(const double2* partial, int nparts,
                                                                 double2* out) {
  const double2 s = fold_partials(partial + (long long)blockIdx.x * nparts, nparts);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// w = wscale (w - sum_i c_i V[i]) and, when V2 is given, z -= sum_i c_i V2[i]
// (the same coefficients), eight basis vectors per unrolled step.
__global__ __launch_bounds__(kRedThreads) void k_multi_axpy(const double2* __restrict__ V,
                                                            const double2* __restrict__ V2,
                                                            long long ld, int m,
                                                            const double2* __restrict__ c,
                                                            double2* __restrict__ w,
                                                            double2* __restrict__ z,
                                                            long long len, double wscale) {
  __shared__ double2 cs[512];
  for (int i = threadIdx.x; i < m; i += kRedThreads) cs[i] = c[i];
  __syncthreads();
  for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < len;
       e += (long long)gridDim.x * kRedThreads) {
    double2 acc = w[e];
    double2 acz = V2 ? z[e] : make_double2(0, 0);
#pragma unroll 8
    for (int i = 0; i < m; ++i) {
      acc = csub(acc, cmul(cs[i], V[i * ld + e]));
      if (V2) acz = csub(acz, cmul(cs[i], V2[i * ld + e]));
    }
    w[e] = cscale(acc, wscale);
    if (V2) z[e] = acz;
  }
}

// In place V[:, 0:k] = V[:, 0:m] S with each thread holding one element of all
// m vectors in registers (m <= MM): a thread reads element e of every vector
// before it writes element e of any, and no other thread touches element e.
template <int MM>
__global__ __launch_bounds__(kRedThreads) void k_rotate_reg(double2* V, long long ld, int m, int k,
                                                            const double2* __restrict__ S,
                                                            long long len) {
  for (long long e = blockIdx.x * (long long)kRedThreads + threadIdx.x; e < len;
       e += (long long)gridDim.x * kRedThreads) {
    double2 x[MM];
#pragma unroll
    for (int i = 0; i < MM; ++i) x[i] = (i < m) ? V[i * ld + e] : make_double2(0, 0);
    for (int c = 0; c < k; ++c) {
      double2 acc = make_double2(0, 0);
#pragma unroll
      for (int i = 0; i < MM; ++i)
        if (i < m) acc = cadd(acc, cmul(x[i], S[c * m + i]));
      V[c * ld + e] = acc;
    }
  }
}

// The same for any m: a slab of `cols` elements of all m vectors is read into
// LDS before any of it is overwritten.
__global__ __launch_bounds__(kRedThreads) void k_rotate(double2* V, long long ld, int m, int k,
                                                        const double2* __restrict__ S,
                                                        long long len, int kRotCols) {
  extern __shared__ double2 slab[];  // m * kRotCols
  const long long e0 = (long long)blockIdx.x * kRotCols;
  for (int t = threadIdx.x; t < m * kRotCols; t += kRedThreads) {
    const int i = t / kRotCols, e = t - i * kRotCols;
    slab[t] = (e0 + e < len) ? V[i * ld + e0 + e] : make_double2(0, 0);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k * kRotCols; t += kRedThreads) {
    const int c = t / kRotCols, e = t - c * kRotCols;
    if (e0 + e >= len) continue;
    double2 acc = make_double2(0, 0);
    for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(slab[i * kRotCols + e], S[c * m + i]));
    V[c * ld + e0 + e] = acc;
  }
}

__global__ void k_scale_copy(const double2* __restrict__ x, double2* __restrict__ y, double sre,
                             double sim, long long len) {
  const double2 s = make_double2(sre, sim);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = cmul(s, x[i]);
}

// splitmix64 finaliser: a counter-based hash of (seed, index).
__device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_randn(double2* v, long long len, unsigned long long seed) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < len;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned long long h1 = mix64(seed ^ mix64(2ull * (unsigned long long)i));
    const unsigned long long h2 = mix64(seed ^ mix64(2ull * (unsigned long long)i + 1ull));
    const double u1 = ((h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);  // (0,1)
    const double u2 = ((h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586476925 * u2, &sn, &cs);
    v[i] = make_double2(rad * cs, rad * sn);
  }
}

// Per frequency: (B_r u)_a = i u_c/s, _b = i u_d/s, _c = -i u_a/s, _d = -i u_b/s.
__global__ __launch_bounds__(kRedThreads) void k_residual(Geom g, Tables t,
                                                          const double2* __restrict__ u,
                                                          const double2* __restrict__ Au,
                                                          double theta, double2* partial) {
  const long long n = g.n;
  double2 acc = make_double2(0, 0);
  for (long long f = blockIdx.x * (long long)kRedThreads + threadIdx.x; f < n;
       f += (long long)gridDim.x * kRedThreads) {
    const int i1 = (int)(f % g.n1);
    const int i2 = (int)((f / g.n1) % g.n2);
    const int i3 = (int)(f / ((long long)g.n1 * g.n2));
    const double s2 = cabs2(t.lam[i1]) + cabs2(t.lam[g.n1 + i2]) + cabs2(t.lam[g.n1 + g.n2 + i3]);
    const double is = 1.0 / sqrt(s2);
    const double2 ua = u[f], ub = u[n + f], uc = u[2 * n + f], ud = u[3 * n + f];
    const double2 B[4] = {cscale(cmuli(uc), is), cscale(cmuli(ud), is), cscale(cmuli(ua), -is),
                          cscale(cmuli(ub), -is)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 a = Au[q * n + f];
      acc.x += cabs2(csub(B[q], cscale(a, theta)));
      acc.y += cabs2(a);
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

int red_grid(long long len) {
  long long b = (len + kRedThreads - 1) / kRedThreads;
  return (int)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

int ew_grid(long long len) {
  long long b = (len + 255) / 256;
  return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

}  // namespace

hipError_t launch_dot_partials(const double2* x, const double2* y, long long len, double2* partial,
                               const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(red_grid(len)), dim3(kRedThreads), 0, s, x, y, len, partial, skip);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double2* partial, int nparts, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partial, nparts, out);
  return hipGetLastError();
}

hipError_t launch_cg_init(const double2* b, double2* x, double2* r, double2* p, long long len,
                          double2* partial, CgState* st, double rtol, int maxit, hipStream_t s,
                          const double2* AV, long long ld, int m, const double2* c, int ring) {
  if (m < 0 || m > 512 || (m > 0 && (!AV || !c))) return hipErrorInvalidValue;
  if (ring < 0 || ring > kCgRing) return hipErrorInvalidValue;
  const int nb = red_grid(len);
  hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kRedThreads), 0, s, b, x, r, p, len, partial, AV, ld, m, c);
  hipLaunchKernelGGL(k_cg_init_final, dim3(1), dim3(kRedThreads), 0, s, partial, nb, st, rtol, maxit, ring);
  return hipGetLastError();
}

hipError_t launch_cg_alpha(const double2* partial, int nparts, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kRedThreads), 0, s, partial, nparts, st);
  return hipGetLastError();
}

hipError_t launch_cg_update(double2* x, double2* r, const double2* p, const double2* q,
                            long long len, double2* partial, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3(red_grid(len)), dim3(kRedThreads), 0, s, x, r, p, q, len,
                     partial, st);
  return hipGetLastError();
}

hipError_t launch_cg_beta(const double2* partial, int nparts, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kRedThreads), 0, s, partial, nparts, st);
  return hipGetLastError();
}

hipError_t launch_cg_p(double2* p, const double2* r, long long len, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p, dim3(red_grid(len)), dim3(kRedThreads), 0, s, p, r, len, st);
  return hipGetLastError();
}

hipError_t launch_cgf_check(const double* part_in, int nparts, CgState* st, hipStream_t s,
                            const InstDesc* insts, int ninst) {
  hipLaunchKernelGGL(k_cgf_check, dim3(ninst), dim3(kRedThreads), 0, s, part_in, nparts, st, insts);
  return hipGetLastError();
}

hipError_t launch_cgf_step(const double* part_out, int nparts, CgState* st, hipStream_t s,
                           const InstDesc* insts, int ninst, const double* part_mid, int np_mid) {
  hipLaunchKernelGGL(k_cgf_step, dim3(ninst), dim3(kRedThreads), 0, s, part_out, nparts, st, insts, part_mid,
                     np_mid);
  return hipGetLastError();
}

hipError_t launch_cgf_alpha(const double* part_mid, int np_mid, CgState* st, hipStream_t s,
                            const InstDesc* insts, int ninst, const double* part_in, int np_in) {
  hipLaunchKernelGGL(k_cgf_alpha, dim3(ninst), dim3(kRedThreads), 0, s, part_mid, np_mid, st, insts, part_in,
                     np_in);
  return hipGetLastError();
}

hipError_t launch_cgf_step_qf(const double* part_out, int nparts, CgState* st, hipStream_t s,
                              const InstDesc* insts, int ninst) {
  hipLaunchKernelGGL(k_cgf_step_qf, dim3(ninst), dim3(kRedThreads), 0, s, part_out, nparts, st, insts);
  return hipGetLastError();
}

hipError_t launch_cg_finish(double2* x, const double2* p, long long len, const CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_finish, dim3(ew_grid(len)), dim3(256), 0, s, x, p, len, st);
  return hipGetLastError();
}

hipError_t launch_cg_fold(double2* x, const double2* ring, long long len, const CgState* st, bool final,
                          hipStream_t s, const InstDesc* insts, int ninst) {
  // a grid of 1024 workgroups: the launch inside every iteration returns at
  // once except when the ring is full
  const dim3 grid((unsigned)std::min(ew_grid(len), 1024), 1, (unsigned)ninst);
  hipLaunchKernelGGL(k_cg_fold, grid, dim3(256), 0, s, x, ring, len, st, final ? 1 : 0, insts);
  return hipGetLastError();
}

hipError_t launch_multi_dot(const double2* V, long long ld, int m, const double2* w, long long len,
                            double2* partial, double2* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  // about 4096 workgroups in all, within the partial-sum slots (m x nb)
  const int rows = (m + kDotChunk - 1) / kDotChunk;
  long long nb = std::min<long long>((len + kRedThreads - 1) / kRedThreads, 4096 / rows);
  nb = std::min<long long>(nb, kPartialSlots / m);
  if (nb < 1) nb = 1;
  const dim3 grid((unsigned)nb, rows);
  hipLaunchKernelGGL(k_multi_dot, grid, dim3(kRedThreads), 0, s, V, ld, m, w, len, partial);
  hipLaunchKernelGGL(k_multi_dot_final, dim3(m), dim3(kRedThreads), 0, s, partial, (int)nb, out);
  return hipGetLastError();
}

hipError_t launch_multi_dot2(const double2* V, long long ld, int m, const double2* w1, const double2* w2,
                             long long len, double2* partial, double2* out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int rows = (m + kDotChunk - 1) / kDotChunk;
  long long nb = std::min<long long>((len + kRedThreads - 1) / kRedThreads, 4096 / rows);
  nb = std::min<long long>(nb, kPartialSlots / (2 * m));
  if (nb < 1) nb = 1;
  const dim3 grid((unsigned)nb, rows);
  hipLaunchKernelGGL(k_multi_dot2, grid, dim3(kRedThreads), 0, s, V, ld, m, w1, w2, len, partial);
  hipLaunchKernelGGL(k_multi_dot_final, dim3(2 * m), dim3(kRedThreads), 0, s, partial, (int)nb, out);
  return hipGetLastError();
}

// The Lanczos step's updates fused with B_r w and the two inner products that
// follow them (launch_step_fused).  B_r at frequency f is i / sigma_f times
// (y_c, y_d, -y_a, -y_b), sigma_f^2 = |lambda_1|^2 + |lambda_2|^2 + |lambda_3|^2.
constexpr int kStepParts = 2048;

__global__ __launch_bounds__(kRedThreads) void k_step_fused(Geom g, Tables t, int mode, double2* w,
                                                            double2* __restrict__ z, double2* b,
                                                            const double2* __restrict__ r,
                                                            const double2* __restrict__ V,
                                                            const double2* __restrict__ AV, long long ld,
                                                            int m, const double2* __restrict__ c,
                                                            double2* partial) {
  __shared__ double2 cs[512];
  __shared__ int ix[512];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    cs[i] = c[i];
    ix[i] = (int)c[m + i].x;
  }
  __syncthreads();
  const long long n = g.n;
  double2 a0 = make_double2(0, 0), a1 = make_double2(0, 0);
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < n;
       f += (long long)gridDim.x * blockDim.x) {
    double2 wv[4], zv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long i = q * n + f;
      if (mode == 0) {
        double2 v = csub(b[i], r[i]);
#pragma unroll 4
        for (int j = 0; j < m; ++j) v = csub(v, cmul(cs[j], AV[ix[j] * ld + i]));
        zv[q] = v;
        wv[q] = w[i];
      } else {
        double2 a = w[i], e = z[i];
#pragma unroll 4
        for (int j = 0; j < m; ++j) {
          a = csub(a, cmul(cs[j], V[ix[j] * ld + i]));
          e = csub(e, cmul(cs[j], AV[ix[j] * ld + i]));
        }
        wv[q] = a;
        zv[q] = e;
      }
    }
    const int i1 = (int)(f % g.n1);
    const int i2 = (int)((f / g.n1) % g.n2);
    const int i3 = (int)(f / ((long long)g.n1 * g.n2));
    const double s2 = cabs2(t.lam[i1]) + cabs2(t.lam[g.n1 + i2]) + cabs2(t.lam[g.n1 + g.n2 + i3]);
    const double is = 1.0 / sqrt(s2);
    const double2 bv[4] = {cscale(cmuli(wv[2]), is), cscale(cmuli(wv[3]), is), cscale(cmuli(wv[0]), -is),
                           cscale(cmuli(wv[1]), -is)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long i = q * n + f;
      if (mode == 1) w[i] = wv[q];
      z[i] = zv[q];
      b[i] = bv[q];
      a0 = cadd(a0, cmulc(wv[q], zv[q]));
      a1 = cadd(a1, cmulc(wv[q], bv[q]));
    }
  }
  a0 = block_sum(a0);
  a1 = block_sum(a1);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a0;
    partial[kStepParts + blockIdx.x] = a1;
  }
}

hipError_t launch_step_fused(const Geom& g, const Tables& t, int mode, double2* w, double2* z, double2* b,
                             const double2* r, const double2* V, const double2* AV, long long ld, int m,
                             const double2* c, double2* partial, double2* res2, hipStream_t s) {
  if (m < 0 || m > 512 || (m > 0 && (!AV || !c)) || (mode == 1 && m > 0 && !V) || (mode == 0 && !r))
    return hipErrorInvalidValue;
  const int nb = (int)std::min<long long>((g.n + kRedThreads - 1) / kRedThreads, kStepParts);
  hipLaunchKernelGGL(k_step_fused, dim3(nb), dim3(kRedThreads), 0, s, g, t, mode, w, z, b, r, V, AV, ld, m, c,
                     partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partial, nb, res2);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partial + kStepParts, nb, res2 + 1);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(const double2* V, long long ld, int m, const double2* c, double2* w,
                             long long len, hipStream_t s, const double2* V2, double2* z, double wscale) {
  if (m <= 0 && wscale == 1.0) return hipSuccess;
  if (m < 0 || m > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_multi_axpy, dim3(ew_grid(len)), dim3(kRedThreads), 0, s, V, V2, ld, m, c, w, z, len,
                     wscale);
  return hipGetLastError();
}

hipError_t launch_rotate(double2* V, long long ld, int m, int k, const double2* S, long long len,
                         hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  const dim3 g(ew_grid(len)), b(kRedThreads);
  if (m <= 16) {
    hipLaunchKernelGGL(k_rotate_reg<16>, g, b, 0, s, V, ld, m, k, S, len);
  } else if (m <= 32) {
    hipLaunchKernelGGL(k_rotate_reg<32>, g, b, 0, s, V, ld, m, k, S, len);
  } else if (m <= 48) {
    hipLaunchKernelGGL(k_rotate_reg<48>, g, b, 0, s, V, ld, m, k, S, len);
  } else {
    int cols = 4096 / m;
    if (cols > 32) cols = 32;
    if (cols < 1) cols = 1;
    const long long blocks = (len + cols - 1) / cols;
    const size_t lds = sizeof(double2) * (size_t)m * cols;
    hipLaunchKernelGGL(k_rotate, dim3((unsigned)blocks), b, lds, s, V, ld, m, k, S, len, cols);
  }
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double2* x, double2* y, double sre, double sim, long long len,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(ew_grid(len)), dim3(256), 0, s, x, y, sre, sim, len);
  return hipGetLastError();
}

hipError_t launch_randn(double2* v, long long len, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_randn, dim3(ew_grid(len)), dim3(256), 0, s, v, len, seed);
  return hipGetLastError();
}

hipError_t launch_residual_norms(const Geom& g, const Tables& t, const double2* u, const double2* Au,
                                 double theta, double2* partial, double* out2, hipStream_t s) {
  const int nb = red_grid(g.n);
  hipLaunchKernelGGL(k_residual, dim3(nb), dim3(kRedThreads), 0, s, g, t, u, Au, theta, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partial, nb,
                     reinterpret_cast<double2*>(out2));
  return hipGetLastError();
}

int reduce_parts_for(long long len) { return red_grid(len); }

}  // namespace nsf
