// adjoint.hip -- kernels of the adjoint gradient (Form (3)) on gfx950.
//
// The backward pass walks the recorded steps in reverse.  Per step it
//   1. propagates the adjoint vector back, mu = exp(+i H dt) lambda, with
//      the step kernels' Clenshaw launches and conjugated coefficients;
//   2. propagates mu and phi = T_s psi_s to the Gauss-Legendre nodes tau_q
//      of [0, 1] with one three-term Chebyshev recurrence per vector, both
//      chains in the same launch (they share the ELL columns and payload),
//      each term added to one accumulator per node;
//   3. contracts the node vectors with dH/dtheta_p for every parameter at
//      once (hops per axis, e-ph slots per mode, totals per mode, exciton
//      site) into per-block partials;
//   4. maps mu back onto the previous set through the recorded row map.
// Like the step kernels these are memory-bound row streams on wave64,
// 256-lane blocks; the arithmetic is FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "adjoint.hpp"
#include "common.hpp"

namespace paces {

namespace {

__global__ void k_adj_set_frozen(StepCtl* ctl, uint32_t* cnt, uint32_t nM,
                                 const int* err) {
  if (*err) return;
  ctl->nM = nM;
  ctl->fstart[0] = 0;
  ctl->fstart[1] = nM;
  cnt[0] = nM;
}

__global__ void k_adj_set_rows(StepCtl* ctl, uint32_t n) { ctl->n_new = n; }

__global__ void k_adj_conj_coef(const ChebCoef* in, ChebCoef* out) {
  for (int k = threadIdx.x; k < kMaxTerms; k += blockDim.x) {
    out->c[k][0] = in->c[k][0];
    out->c[k][1] = -in->c[k][1];
  }
  if (threadIdx.x == 0) {
    out->emin = in->emin;
    out->emax = in->emax;
    out->a = in->a;
    out->b = in->b;
    out->alpha = in->alpha;
    out->beta = in->beta;
    out->phase[0] = in->phase[0];
    out->phase[1] = -in->phase[1];
    out->K = in->K;
  }
}

// Block q: coefficients of exp(-i tau_q H dt) on the step's interval,
// c_k = (2 - delta_k0) (-i)^k J_k(a tau_q dt) times exp(-i b tau_q dt),
// zero beyond the node's own term count.
__global__ void __launch_bounds__(kBlock)
    k_adj_node_coef(const ChebCoef* cc, double dt, const double* tau,
                    double tol, double2* cn, int* err) {
  __shared__ double J[kMaxTerms + 1];
  if (*err) return;
  const int q = blockIdx.x;
  const double x = cc->a * tau[q] * dt;
  const int kcap = kMaxTerms - 1;
  if (!(x <= double(kcap))) {  // the step itself had a finite, smaller x
    if (threadIdx.x == 0) atomicOr(err, kErrTerms);
    return;
  }
  if (x <= 2.0) {
    for (int k = threadIdx.x; k <= kcap; k += blockDim.x)
      J[k] = bessel_series(x, k);
  } else if (threadIdx.x == 0) {
    bessel_miller(x, kcap, J);
  }
  __syncthreads();
  // the step's own rule (omitted tail within tol): a node's x is at most
  // the step's, so its term count is too
  const double thresh = ldexp(tol, -2);
  double last = 0;
  for (int k = threadIdx.x; k <= kcap; k += blockDim.x)
    if (fabs(J[k]) > thresh) last = fmax(last, double(k));
  last = block_max(last);
  const int K = int(last) + 1;
  if (K > cc->K && threadIdx.x == 0) atomicOr(err, kErrTerms);
  double sn, cs;
  sincos(cc->b * tau[q] * dt, &sn, &cs);
  const double pr = cs, pi = -sn;  // exp(-i b tau dt)
  for (int k = threadIdx.x; k < kMaxTerms; k += blockDim.x) {
    double cr = 0, ci = 0;
    if (k < K) {
      const double v = (k == 0 ? 1.0 : 2.0) * J[k];
      const int r = k & 3;  // (-i)^k
      cr = (r == 0) ? v : (r == 2 ? -v : 0.0);
      ci = (r == 1) ? -v : (r == 3 ? v : 0.0);
    }
    double2 o;
    o.x = pr * cr - pi * ci;
    o.y = pr * ci + pi * cr;
    cn[q * kMaxTerms + k] = o;
  }
}

// H applied to row i of v (ELL, values implied by slot and payload).
template <int ND, int NV>
__device__ __forceinline__ double2 h_row(const DevModel& m, int64_t i,
                                         int64_t n, const int32_t* col,
                                         uint64_t p, uint64_t t,
                                         const double2* v) {
  constexpr int D = 2 * ND + 2 * NV;
  const double d = row_diag(m, p, NV > 2 ? t : 0);
  const double2 xi = v[i];
  double hr = d * xi.x, hi = d * xi.y;
#pragma unroll
  for (int s = 0; s < D; ++s) {
    const int32_t c = col[i * D + s];
    if (c >= 0) {
      const double val = slot_value(m, p, s);
      const double2 xj = v[c];
      hr += val * xj.x;
      hi += val * xj.y;
    }
  }
  return make_double2(hr, hi);
}

// Launch kk of the recurrence T_{k+1} = 2 H~ T_k - T_{k-1} (T_1 = H~ T_0)
// for both chains; T_{k+1} overwrites T_{k-1} row by row (a row reads only
// its own T_{k-1} entry, and neighbours read T_k).  acc[q] += cn[q][kk] T_kk.
template <int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_adj_nodes(DevModel m, int kk, int K, int64_t n,
                const int32_t* __restrict__ col,
                const uint64_t* __restrict__ pay,
                const uint64_t* __restrict__ tot,
                const ChebCoef* __restrict__ cc,
                const double2* __restrict__ cn, int nq, double2* tx0,
                double2* tx1, double2* ty0, double2* ty1, double2* accx,
                double2* accy, const int* err) {
  if (*err) return;
  const double alpha = cc->alpha, beta = cc->beta;
  double2* xk = (kk & 1) ? tx1 : tx0;   // T_k
  double2* xo = (kk & 1) ? tx0 : tx1;   // T_{k-1} in, T_{k+1} out
  double2* yk = (kk & 1) ? ty1 : ty0;
  double2* yo = (kk & 1) ? ty0 : ty1;
  const bool more = kk + 1 < K;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const double2 xv = xk[i], yv = yk[i];
    for (int q = 0; q < nq; ++q) {
      const double2 c = cn[q * kMaxTerms + kk];
      double2 ax = kk ? accx[q * n + i] : make_double2(0.0, 0.0);
      double2 ay = kk ? accy[q * n + i] : make_double2(0.0, 0.0);
      ax.x += c.x * xv.x - c.y * xv.y;
      ax.y += c.x * xv.y + c.y * xv.x;
      ay.x += c.x * yv.x - c.y * yv.y;
      ay.y += c.x * yv.y + c.y * yv.x;
      accx[q * n + i] = ax;
      accy[q * n + i] = ay;
    }
    if (!more) continue;
    const uint64_t p = pay[i];
    const uint64_t t = NV > 2 ? tot[i] : 0;
    const double2 hx = h_row<ND, NV>(m, i, n, col, p, t, xk);
    const double2 hy = h_row<ND, NV>(m, i, n, col, p, t, yk);
    double2 ox, oy;
    ox.x = alpha * hx.x + beta * xv.x;
    ox.y = alpha * hx.y + beta * xv.y;
    oy.x = alpha * hy.x + beta * yv.x;
    oy.y = alpha * hy.y + beta * yv.y;
    if (kk > 0) {
      const double2 xm = xo[i], ym = yo[i];
      ox.x = 2.0 * ox.x - xm.x;
      ox.y = 2.0 * ox.y - xm.y;
      oy.x = 2.0 * oy.x - ym.x;
      oy.y = 2.0 * oy.y - ym.y;
    }
    xo[i] = ox;
    yo[i] = oy;
  }
}

// Im(conj(a) b)
__device__ __forceinline__ double im_cb(double2 a, double2 b) {
  return a.x * b.y - a.y * b.x;
}

// Per-block partials of sum_q w_q Im <x_q| dH/dtheta_p |y_q>, parameters
// ordered J (ND axes), g (NV modes), omega (NV modes), eps (N sites).  The
// site bins live in LDS (dynamic, N doubles).
template <int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_adj_contract(DevModel m, int64_t n, const int32_t* __restrict__ col,
                   const uint64_t* __restrict__ pay,
                   const uint64_t* __restrict__ tot, int nq,
                   const double* __restrict__ w,
                   const double2* __restrict__ accx,
                   const double2* __restrict__ accy, double* part,
                   const int* err) {
  extern __shared__ double site_bins[];
  if (*err) return;
  constexpr int D = 2 * ND + 2 * NV;
  const int N = m.N, P = ND + 2 * NV + N;
  for (int j = threadIdx.x; j < N; j += blockDim.x) site_bins[j] = 0.0;
  __syncthreads();
  double gJ[ND], gG[NV], gW[NV];
#pragma unroll
  for (int a = 0; a < ND; ++a) gJ[a] = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) gG[v] = gW[v] = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint64_t p = pay[i];
    const uint64_t t = NV > 2 ? tot[i] : 0;
    double diag = 0;  // sum_q w_q Im(conj(x) y)
    for (int q = 0; q < nq; ++q) {
      const double wq = w[q];
      const double2* xq = accx + q * n;
      const double2* yq = accy + q * n;
      const double2 xi = xq[i];
      diag += wq * im_cb(xi, yq[i]);
#pragma unroll
      for (int s = 0; s < 2 * ND; ++s) {
        const int32_t c = col[i * D + s];
        if (c >= 0) gJ[s >> 1] += wq * im_cb(xi, yq[c]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int occ = pay_occ(p, v);
        const int32_t cl = col[i * D + 2 * ND + 2 * v];
        const int32_t cr = col[i * D + 2 * ND + 2 * v + 1];
        double e = 0;
        if (cl >= 0) e += sqrt(double(occ)) * im_cb(xi, yq[cl]);
        if (cr >= 0) e += sqrt(double(occ + 1)) * im_cb(xi, yq[cr]);
        gG[v] += wq * e;
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      gW[v] += double(row_total(NV, p, t, v)) * diag;
    atomicAdd(&site_bins[pay_site(p)], diag);
  }
  double* out = part + int64_t(blockIdx.x) * P;
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    const double r = block_sum(gJ[a]);
    if (threadIdx.x == 0) out[a] = r;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double r = block_sum(gG[v]);
    if (threadIdx.x == 0) out[ND + v] = r;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double r = block_sum(gW[v]);
    if (threadIdx.x == 0) out[ND + NV + v] = r;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x)
    out[ND + 2 * NV + j] = site_bins[j];
}

// Block p: grad[p] += scale * sum_b part[b][p], partials in a fixed order.
__global__ void __launch_bounds__(kBlock)
    k_adj_fold(const double* part, int nb, int P, double scale, double* grad,
               const int* err) {
  if (*err) return;
  const int p = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    s += part[int64_t(b) * P + p];
  s = block_sum(s);
  if (threadIdx.x == 0) grad[p] += scale * s;
}

__global__ void __launch_bounds__(kBlock)
    k_adj_back(int64_t n, const int32_t* tmap, const double2* mu,
               double2* lam, const int* err) {
  if (*err) return;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int32_t r = tmap[i];
    lam[i] = r >= 0 ? mu[r] : make_double2(0.0, 0.0);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_adj_add_psi0(int64_t n0, const int32_t* p0, const double* amps0,
                   const double* g, double2* lam, const int* err) {
  if (*err) return;
  const double gr = g[0], gi = g[1];
  for (int64_t q = gtid(); q < n0; q += gstride()) {
    const int32_t r = p0[q];
    if (r < 0) continue;
    const double ar = amps0[2 * q], ai = amps0[2 * q + 1];
    double2 v = lam[r];
    v.x += gr * ar - gi * ai;
    v.y += gr * ai + gi * ar;
    lam[r] = v;
  }
}

template <int W>
__global__ void __launch_bounds__(kBlock)
    k_adj_permute(DevModel m, const uint64_t* keys_in, int64_t n,
                  const uint64_t* table, uint64_t mask,
                  const uint64_t* keys_tab, const double2* in, double2* out,
                  int* err) {
  if (*err) return;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    uint64_t k[W];
    load_key<W>(keys_in, i, k);
    const int64_t r = table_find<W>(table, mask, keys_tab, k, key_hash<W>(m, k));
    if (r < 0) {
      atomicOr(err, kErrCapacity);
      continue;
    }
    out[r] = in[i];
  }
}

__global__ void __launch_bounds__(kBlock)
    k_adj_zero(double2* v, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) v[i] = make_double2(0.0, 0.0);
}

}  // namespace

void adj_set_frozen(StepCtl* ctl, uint32_t* cnt, uint32_t nM, int* err,
                    hipStream_t s) {
  k_adj_set_frozen<<<1, 1, 0, s>>>(ctl, cnt, nM, err);
}

void adj_set_rows(StepCtl* ctl, uint32_t n, hipStream_t s) {
  k_adj_set_rows<<<1, 1, 0, s>>>(ctl, n);
}

void adj_conj_coef(const ChebCoef* in, ChebCoef* out, hipStream_t s) {
  k_adj_conj_coef<<<1, kBlock, 0, s>>>(in, out);
}

void adj_node_coef(const ChebCoef* cc, double dt, const double* tau, int nq,
                   double tol, double2* cn, int* err, hipStream_t s) {
  k_adj_node_coef<<<nq, kBlock, 0, s>>>(cc, dt, tau, tol, cn, err);
}

void adj_nodes(const DevModel& m, int kk, int K, int64_t n,
               const int32_t* col, const uint64_t* pay, const uint64_t* tot,
               const ChebCoef* cc, const double2* cn, int nq,
               double2* tx0, double2* tx1, double2* ty0, double2* ty1,
               double2* accx, double2* accy, int* err, hipStream_t s) {
  if (n <= 0) return;
  const int g = grid_for(n);
  PACES_DISPATCH_SHAPE(m.ndim, m.V,
      k_adj_nodes<A, B><<<g, kBlock, 0, s>>>(m, kk, K, n, col, pay, tot, cc,
                                             cn, nq, tx0, tx1, ty0, ty1,
                                             accx, accy, err));
}

int adj_contract(const DevModel& m, int64_t n, const int32_t* col,
                 const uint64_t* pay, const uint64_t* tot, int nq,
                 const double* w, const double2* accx, const double2* accy,
                 double* part, int* err, hipStream_t s) {
  const int g = std::min(grid_for(n), 1024);
  const size_t lds = sizeof(double) * m.N;
  PACES_DISPATCH_SHAPE(m.ndim, m.V,
      k_adj_contract<A, B><<<g, kBlock, lds, s>>>(m, n, col, pay, tot, nq, w,
                                                  accx, accy, part, err));
  return g;
}

void adj_fold(const double* part, int nb, int P, double scale, double* grad,
              int* err, hipStream_t s) {
  k_adj_fold<<<P, kBlock, 0, s>>>(part, nb, P, scale, grad, err);
}

void adj_back(int64_t n, const int32_t* tmap, const double2* mu,
              double2* lam, int* err, hipStream_t s) {
  if (n <= 0) return;
  k_adj_back<<<grid_for(n), kBlock, 0, s>>>(n, tmap, mu, lam, err);
}

void adj_add_psi0(int64_t n0, const int32_t* p0, const double* amps0,
                  const double* g, double2* lam, int* err, hipStream_t s) {
  if (n0 <= 0) return;
  k_adj_add_psi0<<<grid_for(n0), kBlock, 0, s>>>(n0, p0, amps0, g, lam, err);
}

void adj_permute(const DevModel& m, int Wi, const uint64_t* keys_in,
                 int64_t n, const uint64_t* table, uint64_t mask,
                 const uint64_t* keys_tab, const double2* in, double2* out,
                 int* err, hipStream_t s) {
  if (n <= 0) return;
  PACES_DISPATCH_W(Wi, k_adj_permute<WW><<<grid_for(n), kBlock, 0, s>>>(
                           m, keys_in, n, table, mask, keys_tab, in, out, err));
}

void adj_zero(double2* v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_adj_zero<<<grid_for(n), kBlock, 0, s>>>(v, n);
}

}  // namespace paces
