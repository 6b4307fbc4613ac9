// lanczos.hip -- kernels of the Krylov (Lanczos) propagator (paper: App.
// "Series-based exponentiation compared to a Lanczos algorithm").
//
// Every Lanczos iteration is one SpMV over H_eff (the same ELL layout and
// matrix-element tables as the Chebyshev launches) with its inner products
// reduced per block, a one-block fold per realization, and one streaming
// pass for the three-term recurrence.  The small exponential exp(-i T dt) e_1
// runs in one wave per realization, lane j holding component j of the
// Krylov vectors.  Row counts come from the device StepCtl, so the whole
// sequence is enqueued (and captured) without host waits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "lanczos.hpp"

namespace paces {

namespace {

template <typename R>
struct LzVec;
template <>
struct LzVec<double> {
  using T = double2;
};
template <>
struct LzVec<float> {
  using T = float2;
};

// Realization state s takes part in iteration j.
__device__ __forceinline__ bool lz_live(const LanczosState& s, int j) {
  return !s.done && s.dim == j;
}

__global__ void k_lz_begin(LanczosState* st, int R, const int* err) {
  if (*err) return;
  for (int r = threadIdx.x; r < R; r += blockDim.x) {
    st[r].dim = 0;
    st[r].done = 0;
  }
}

// z = H w_j for the rows of live realizations, with per-block partial sums
// of Re<w_j, z>, |w_j|^2 and |z|^2 (per realization in LDS when batched).
template <typename R, int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_lz_spmv(DevModel m, int j, const StepCtl* __restrict__ ctl,
              const int* __restrict__ err, const int32_t* __restrict__ col,
              const uint64_t* __restrict__ pay,
              const uint64_t* __restrict__ tot,
              const LanczosState* __restrict__ st,
              const typename LzVec<R>::T* __restrict__ in,
              typename LzVec<R>::T* out, double* part) {
  using Amp = typename LzVec<R>::T;
  constexpr int D = 2 * ND + 2 * NV;
  __shared__ double acc[3 * kMaxReal];
  if (*err) return;
  const int Rn = m.R;
  if (Rn == 1 && !lz_live(st[0], j)) return;
  const int64_t n = ctl->n_new;
  R jv[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < ND; ++a) jv[a] = R(m.J[a]);
  if (Rn > 1) {
    for (int q = threadIdx.x; q < 3 * Rn; q += blockDim.x) acc[q] = 0.0;
    __syncthreads();
  }
  double sp = 0, sn = 0, sz = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint64_t p = ld_stream(pay + i);
    const int r = Rn > 1 ? pay_real(p) : 0;
    if (Rn > 1 && !lz_live(st[r], j)) continue;
    const Amp xi = in[i];
    const R d = R(row_diag(m, p, NV > 2 ? ld_stream(tot + i) : 0));
    R hr = d * xi.x, hi = d * xi.y;
    R gv[NV][2];
#pragma unroll
    for (int nu = 0; nu < NV; ++nu) {
      const int occ = pay_occ(p, nu);
      gv[nu][0] = R(m.gsq[nu * kGsqStride + occ]);
      gv[nu][1] = R(m.gsq[nu * kGsqStride + occ + 1]);
    }
    int32_t cols[D];
    load_cols<D>(col + i * D, cols);
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int32_t c = cols[s];
      if (c >= 0) {
        const R v = s < 2 * ND ? jv[s >> 1] : gv[(s - 2 * ND) >> 1][(s - 2 * ND) & 1];
        const Amp xj = in[c];
        hr += v * xj.x;
        hi += v * xj.y;
      }
    }
    if (out) {
      Amp o;
      o.x = hr;
      o.y = hi;
      out[i] = o;
    }
    const double xr = double(xi.x), xim = double(xi.y);
    const double zr = double(hr), zi = double(hi);
    const double vp = xr * zr + xim * zi, vn = xr * xr + xim * xim,
                 vz = zr * zr + zi * zi;
    if (Rn == 1) {
      sp += vp;
      sn += vn;
      sz += vz;
    } else {
      atomicAdd(&acc[3 * r], vp);
      atomicAdd(&acc[3 * r + 1], vn);
      atomicAdd(&acc[3 * r + 2], vz);
    }
  }
  if (Rn == 1) {
    sp = block_sum(sp);
    sn = block_sum(sn);
    sz = block_sum(sz);
    if (threadIdx.x == 0) {
      part[3 * blockIdx.x] = sp;
      part[3 * blockIdx.x + 1] = sn;
      part[3 * blockIdx.x + 2] = sz;
    }
  } else {
    __syncthreads();
    for (int q = threadIdx.x; q < 3 * Rn; q += blockDim.x)
      part[int64_t(blockIdx.x) * 3 * Rn + q] = acc[q];
  }
}

// Block r: fold the partials of SpMV j for realization r.
__global__ void __launch_bounds__(kBlock)
    k_lz_fold(int j, const double* part, int nparts, int Rn, double brk2,
              LanczosState* st, double* energy, const int* err) {
  if (*err) return;
  const int r = blockIdx.x;
  LanczosState& s = st[r];
  if (!lz_live(s, j)) return;
  double P = 0, N = 0, Z = 0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    const double* q = part + (int64_t(b) * Rn + r) * 3;
    P += q[0];
    N += q[1];
    Z += q[2];
  }
  P = block_sum(P);
  N = block_sum(N);
  Z = block_sum(Z);
  if (threadIdx.x != 0) return;
  if (j == 0) {
    energy[r] = P;  // <phi|H|phi>
    s.beta[0] = sqrt(N);
    if (!(N > 0.0)) {  // zero start: the result is zero
      s.done = 1;
      return;
    }
  } else if (N <= brk2 * s.hn2[j - 1]) {  // invariant space: stop here
    s.done = 1;
    return;
  } else {
    s.beta[j] = sqrt(N);
  }
  s.alpha[j] = P / N;
  s.hn2[j] = Z / N;
  s.dim = j + 1;
}

// w_{j+1} = (z - alpha_j w_j) / beta_j - (beta_j / beta_{j-1}) w_{j-1}, in
// place over z, for realizations that accepted v_j.
template <typename R>
__global__ void __launch_bounds__(kBlock)
    k_lz_orth(int Rn, int j, const StepCtl* __restrict__ ctl,
              const int* __restrict__ err, const uint64_t* __restrict__ pay,
              const LanczosState* __restrict__ st,
              typename LzVec<R>::T* z,
              const typename LzVec<R>::T* __restrict__ wj,
              const typename LzVec<R>::T* __restrict__ wjm1) {
  using Amp = typename LzVec<R>::T;
  if (*err) return;
  if (Rn == 1 && !lz_live(st[0], j + 1)) return;
  const int64_t n = ctl->n_new;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int r = Rn > 1 ? pay_real(ld_stream(pay + i)) : 0;
    const LanczosState& s = st[r];
    if (Rn > 1 && !lz_live(s, j + 1)) continue;
    const R ib = R(1.0 / s.beta[j]), a = R(s.alpha[j]);
    const Amp zi = z[i], x = ld_stream(wj + i);
    Amp o;
    o.x = (zi.x - a * x.x) * ib;
    o.y = (zi.y - a * x.y) * ib;
    if (j > 0) {
      const R c = R(s.beta[j] / s.beta[j - 1]);
      const Amp q = ld_stream(wjm1 + i);
      o.x -= c * q.x;
      o.y -= c * q.y;
    }
    z[i] = o;
  }
}

// One wave per realization: u = exp(-i T dt) e_1 by the Chebyshev series of
// the padded Gershgorin interval of T (same coefficients and term rule as
// the series propagator), evaluated with Clenshaw's recurrence; lane l
// holds component l, neighbours through lane shuffles.
__global__ void __launch_bounds__(64)
    k_lz_small(int Rn, double dt, double tol, int k_max, LanczosState* st,
               ChebCoef* cc_all, StepCtl* ctl, int* err) {
  __shared__ double J[kMaxTerms + 1];
  if (*err) return;
  const int r = blockIdx.x, l = threadIdx.x;
  LanczosState& s = st[r];
  ChebCoef* cc = cc_all + r;
  const int n = s.dim;
  if (n == 0) {
    s.s[l][0] = s.s[l][1] = 0.0;
    if (l == 0) {
      cc->K = 0;
      cc->emin = cc->emax = 0.0;
    }
    return;
  }
  double lo = INFINITY, hi = -INFINITY;
  if (l < n) {
    double rad = 0;
    if (l > 0) rad += fabs(s.beta[l]);
    if (l + 1 < n) rad += fabs(s.beta[l + 1]);
    lo = s.alpha[l] - rad;
    hi = s.alpha[l] + rad;
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  const double pad = 1e-12 * (fabs(hi) + fabs(lo));
  const double emin = lo - pad, emax = hi + pad;
  double a = 0.5 * (emax - emin);
  const double b = 0.5 * (emax + emin);
  if (!(a > 1e-300)) a = 1e-300;
  const double x = a * dt;
  const int kcap = k_max < kMaxTerms ? k_max : kMaxTerms;
  if (!(x <= double(kcap))) {
    if (l == 0) atomicOr(err, isfinite(x) ? kErrTerms : kErrNonFinite);
    return;
  }
  if (x <= 2.0) {
    for (int k = l; k <= kcap; k += 64) J[k] = bessel_series(x, k);
  } else if (l == 0) {
    bessel_miller(x, kcap, J);
  }
  __syncthreads();
  // the Clenshaw step's rule: terms up to the last |J_k| above tol / 4
  const double thresh = ldexp(tol, -2);
  double last = 0;
  for (int k = l; k <= kcap; k += 64)
    if (fabs(J[k]) > thresh) last = fmax(last, double(k));
  last = wave_max(last);
  int K = int(last) + 1;
  if (K > kcap) {
    if (l == 0) atomicOr(err, kErrTerms);
    return;
  }
  // T~ = (T - b) / a restricted to the lanes below n
  const double dl = l < n ? (s.alpha[l] - b) / a : 0.0;
  const double bl = (l > 0 && l < n) ? s.beta[l] / a : 0.0;     // (l-1, l)
  const double bu = (l + 1 < n) ? s.beta[l + 1] / a : 0.0;      // (l, l+1)
  const double e1 = l == 0 ? 1.0 : 0.0;
  double b1r = 0, b1i = 0, b2r = 0, b2i = 0;  // b_{k+1}, b_{k+2}
  for (int k = K - 1; k >= 1; --k) {
    const double tr = dl * b1r + bl * __shfl_up(b1r, 1, 64) + bu * __shfl_down(b1r, 1, 64);
    const double ti = dl * b1i + bl * __shfl_up(b1i, 1, 64) + bu * __shfl_down(b1i, 1, 64);
    // c_k = 2 J_k (-i)^k
    const double v = 2.0 * J[k];
    const int q = k & 3;
    const double ckr = (q == 0) ? v : (q == 2 ? -v : 0.0);
    const double cki = (q == 1) ? -v : (q == 3 ? v : 0.0);
    const double nr = ckr * e1 + 2.0 * tr - b2r;
    const double ni = cki * e1 + 2.0 * ti - b2i;
    b2r = b1r;
    b2i = b1i;
    b1r = nr;
    b1i = ni;
  }
  const double tr = dl * b1r + bl * __shfl_up(b1r, 1, 64) + bu * __shfl_down(b1r, 1, 64);
  const double ti = dl * b1i + bl * __shfl_up(b1i, 1, 64) + bu * __shfl_down(b1i, 1, 64);
  const double yr = J[0] * e1 + tr - b2r, yi = ti - b2i;  // c_0 = J_0
  double sn, cs;
  sincos(b * dt, &sn, &cs);  // exp(-i b dt) = cs - i sn
  const double ur = cs * yr + sn * yi, ui = cs * yi - sn * yr;
  if (l < n) {
    const double w = s.beta[0] / s.beta[l];  // beta_0 u_l / beta_l
    s.s[l][0] = w * ur;
    s.s[l][1] = w * ui;
  } else {
    s.s[l][0] = s.s[l][1] = 0.0;
  }
  if (l == 0) {
    cc->emin = emin;
    cc->emax = emax;
    cc->a = a;
    cc->b = b;
    cc->alpha = 1.0 / a;
    cc->beta = -b / a;
    cc->phase[0] = cs;
    cc->phase[1] = -sn;
    cc->K = n;
    atomicMax(&ctl->kmax, uint32_t(n));
  }
}

// out = sum_{j < dim} s_j w_j per row.
template <typename R>
__global__ void __launch_bounds__(kBlock)
    k_lz_combine(int Rn, const StepCtl* __restrict__ ctl,
                 const int* __restrict__ err, const uint64_t* __restrict__ pay,
                 const LanczosState* __restrict__ st, KrylovVecs w, int nv,
                 typename LzVec<R>::T* out) {
  using Amp = typename LzVec<R>::T;
  if (*err) return;
  const int64_t n = ctl->n_new;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const int r = Rn > 1 ? pay_real(ld_stream(pay + i)) : 0;
    const LanczosState& s = st[r];
    const int dim = s.dim < nv ? s.dim : nv;
    R yr = 0, yi = 0;
    for (int j = 0; j < dim; ++j) {
      const Amp x = ld_stream(static_cast<const Amp*>(w.w[j]) + i);
      const R cr = R(s.s[j][0]), ci = R(s.s[j][1]);
      yr += cr * x.x - ci * x.y;
      yi += cr * x.y + ci * x.x;
    }
    Amp o;
    o.x = yr;
    o.y = yi;
    out[i] = o;
  }
}

// Record field 2 (energy) of the step being recorded: <phi|H|phi> from the
// first Lanczos SpMV.  Runs after the record is written and before the step
// is committed; skipped like the record when an error is latched.
__global__ void k_lz_energy(int Rn, const double* energy, const StepCtl* ctl,
                            double* ring, int rec_doubles, int64_t ring_cap,
                            const int* err) {
  if (*err) return;
  if (int64_t(ctl->nrec) + 1 > ring_cap) return;
  for (int r = threadIdx.x; r < Rn; r += blockDim.x)
    ring[(int64_t(ctl->nrec) * Rn + r) * rec_doubles + 2] = energy[r];
}

}  // namespace

void lz_record_energy(int R, const double* energy, const StepCtl* ctl,
                      double* ring, int rec_doubles, int64_t ring_cap,
                      const int* err, hipStream_t s) {
  k_lz_energy<<<1, kBlock, 0, s>>>(R, energy, ctl, ring, rec_doubles,
                                   ring_cap, err);
}

void lz_begin(LanczosState* st, int R, const int* err, hipStream_t s) {
  k_lz_begin<<<1, kBlock, 0, s>>>(st, R, err);
}

int lz_spmv(const DevModel& m, int prec, int j, int64_t est,
            const StepCtl* ctl, const int32_t* col, const Side& n,
            const LanczosState* st, const void* in, void* out, double* part,
            const int* err, hipEvent_t ev_a, hipEvent_t ev_b,
            hipStream_t s) {
  const int g = grid_for(est, m.R == 1 ? kLzGrid1 : kPartBlocks);
  if (prec == 64) {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        launch_ev(k_lz_spmv<double, A, B>, g, s, ev_a, ev_b,
                  m, j, ctl, err, col, n.pay, n.tot, st, (const double2*)in,
                  (double2*)out, part));
  } else {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        launch_ev(k_lz_spmv<float, A, B>, g, s, ev_a, ev_b,
                  m, j, ctl, err, col, n.pay, n.tot, st, (const float2*)in,
                  (float2*)out, part));
  }
  return g;
}

void lz_fold(int j, const double* part, int nparts, int R, double brk2,
             LanczosState* st, double* energy, const int* err, hipStream_t s) {
  k_lz_fold<<<R, kBlock, 0, s>>>(j, part, nparts, R, brk2, st, energy, err);
}

void lz_orth(const DevModel& m, int prec, int j, int64_t est,
             const StepCtl* ctl, const uint64_t* pay, const LanczosState* st,
             void* z, const void* wj, const void* wjm1, const int* err,
             hipStream_t s) {
  const int g = grid_for(est);
  if (prec == 64)
    k_lz_orth<double><<<g, kBlock, 0, s>>>(m.R, j, ctl, err, pay, st,
                                           (double2*)z, (const double2*)wj,
                                           (const double2*)wjm1);
  else
    k_lz_orth<float><<<g, kBlock, 0, s>>>(m.R, j, ctl, err, pay, st,
                                          (float2*)z, (const float2*)wj,
                                          (const float2*)wjm1);
}

void lz_small(int R, double dt, double tol, int k_max, LanczosState* st,
              ChebCoef* cc, StepCtl* ctl, int* err, hipStream_t s) {
  k_lz_small<<<R, 64, 0, s>>>(R, dt, tol, k_max, st, cc, ctl, err);
}

void lz_combine(const DevModel& m, int prec, int64_t est, const StepCtl* ctl,
                const uint64_t* pay, const LanczosState* st,
                const KrylovVecs& w, int nv, void* out, const int* err,
                hipStream_t s) {
  const int g = grid_for(est);
  if (prec == 64)
    k_lz_combine<double><<<g, kBlock, 0, s>>>(m.R, ctl, err, pay, st, w, nv,
                                              (double2*)out);
  else
    k_lz_combine<float><<<g, kBlock, 0, s>>>(m.R, ctl, err, pay, st, w, nv,
                                             (float2*)out);
}

}  // namespace paces
