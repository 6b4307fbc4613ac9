// taylor.hip -- truncated Taylor propagator (see taylor.hpp): the per-step
// plan (Gershgorin interval, degree and substeps per realization) and the
// term launches, which fuse the ELL SpMV with the series update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "taylor.hpp"

namespace paces {

namespace {

template <typename R>
struct TVec;
template <>
struct TVec<double> {
  using T = double2;
};
template <>
struct TVec<float> {
  using T = float2;
};

// theta_m: the largest theta with sum_{k > m} |h_k| theta^(k-1) <= 2^-53,
// where log(exp(-x) T_m(x)) = sum_k h_k x^k.  Here the logarithm is taken
// as the series log(1 + u) = sum_n (-1)^(n+1) u^n / n of
// u = exp(-x) T_m(x) - 1 (which starts at x^(m+1)), the product and powers
// truncated at degree m + 121, in long double.
double theta_of(int m) {
  const int M = m + 121;
  std::vector<long double> ex(M + 1), tm(M + 1, 0.0L), u(M + 1, 0.0L);
  ex[0] = 1.0L;
  for (int i = 1; i <= M; ++i) ex[i] = -ex[i - 1] / i;
  tm[0] = 1.0L;
  for (int j = 1; j <= m; ++j) tm[j] = tm[j - 1] / j;
  for (int k = m + 1; k <= M; ++k) {  // degrees 0..m cancel exactly
    long double sum = 0.0L;
    for (int j = 0; j <= m && j <= k; ++j) sum += ex[k - j] * tm[j];
    u[k] = sum;
  }
  std::vector<long double> h(M + 1, 0.0L), pw = u, nx(M + 1);
  for (int n = 1; n * (m + 1) <= M; ++n) {
    const long double c = ((n & 1) ? 1.0L : -1.0L) / n;
    for (int k = 0; k <= M; ++k) h[k] += c * pw[k];
    std::fill(nx.begin(), nx.end(), 0.0L);
    for (int a = m + 1; a <= M; ++a) {
      if (pw[a] == 0.0L) continue;
      for (int b = m + 1; a + b <= M; ++b) nx[a + b] += pw[a] * u[b];
    }
    pw.swap(nx);
  }
  const long double tol = std::ldexp(1.0L, -53);
  auto over = [&](long double th) {
    long double sum = 0.0L, p = 1.0L;
    for (int k = 1; k <= M; ++k) {
      if (k > m) sum += std::fabs(h[k]) * p;
      p *= th;
    }
    return sum > tol;
  };
  long double lo = 0.0L, hi = 1.0L;
  while (!over(hi)) hi *= 2.0L;
  for (int it = 0; it < 200; ++it) {
    const long double mid = 0.5L * (lo + hi);
    if (over(mid))
      hi = mid;
    else
      lo = mid;
  }
  return double(lo);
}

__global__ void __launch_bounds__(kBlock)
    k_taylor_plan(int Rn, const double* part, int nparts, double dt, int order,
                  const double* thetas, int k_max, int launched,
                  TaylorPlan* plan, ChebCoef* cc, StepCtl* ctl, int* err) {
  if (*err) return;
  const int r = blockIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    lo = fmin(lo, part[(int64_t(i) * Rn + r) * 2]);
    hi = fmax(hi, part[(int64_t(i) * Rn + r) * 2 + 1]);
  }
  lo = block_min(lo);
  hi = block_max(hi);
  if (threadIdx.x != 0) return;
  if (lo > hi) lo = hi = 0.0;  // empty set
  const double pad = 1e-12 * (fabs(hi) + fabs(lo));
  const double emin = lo - pad, emax = hi + pad;
  const double a = 0.5 * (emax - emin), b = 0.5 * (emax + emin);
  const double x = a * dt;
  if (!isfinite(x)) {
    atomicOr(err, kErrNonFinite);
    return;
  }
  int m = order, s = 1;
  if (order <= 0) {
    double best = INFINITY;
    for (int q = 1; q <= kTaylorMaxDeg; ++q) {
      const double sd = fmax(1.0, ceil(x / thetas[q]));
      if (q * sd < best) {
        best = q * sd;
        m = q;
        s = sd < 1e9 ? int(sd) : 1000000000;
      }
    }
    if (best > double(k_max)) {
      atomicOr(err, kErrTerms);
      return;
    }
  }
  const int total = m * s;
  if (total > k_max) {
    atomicOr(err, kErrTerms);
    return;
  }
  if (total > launched) atomicOr(err, kErrNeedTerms);
  atomicMax(&ctl->kmax, uint32_t(total));
  TaylorPlan& p = plan[r];
  p.m = m;
  p.s = s;
  p.b = b;
  double sn, cs;
  sincos(b * dt, &sn, &cs);
  p.phase[0] = cs;
  p.phase[1] = -sn;
  ChebCoef& c = cc[r];
  c.emin = emin;
  c.emax = emax;
  c.a = a;
  c.b = b;
  c.K = total;
}

// Launch L: rows whose realization still has terms take term j of substep
// sig (L = sig m + j - 1).  The substep's start vector v is phi or the other
// F buffer; b_j = -i (dt / (s j)) (H - b) b_(j-1) with b_0 = v; the sum of
// the substep builds in F[sig & 1]; the last launch writes exp(-i b dt) f.
template <typename R, int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_taylor_term(DevModel m, int L, int want_energy, double dt,
                  const StepCtl* __restrict__ ctl, const int* __restrict__ err,
                  const int32_t* __restrict__ col,
                  const uint64_t* __restrict__ pay,
                  const uint64_t* __restrict__ tot,
                  const TaylorPlan* __restrict__ plan,
                  const typename TVec<R>::T* __restrict__ phi,
                  typename TVec<R>::T* B0, typename TVec<R>::T* B1,
                  typename TVec<R>::T* F0, typename TVec<R>::T* F1,
                  typename TVec<R>::T* out, double* e_part, double* e_row) {
  using Amp = typename TVec<R>::T;
  constexpr int D = 2 * ND + 2 * NV;
  if (*err) return;
  const int Rn = m.R;
  if (Rn == 1 && L >= plan[0].m * plan[0].s) return;
  const int64_t n = ctl->n_new;
  R jv[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < ND; ++q) jv[q] = R(m.J[q]);
  const bool energy = L == 0 && want_energy;
  double esum = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint64_t p = ld_stream(pay + i);
    const TaylorPlan& P = plan[Rn > 1 ? pay_real(p) : 0];
    const int total = P.m * P.s;
    if (L >= total) continue;
    const int sig = L / P.m, j = L - sig * P.m + 1;
    const Amp* in = j == 1 ? (sig == 0 ? phi : (((sig - 1) & 1) ? F1 : F0))
                           : (((L - 1) & 1) ? B1 : B0);
    Amp* Bo = (L & 1) ? B1 : B0;
    Amp* Fc = (sig & 1) ? F1 : F0;
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
    if (energy) {
      const double e = double(xi.x) * double(hr) + double(xi.y) * double(hi);
      if (Rn == 1)
        esum += e;
      else
        e_row[i] = e;
    }
    const R bs = R(P.b);
    hr -= bs * xi.x;
    hi -= bs * xi.y;
    const R g = R(dt / (double(P.s) * double(j)));
    Amp t;  // -i g (H - b) x
    t.x = g * hi;
    t.y = -g * hr;
    Amp f;
    if (j == 1) {
      f.x = xi.x + t.x;
      f.y = xi.y + t.y;
    } else {
      const Amp fo = Fc[i];
      f.x = fo.x + t.x;
      f.y = fo.y + t.y;
    }
    if (L == total - 1) {
      const R pr = R(P.phase[0]), pim = R(P.phase[1]);
      Amp o;
      o.x = pr * f.x - pim * f.y;
      o.y = pr * f.y + pim * f.x;
      out[i] = o;
    } else {
      Fc[i] = f;
      if (j < P.m) Bo[i] = t;
    }
  }
  if (Rn == 1 && energy) {
    esum = block_sum(esum);
    if (threadIdx.x == 0) e_part[blockIdx.x] = esum;
  }
}

// <psi|H|psi> of the step's result, for the fixed-order series (which is
// not unitary, so the energy of phi is not that of psi): per-block partials
// (one realization) or per row (batched).
template <typename R, int ND, int NV>
__global__ void __launch_bounds__(kBlock)
    k_taylor_energy(DevModel m, const StepCtl* __restrict__ ctl,
                    const int* __restrict__ err,
                    const int32_t* __restrict__ col,
                    const uint64_t* __restrict__ pay,
                    const uint64_t* __restrict__ tot,
                    const typename TVec<R>::T* __restrict__ psi,
                    double* e_part, double* e_row) {
  using Amp = typename TVec<R>::T;
  constexpr int D = 2 * ND + 2 * NV;
  if (*err) return;
  const int Rn = m.R;
  const int64_t n = ctl->n_new;
  double esum = 0;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint64_t p = ld_stream(pay + i);
    const Amp xi = psi[i];
    const double d = row_diag(m, p, NV > 2 ? ld_stream(tot + i) : 0);
    double hr = d * double(xi.x), hi = d * double(xi.y);
    int32_t cols[D];
    load_cols<D>(col + i * D, cols);
#pragma unroll
    for (int s = 0; s < D; ++s) {
      const int32_t c = cols[s];
      if (c >= 0) {
        double v;
        if (s < 2 * ND) {
          v = m.J[s >> 1];
        } else {
          const int nu = (s - 2 * ND) >> 1;
          v = m.gsq[nu * kGsqStride + pay_occ(p, nu) + ((s - 2 * ND) & 1)];
        }
        const Amp xj = psi[c];
        hr += v * double(xj.x);
        hi += v * double(xj.y);
      }
    }
    const double e = double(xi.x) * hr + double(xi.y) * hi;
    if (Rn == 1)
      esum += e;
    else
      e_row[i] = e;
  }
  if (Rn == 1) {
    esum = block_sum(esum);
    if (threadIdx.x == 0) e_part[blockIdx.x] = esum;
  }
}

}  // namespace

const double* taylor_thetas_host() {
  static const std::vector<double> t = [] {
    std::vector<double> v(kTaylorMaxDeg + 1, 0.0);
    for (int q = 1; q <= kTaylorMaxDeg; ++q) v[q] = theta_of(q);
    return v;
  }();
  return t.data();
}

void taylor_plan(int R, const double* part, int nparts, double dt, int order,
                 const double* thetas_dev, int k_max, int launched,
                 TaylorPlan* plan, ChebCoef* cc, StepCtl* ctl, int* err,
                 hipStream_t s) {
  k_taylor_plan<<<R, kBlock, 0, s>>>(R, part, nparts, dt, order, thetas_dev,
                                     k_max, launched, plan, cc, ctl, err);
}

int taylor_term(const DevModel& m, int prec, int L, bool energy, double dt,
                int64_t est, const StepCtl* ctl, const int32_t* col,
                const Side& n, const TaylorPlan* plan, const void* phi,
                void* const* bufB, void* const* bufF, void* out, double* e_part,
                double* e_row, const int* err, hipEvent_t ev_a,
                hipEvent_t ev_b, hipStream_t s) {
  const int g = grid_for(est);
  const int e = energy ? 1 : 0;
  if (prec == 64) {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        launch_ev(k_taylor_term<double, A, B>, g, s, ev_a, ev_b,
                  m, L, e, dt, ctl, err, col, n.pay, n.tot, plan,
                  (const double2*)phi, (double2*)bufB[0], (double2*)bufB[1],
                  (double2*)bufF[0], (double2*)bufF[1], (double2*)out, e_part,
                  e_row));
  } else {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        launch_ev(k_taylor_term<float, A, B>, g, s, ev_a, ev_b,
                  m, L, e, dt, ctl, err, col, n.pay, n.tot, plan,
                  (const float2*)phi, (float2*)bufB[0], (float2*)bufB[1],
                  (float2*)bufF[0], (float2*)bufF[1], (float2*)out, e_part,
                  e_row));
  }
  return g;
}

int taylor_energy(const DevModel& m, int prec, int64_t est,
                  const StepCtl* ctl, const int32_t* col, const Side& n,
                  const void* psi, double* e_part, double* e_row,
                  const int* err, hipStream_t s) {
  const int g = grid_for(est);
  if (prec == 64) {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        k_taylor_energy<double, A, B><<<g, kBlock, 0, s>>>(
            m, ctl, err, col, n.pay, n.tot, (const double2*)psi, e_part,
            e_row));
  } else {
    PACES_DISPATCH_SHAPE(m.ndim, m.V,
        k_taylor_energy<float, A, B><<<g, kBlock, 0, s>>>(
            m, ctl, err, col, n.pay, n.tot, (const float2*)psi, e_part,
            e_row));
  }
  return g;
}

}  // namespace paces
