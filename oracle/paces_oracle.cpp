// paces_oracle.cpp -- plain FP64 CPU reference of the co-evolving-subspace
// step for single-exciton Holstein lattices.
//
// TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
// baseline of the benchmark.  It shares no code with the GPU library.  It is
// written for obvious correctness, not speed: basis states are decoded into
// (exciton site, occupation list) tuples, edited as tuples and re-packed;
// sets are sorted key vectors with binary search; H_eff is CSR; the
// propagator is a shifted Taylor series.
//
// Paper passages followed (cited by section / equation):
//   model         Eqs. (tb), (holstein), extended to square and cubic lattices
//                 as in Sec. "Application to vibronic nanoaggregates".
//   neighbours    Eqs. (def_neighbor), (def_neighbor_k), (H_eff).
//   truncation    Sec. "Truncation & post-adaptation detruncation".
//   assembly      Sec. "Generating the effective Hamiltonian from the
//                 effective Hilbert space".
//   step          Sec. "Formal operator representation and notes on
//                 parallelization": psi -> Q exp(-i P H P dt) psi.
//   propagator    App. "The action of the exponential of a sparse matrix";
//                 the Krylov alternative of App. "Series-based
//                 exponentiation compared to a Lanczos algorithm".
//   key codec     App. "Lossless bit-level compression of state information".
//   observables   Eq. (RMSD) populations; Eq. (init_state_spec) overlap.
//
// Where the paper leaves a choice open the reading taken is stated at the
// point of use.
#include "paces_oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include <omp.h>

namespace {

using cplx = std::complex<double>;
thread_local std::string g_err;

int fail(const std::string& msg) {
  g_err = msg;
  return 1;
}

// ---------------------------------------------------------------------------
// Bit-field codec (App. "Lossless bit-level compression of state
// information").  A key is a B-bit unsigned integer held in W 64-bit words,
// word 0 most significant.  Fields are listed most significant first and
// packed without gaps, so the last field occupies the lowest bits.  A field
// may straddle a word boundary; bits are moved one at a time so that no
// special case is needed.
// ---------------------------------------------------------------------------
void set_bit(uint64_t* key, int W, int pos) {
  key[W - 1 - pos / 64] |= (uint64_t(1) << (pos % 64));
}
int get_bit(const uint64_t* key, int W, int pos) {
  return int((key[W - 1 - pos / 64] >> (pos % 64)) & 1u);
}

// offsets[f] = bit position (from the least significant end) of field f.
void pack_bits(int nf, const int* widths, const int* offsets,
               const uint64_t* values, int W, uint64_t* out) {
  for (int w = 0; w < W; ++w) out[w] = 0;
  for (int f = 0; f < nf; ++f)
    for (int b = 0; b < widths[f]; ++b)
      if ((values[f] >> b) & 1u) set_bit(out, W, offsets[f] + b);
}

uint64_t get_field(const uint64_t* key, int W, int off, int width) {
  uint64_t v = 0;
  for (int b = 0; b < width; ++b)
    v |= uint64_t(get_bit(key, W, off + b)) << b;
  return v;
}

int bits_for(int count) {  // smallest b with 2^b >= count
  int b = 0;
  while ((int64_t(1) << b) < count) ++b;
  return b;
}

// ---------------------------------------------------------------------------
// Model: Eq. (holstein) on a lattice.  Sites are numbered row-major,
// i = x + Lx*(y + Ly*z).  Each site carries V modes with cutoffs c_nu.
// ---------------------------------------------------------------------------
struct Model {
  int ndim = 1, ext[3] = {1, 1, 1}, per[3] = {0, 0, 0};
  int N = 1, V = 1, cut[4] = {0, 0, 0, 0};
  double omega[4] = {0, 0, 0, 0}, g[4] = {0, 0, 0, 0}, J[3] = {0, 0, 0};
  std::vector<double> eps;
  // Key layout (reading of the compression appendix for this model):
  // fields most significant first n_{0,0}..n_{0,V-1}, n_{1,0}, ...,
  // n_{N-1,V-1}, then the exciton site j in the lowest bits.
  int bnu[4] = {0, 0, 0, 0}, bj = 1, B = 0, W = 1, D = 0;
  std::vector<int> nbr;  // [N][2*ndim]: +1 then -1 neighbour per axis, -1 none
  std::vector<int> widths, offsets;  // per field, field order as above

  int nfields() const { return N * V + 1; }
  int slot_count() const { return 2 * ndim + 2 * V; }
};

struct State {  // decoded basis state
  int j = 0;
  std::vector<int> n;  // [N*V], site-major
};

void encode(const Model& m, const State& s, uint64_t* key) {
  std::vector<uint64_t> vals(m.nfields());
  for (int f = 0; f < m.N * m.V; ++f) vals[f] = uint64_t(s.n[f]);
  vals[m.N * m.V] = uint64_t(s.j);
  pack_bits(m.nfields(), m.widths.data(), m.offsets.data(), vals.data(), m.W,
            key);
}

void decode(const Model& m, const uint64_t* key, State& s) {
  s.n.assign(m.N * m.V, 0);
  for (int f = 0; f < m.N * m.V; ++f)
    s.n[f] = int(get_field(key, m.W, m.offsets[f], m.widths[f]));
  s.j = int(get_field(key, m.W, m.offsets[m.N * m.V], m.widths[m.N * m.V]));
}

// Diagonal element eps_j + sum_nu omega_nu * T_nu with T_nu the total
// occupation of mode nu (Eq. (holstein); no zero-point term), evaluated in
// this order.
double diagonal(const Model& m, const State& s) {
  double d = m.eps[s.j];
  for (int nu = 0; nu < m.V; ++nu) {
    long T = 0;
    for (int i = 0; i < m.N; ++i) T += s.n[i * m.V + nu];
    d = d + m.omega[nu] * double(T);
  }
  return d;
}

// The D off-diagonal slots of a row, in a fixed order: for each axis the +1
// hop then the -1 hop, then for each mode the lowering then the raising
// term at the exciton site.  A slot exists iff its matrix element is
// structurally nonzero (reading of Eq. (def_neighbor): "nonzero" is taken
// structurally, so that the set does not depend on rounding).
struct Slot {
  bool exists = false;
  State s;
  double val = 0;
};

void slots_of(const Model& m, const State& s, std::vector<Slot>& out) {
  out.assign(m.slot_count(), Slot());
  int q = 0;
  for (int a = 0; a < m.ndim; ++a)
    for (int dir = 0; dir < 2; ++dir, ++q) {
      int jn = m.nbr[s.j * 2 * m.ndim + 2 * a + dir];
      if (jn < 0 || m.J[a] == 0.0) continue;
      out[q].exists = true;
      out[q].s = s;
      out[q].s.j = jn;
      out[q].val = m.J[a];  // Eq. (tb): J |j><j+1| + h.c.
    }
  for (int nu = 0; nu < m.V; ++nu) {
    int n = s.n[s.j * m.V + nu];
    // lowering: <n-1| a |n> = sqrt(n)
    if (m.g[nu] != 0.0 && n > 0) {
      out[q].exists = true;
      out[q].s = s;
      out[q].s.n[s.j * m.V + nu] = n - 1;
      out[q].val = m.g[nu] * std::sqrt(double(n));
    }
    ++q;
    // raising: <n+1| a^dag |n> = sqrt(n+1)
    if (m.g[nu] != 0.0 && n < m.cut[nu]) {
      out[q].exists = true;
      out[q].s = s;
      out[q].s.n[s.j * m.V + nu] = n + 1;
      out[q].val = m.g[nu] * std::sqrt(double(n + 1));
    }
    ++q;
  }
}

// ---------------------------------------------------------------------------
// Key sets: flat arrays of W-word keys, compared as B-bit integers.
// ---------------------------------------------------------------------------
struct Keys {
  int W = 1;
  std::vector<uint64_t> d;
  int64_t size() const { return int64_t(d.size()) / W; }
  const uint64_t* at(int64_t i) const { return d.data() + i * W; }
  void push(const uint64_t* k) { d.insert(d.end(), k, k + W); }
};

bool key_less(const uint64_t* a, const uint64_t* b, int W) {
  for (int w = 0; w < W; ++w)
    if (a[w] != b[w]) return a[w] < b[w];
  return false;
}
bool key_eq(const uint64_t* a, const uint64_t* b, int W) {
  for (int w = 0; w < W; ++w)
    if (a[w] != b[w]) return false;
  return true;
}

// Sorted permutation of k.
std::vector<int64_t> sort_order(const Keys& k) {
  std::vector<int64_t> idx(k.size());
  for (int64_t i = 0; i < k.size(); ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return key_less(k.at(a), k.at(b), k.W);
  });
  return idx;
}

Keys sort_unique(const Keys& k) {
  std::vector<int64_t> idx = sort_order(k);
  Keys out;
  out.W = k.W;
  for (int64_t i = 0; i < int64_t(idx.size()); ++i)
    if (i == 0 || !key_eq(k.at(idx[i]), k.at(idx[i - 1]), k.W))
      out.push(k.at(idx[i]));
  return out;
}

int64_t find_key(const Keys& sorted, const uint64_t* key) {
  int64_t lo = 0, hi = sorted.size();
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (key_less(sorted.at(mid), key, sorted.W))
      lo = mid + 1;
    else
      hi = mid;
  }
  if (lo < sorted.size() && key_eq(sorted.at(lo), key, sorted.W)) return lo;
  return -1;
}

// Elements of sorted a that are not in sorted b.
Keys set_minus(const Keys& a, const Keys& b) {
  Keys out;
  out.W = a.W;
  for (int64_t i = 0; i < a.size(); ++i)
    if (find_key(b, a.at(i)) < 0) out.push(a.at(i));
  return out;
}

Keys set_union(const Keys& a, const Keys& b) {
  Keys all;
  all.W = a.W;
  all.d = a.d;
  all.d.insert(all.d.end(), b.d.begin(), b.d.end());
  return sort_unique(all);
}

// ---------------------------------------------------------------------------
// Neighbour ball: union over r = 0..k of N^(r)_M (Eqs. (def_neighbor_k),
// (H_eff)) computed breadth first.  frontier[r] holds the states at graph
// distance exactly r from M, so frontier[0] = M.
// ---------------------------------------------------------------------------
void expand(const Model& m, const Keys& M, int k, Keys& ball,
            std::vector<Keys>& frontier) {
  frontier.clear();
  frontier.push_back(M);
  ball = M;
  const int D = m.slot_count(), W = m.W;
  for (int r = 1; r <= k; ++r) {
    const Keys& F = frontier.back();
    Keys cand;
    cand.W = W;
    std::vector<uint64_t> buf(size_t(F.size()) * D * W, 0);
    std::vector<uint8_t> ex(size_t(F.size()) * D, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < F.size(); ++i) {
      State s;
      std::vector<Slot> sl;
      decode(m, F.at(i), s);
      slots_of(m, s, sl);
      for (int q = 0; q < D; ++q)
        if (sl[q].exists) {
          ex[i * D + q] = 1;
          encode(m, sl[q].s, &buf[(size_t(i) * D + q) * W]);
        }
    }
    for (int64_t c = 0; c < int64_t(ex.size()); ++c)
      if (ex[c]) cand.push(&buf[size_t(c) * W]);
    Keys fresh = set_minus(sort_unique(cand), ball);
    ball = set_union(ball, fresh);
    frontier.push_back(fresh);
  }
}

// ---------------------------------------------------------------------------
// Effective Hamiltonian over a sorted set (Sec. "Generating the effective
// Hamiltonian from the effective Hilbert space"): every row gets its
// diagonal and one entry per existing slot whose target lies in the set.
// Distinct slots of a row lead to distinct states, so no entry is
// duplicated.  Columns are sorted within a row.
// ---------------------------------------------------------------------------
struct CSR {
  int64_t n = 0;
  std::vector<int64_t> rowptr, cols;
  std::vector<double> vals;
  double emin = 0, emax = 0;  // Gershgorin bounds of the spectrum
};

void build_csr(const Model& m, const Keys& S, CSR& H) {
  const int D = m.slot_count();
  const int64_t n = S.size();
  H.n = n;
  std::vector<std::vector<std::pair<int64_t, double>>> rows(n);
  std::vector<double> lo(n), hi(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    State s;
    std::vector<Slot> sl;
    std::vector<uint64_t> key(m.W);
    decode(m, S.at(i), s);
    slots_of(m, s, sl);
    const double d = diagonal(m, s);
    rows[i].push_back({i, d});
    double radius = 0;
    for (int q = 0; q < D; ++q) {
      if (!sl[q].exists) continue;
      encode(m, sl[q].s, key.data());
      int64_t c = find_key(S, key.data());
      if (c < 0) continue;
      rows[i].push_back({c, sl[q].val});
      radius = radius + std::fabs(sl[q].val);
    }
    std::sort(rows[i].begin(), rows[i].end());
    lo[i] = d - radius;
    hi[i] = d + radius;
  }
  H.rowptr.assign(n + 1, 0);
  H.cols.clear();
  H.vals.clear();
  for (int64_t i = 0; i < n; ++i) {
    for (auto& e : rows[i]) {
      H.cols.push_back(e.first);
      H.vals.push_back(e.second);
    }
    H.rowptr[i + 1] = int64_t(H.cols.size());
  }
  // Gershgorin interval, widened by 1e-12 of its magnitude so that it
  // strictly contains the spectrum (reading: the paper names no bound).
  double emin = n ? lo[0] : 0.0, emax = n ? hi[0] : 0.0;
  for (int64_t i = 1; i < n; ++i) {
    emin = std::min(emin, lo[i]);
    emax = std::max(emax, hi[i]);
  }
  const double pad = 1e-12 * (std::fabs(emax) + std::fabs(emin));
  H.emin = emin - pad;
  H.emax = emax + pad;
}

void spmv(const CSR& H, const std::vector<cplx>& x, std::vector<cplx>& y) {
  y.assign(H.n, cplx(0, 0));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < H.n; ++i) {
    cplx acc(0, 0);
    for (int64_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e)
      acc += H.vals[e] * x[H.cols[e]];
    y[i] = acc;
  }
}

double inf_norm(const std::vector<cplx>& v) {
  double r = 0;
  for (const cplx& z : v) r = std::max(r, std::abs(z));
  return r;
}

// ---------------------------------------------------------------------------
// exp(-i H dt) v by the Taylor series of App. "The action of the exponential
// of a sparse matrix", applied term by term to the vector.  Two choices the
// paper leaves open (it names only "a convergence criterion" and the
// scaling of Al-Mohy & Higham):
//   * H is shifted by sigma = (emax + emin)/2 and the step is split into
//     ceil(a dt) substeps when a dt > 1, a = (emax - emin)/2, so that every
//     substep's series converges fast;
//   * a substep stops after the first term n with |term_n|_inf <=
//     2^-60 |acc|_inf and |term_{n-1}|_inf <= 2^-50 |acc|_inf.
// ---------------------------------------------------------------------------
int expmv(const CSR& H, double dt, int max_terms, const std::vector<cplx>& v,
          std::vector<cplx>& out, int& terms) {
  const double sigma = 0.5 * (H.emax + H.emin);
  const double a = 0.5 * (H.emax - H.emin);
  int nsub = int(std::ceil(a * dt));
  if (nsub < 1) nsub = 1;
  const double h = dt / nsub;
  std::vector<cplx> w = v, term, prev, y;
  terms = 0;
  for (int sub = 0; sub < nsub; ++sub) {
    std::vector<cplx> acc = w;
    term = w;
    for (int n = 1;; ++n) {
      if (n > max_terms)
        return fail("Taylor series did not converge within max_terms");
      prev = term;
      spmv(H, term, y);
      const cplx f(0.0, -h / n);
      for (int64_t i = 0; i < H.n; ++i) {
        term[i] = (y[i] - sigma * prev[i]) * f;
        acc[i] += term[i];
      }
      ++terms;
      const double an = inf_norm(acc);
      if (inf_norm(term) <= std::ldexp(an, -60) &&
          inf_norm(prev) <= std::ldexp(an, -50))
        break;
    }
    w = acc;
  }
  const cplx phase = std::exp(cplx(0.0, -sigma * dt));
  out.resize(H.n);
  for (int64_t i = 0; i < H.n; ++i) out[i] = phase * w[i];
  return 0;
}

// |c|^2 evaluated as fl(fl(re*re) + fl(im*im)); the build disables FMA
// contraction so the threshold decision is reproducible.
double weight(const cplx& c) {
  const double a = c.real() * c.real();
  const double b = c.imag() * c.imag();
  return a + b;
}

// ---------------------------------------------------------------------------
// Eigen-decomposition of a symmetric n x n matrix by cyclic Jacobi
// rotations (Golub & Van Loan, "Matrix Computations", the symmetric Schur
// decomposition and the cyclic Jacobi method).  a is row-major and is
// overwritten; on return its diagonal holds the eigenvalues and the columns
// of q the eigenvectors.
// ---------------------------------------------------------------------------
void jacobi_eigen(int n, std::vector<double>& a, std::vector<double>& q) {
  q.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) q[size_t(i) * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, all = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = a[size_t(i) * n + j] * a[size_t(i) * n + j];
        all += v;
        if (i != j) off += v;
      }
    if (off == 0.0 || off <= 1e-36 * all) break;
    for (int p = 0; p < n; ++p)
      for (int r = p + 1; r < n; ++r) {
        const double apr = a[size_t(p) * n + r];
        if (apr == 0.0) continue;
        // rotation J with J_pp = J_rr = c, J_pr = s, J_rp = -s that zeroes
        // the (p, r) entry of J^T A J
        const double tau = (a[size_t(r) * n + r] - a[size_t(p) * n + p]) / (2 * apr);
        const double t = (tau >= 0 ? 1.0 : -1.0) /
                         (std::fabs(tau) + std::sqrt(tau * tau + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A J: columns p and r
          const double akp = a[size_t(k) * n + p], akr = a[size_t(k) * n + r];
          a[size_t(k) * n + p] = c * akp - s * akr;
          a[size_t(k) * n + r] = s * akp + c * akr;
        }
        for (int k = 0; k < n; ++k) {  // J^T (A J): rows p and r
          const double apk = a[size_t(p) * n + k], ark = a[size_t(r) * n + k];
          a[size_t(p) * n + k] = c * apk - s * ark;
          a[size_t(r) * n + k] = s * apk + c * ark;
        }
        for (int k = 0; k < n; ++k) {  // Q J
          const double qkp = q[size_t(k) * n + p], qkr = q[size_t(k) * n + r];
          q[size_t(k) * n + p] = c * qkp - s * qkr;
          q[size_t(k) * n + r] = s * qkp + c * qkr;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Truncated Taylor propagator with the degree and substep choice of Al-Mohy
// & Higham ("Computing the action of the matrix exponential", SIAM J. Sci.
// Comput. 33, 2011), the method App. "The action of the exponential of a
// sparse matrix" names, and the fixed-order series of App. "An effective
// Hilbert space up to neighbor order m = 2 is not equivalent to a
// second-order Taylor expansion".
//
// Backward-error threshold theta_m: with T_m the degree-m Taylor polynomial
// of exp, exp(-x) T_m(x) = exp(h(x)), h(x) = sum_{k > m} c_k x^k, and
// theta_m = max { theta : sum_k |c_k| theta^(k-1) <= 2^-53 }.  The c_k come
// from the power series of g = exp(-x) T_m(x) (g_0 = 1, g_1..g_m = 0) by
// the logarithm recurrence k h_k = k g_k - sum_{j<k} j h_j g_(k-j), kept to
// degree m + 120 in long double; theta by bisection.
//
// Readings where the method leaves a choice: A = -i (H - b) dt with b the
// centre of the padded Gershgorin interval and ||A|| bounded by its half
// width a times dt (the bound every norm estimate of the method may be
// replaced by); (m, s) = argmin over m = 1..55 of m * max(1, ceil(a dt /
// theta_m)), the smallest m on ties; no early termination of the series.
// Fixed order N: one substep of N terms.  The result carries exp(-i b dt).
// ---------------------------------------------------------------------------
constexpr int kTaylorMaxDeg = 55;

double taylor_theta(int m) {
  const int M = m + 121;
  std::vector<long double> g(M + 1, 0.0L), h(M + 1, 0.0L);
  for (int k = 0; k <= M; ++k) {
    long double sum = 0;
    for (int j = 0; j <= std::min(k, m); ++j) {
      long double t = 1;  // (-1)^(k-j) / ((k-j)! j!)
      for (int q = 1; q <= k - j; ++q) t /= q;
      for (int q = 1; q <= j; ++q) t /= q;
      sum += ((k - j) & 1) ? -t : t;
    }
    g[k] = k == 0 ? 1.0L : (k <= m ? 0.0L : sum);
  }
  for (int k = 1; k <= M; ++k) {
    long double acc = 0;
    for (int j = 1; j < k; ++j) acc += j * h[j] * g[k - j];
    h[k] = g[k] - acc / k;
  }
  const long double tol = std::ldexp(1.0L, -53);
  auto excess = [&](long double th) {
    long double sum = 0, p = 1;  // p = th^(k-1)
    for (int k = 1; k <= M; ++k) {
      if (k > m) sum += std::fabs(h[k]) * p;
      p *= th;
    }
    return sum - tol;
  };
  long double lo = 0, hi = 1;
  while (excess(hi) < 0) hi *= 2;
  for (int it = 0; it < 200; ++it) {
    const long double mid = 0.5L * (lo + hi);
    if (excess(mid) < 0) lo = mid; else hi = mid;
  }
  return double(lo);
}

const std::vector<double>& taylor_thetas() {
  static const std::vector<double> t = [] {
    std::vector<double> v(kTaylorMaxDeg + 1, 0.0);
    for (int m = 1; m <= kTaylorMaxDeg; ++m) v[m] = taylor_theta(m);
    return v;
  }();
  return t;
}

void taylor_select(double norm, int& m_out, int& s_out) {
  const std::vector<double>& th = taylor_thetas();
  double best = INFINITY;
  m_out = 1;
  s_out = 1;
  for (int m = 1; m <= kTaylorMaxDeg; ++m) {
    const double sd = std::max(1.0, std::ceil(norm / th[m]));
    if (m * sd < best) {
      best = m * sd;
      m_out = m;
      s_out = int(sd);
    }
  }
}

// order > 0: fixed order, one substep; order < 0: (m, s) chosen as above.
int taylor_expmv(const CSR& H, double dt, int order,
                 const std::vector<cplx>& v, std::vector<cplx>& out,
                 int& mvs) {
  const double b = 0.5 * (H.emax + H.emin), a = 0.5 * (H.emax - H.emin);
  int m = order, s = 1;
  if (order <= 0) taylor_select(a * dt, m, s);
  std::vector<cplx> f = v, term, y;
  mvs = 0;
  for (int sub = 0; sub < s; ++sub) {
    term = f;
    std::vector<cplx> acc = f;
    for (int j = 1; j <= m; ++j) {
      spmv(H, term, y);
      const cplx fac(0.0, -dt / (double(s) * j));
      for (int64_t i = 0; i < H.n; ++i) {
        term[i] = fac * (y[i] - b * term[i]);
        acc[i] += term[i];
      }
      ++mvs;
    }
    f = acc;
  }
  const cplx phase = std::exp(cplx(0.0, -b * dt));
  out.resize(H.n);
  for (int64_t i = 0; i < H.n; ++i) out[i] = phase * f[i];
  return 0;
}

// ---------------------------------------------------------------------------
// Krylov (Lanczos) propagator of App. "Series-based exponentiation compared
// to a Lanczos algorithm": exp(-i H dt) v ~ V exp(-i T dt) V^dag v, V an
// orthonormal basis of the Krylov space span{v, Hv, .., H^p v} and
// T = V^dag H V tridiagonal.  Order p in the paper's sense: the order-2
// propagator works in span{v, Hv, H^2 v}, so the space has p + 1
// dimensions.  The basis comes from the three-term recurrence
//   v_0 = v / beta_0, beta_0 = |v|,
//   alpha_j = <v_j|H|v_j>,
//   r = H v_j - alpha_j v_j - beta_j v_{j-1},  beta_{j+1} = |r|,
//   v_{j+1} = r / beta_{j+1}.
// Readings where the paper is silent:
//   * the basis stops early (breakdown: the space is invariant, so the
//     result is exact) when beta_{j+1} <= 1e-11 |H v_j|; beta_0 = 0 gives
//     the zero vector and dimension 0;
//   * no re-orthogonalisation, as in the plain recurrence.
// With V^dag v = beta_0 e_1 the result is beta_0 sum_j u_j v_j where
// u = exp(-i T dt) e_1 = Q exp(-i L dt) Q^T e_1 from the eigen-
// decomposition T = Q L Q^T.  e_lo / e_hi: Gershgorin interval of T,
// widened by 1e-12 of its magnitude like that of H.
// ---------------------------------------------------------------------------
struct KrylovOut {
  int dim = 0;
  std::vector<std::vector<cplx>> V;
  std::vector<double> alpha, beta;  // beta[0] = |v|; beta[j] couples j-1, j
  double e_lo = 0, e_hi = 0;
};

int lanczos_expmv(const CSR& H, double dt, int order,
                  const std::vector<cplx>& v, std::vector<cplx>& out,
                  KrylovOut& ko) {
  if (order < 1) return fail("Krylov order must be at least 1");
  const int nmax = order + 1;
  ko = KrylovOut();
  double b0 = 0;
  for (const cplx& c : v) b0 += weight(c);
  b0 = std::sqrt(b0);
  ko.beta.push_back(b0);
  out.assign(H.n, cplx(0, 0));
  if (b0 == 0.0) return 0;
  std::vector<cplx> v0(H.n), hv, r(H.n);
  for (int64_t i = 0; i < H.n; ++i) v0[i] = v[i] / b0;
  ko.V.push_back(v0);
  for (int j = 0; j < nmax; ++j) {
    const std::vector<cplx>& vj = ko.V[j];
    spmv(H, vj, hv);
    double a = 0;
    for (int64_t i = 0; i < H.n; ++i) a += (std::conj(vj[i]) * hv[i]).real();
    ko.alpha.push_back(a);
    if (j + 1 == nmax) break;
    double rn = 0, hn = 0;
    for (int64_t i = 0; i < H.n; ++i) {
      r[i] = hv[i] - a * vj[i];
      if (j > 0) r[i] -= ko.beta[j] * ko.V[j - 1][i];
      rn += weight(r[i]);
      hn += weight(hv[i]);
    }
    if (rn <= 1e-22 * hn) break;  // invariant subspace
    const double b = std::sqrt(rn);
    ko.beta.push_back(b);
    std::vector<cplx> next(H.n);
    for (int64_t i = 0; i < H.n; ++i) next[i] = r[i] / b;
    ko.V.push_back(next);
  }
  const int n = int(ko.alpha.size());
  ko.dim = n;
  std::vector<double> T(size_t(n) * n, 0.0), Q;
  double lo = 0, hi = 0;
  for (int j = 0; j < n; ++j) {
    T[size_t(j) * n + j] = ko.alpha[j];
    double rad = 0;
    if (j > 0) {
      T[size_t(j) * n + j - 1] = T[size_t(j - 1) * n + j] = ko.beta[j];
      rad += std::fabs(ko.beta[j]);
    }
    if (j + 1 < n) rad += std::fabs(ko.beta[j + 1]);
    const double l = ko.alpha[j] - rad, h = ko.alpha[j] + rad;
    lo = j == 0 ? l : std::min(lo, l);
    hi = j == 0 ? h : std::max(hi, h);
  }
  const double pad = 1e-12 * (std::fabs(hi) + std::fabs(lo));
  ko.e_lo = lo - pad;
  ko.e_hi = hi + pad;
  jacobi_eigen(n, T, Q);
  for (int j = 0; j < n; ++j) {
    cplx u(0, 0);
    for (int k = 0; k < n; ++k)
      u += Q[size_t(j) * n + k] * std::exp(cplx(0.0, -T[size_t(k) * n + k] * dt)) *
           Q[size_t(k)];
    for (int64_t i = 0; i < H.n; ++i) out[i] += b0 * u * ko.V[j][i];
  }
  return 0;
}

struct Obs {
  double f[ORC_OBS_NFIELDS];
  std::vector<double> pop;
};

struct Params {
  double dt = 0.01, theta = 0;
  int k = 2, k_init = 2, max_terms = 200;
  int64_t max_states = 0;  // cap on |S| (0 = none)
  int64_t q_nom = 0;       // fixed-size truncation (0 = threshold)
  int krylov_order = 0;    // > 0: Lanczos propagator of this order
  int taylor_order = 0;    // -1: Taylor with (m, s) chosen; N > 0: N terms
};

// ---------------------------------------------------------------------------
// State cap (reading of the cube4 workload's "capped by the HBM budget";
// the paper itself keeps a fixed number q_nom of the largest amplitudes,
// Sec. "Truncation & post-adaptation detruncation", with a pseudo-random
// tie-break against ordering bias).  When the ball of M exceeds the cap,
// M is cut to its q heaviest rows, ordered by weight descending, then by a
// splitmix64 hash of the key ascending, then by the key ascending, with
// q = floor(cap * |M_prev| / |S_prev|) (q = floor(cap / (D+1)) on the first
// step or after an empty M) and, while the ball of the cut set still
// exceeds the cap, q <- floor(9 min(q, |M|) cap / (10 |ball|)).
// ---------------------------------------------------------------------------

// splitmix64 output function (Steele, Lea & Flood 2014) of a 64-bit value.
uint64_t splitmix_mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Tie-break hash of a canonical key: h = mix(h ^ word) over the words,
// most significant first, from h = 0.
uint64_t tiebreak_hash(const uint64_t* key, int W) {
  uint64_t h = 0;
  for (int w = 0; w < W; ++w) h = splitmix_mix(h ^ key[w]);
  return h;
}

struct Sim {
  const Model* m = nullptr;
  Params p;
  Keys S;                    // sorted current set
  std::vector<cplx> psi;     // amplitudes aligned with S
  Keys psi0_keys;            // sorted support of the initial state
  std::vector<cplx> psi0;
  int64_t steps = 0;
  double t = 0, mass_total = 0;
  bool fresh = true;         // next step is the first after init
  int64_t prev_nS = 0, prev_nM = 0;  // counts of the last step (cap rule)
  // last step
  Keys M;
  std::vector<Keys> frontier;
  std::vector<cplx> phi;
  CSR H;
  std::vector<Obs> obs;
};

// One step of Sec. "Formal operator representation and notes on
// parallelization", with truncation placed before re-growth as in Sec.
// "Truncation & post-adaptation detruncation":
//   select M from psi (first step: all input states, order k_init; the
//   paper grows the initial space with its own order m_init),
//   S' = ball of radius k around M,
//   phi = psi on S' (states of S outside S' are discarded, their weight
//   is the step's discarded mass),
//   psi' = exp(-i H_S' dt) phi.
int sim_step(Sim& sim) {
  const Model& m = *sim.m;
  // select (threshold on |c|, as |c|^2 >= theta^2 in FP64)
  Keys M;
  M.W = m.W;
  int k = sim.p.k;
  if (sim.fresh) {
    M = sim.S;
    k = sim.p.k_init;
  } else if (sim.p.q_nom > 0) {
    // the paper's fixed-size truncation: the q_nom heaviest rows, ties by
    // the splitmix64 key hash, then the key
    std::vector<int64_t> order(sim.S.size());
    std::vector<double> w(sim.S.size());
    std::vector<uint64_t> hs(sim.S.size());
    for (int64_t i = 0; i < sim.S.size(); ++i) {
      order[i] = i;
      w[i] = weight(sim.psi[i]);
      hs[i] = tiebreak_hash(sim.S.at(i), m.W);
    }
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      if (w[a] != w[b]) return w[a] > w[b];
      if (hs[a] != hs[b]) return hs[a] < hs[b];
      return a < b;  // S is sorted: row order is key order
    });
    const int64_t q = std::min<int64_t>(sim.p.q_nom, sim.S.size());
    std::sort(order.begin(), order.begin() + q);
    for (int64_t i = 0; i < q; ++i) M.push(sim.S.at(order[i]));
  } else {
    const double th2 = sim.p.theta * sim.p.theta;
    for (int64_t i = 0; i < sim.S.size(); ++i)
      if (weight(sim.psi[i]) >= th2) M.push(sim.S.at(i));
  }
  Keys ball;
  std::vector<Keys> frontier;
  expand(m, M, k, ball, frontier);
  const int64_t cap = sim.p.max_states;
  if (cap > 0 && ball.size() > cap) {
    // order M by (weight desc, tie-break hash asc, key asc)
    std::vector<int64_t> order(M.size());
    std::vector<double> wM(M.size());
    std::vector<uint64_t> hM(M.size());
    for (int64_t i = 0; i < M.size(); ++i) {
      order[i] = i;
      wM[i] = weight(sim.psi[find_key(sim.S, M.at(i))]);
      hM[i] = tiebreak_hash(M.at(i), m.W);
    }
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      if (wM[a] != wM[b]) return wM[a] > wM[b];
      if (hM[a] != hM[b]) return hM[a] < hM[b];
      return key_less(M.at(a), M.at(b), m.W);
    });
    const int64_t nMfull = M.size();
    int64_t q = (sim.fresh || sim.prev_nM == 0 || sim.prev_nS == 0)
                    ? cap / (m.slot_count() + 1)
                    : cap * sim.prev_nM / sim.prev_nS;
    for (;;) {
      const int64_t qe = std::min(q, nMfull);
      Keys cut;
      cut.W = m.W;
      for (int64_t i = 0; i < qe; ++i) cut.push(M.at(order[i]));
      Keys Mq = sort_unique(cut);
      expand(m, Mq, k, ball, frontier);
      if (ball.size() <= cap) {
        M = Mq;
        break;
      }
      q = 9 * qe * cap / (10 * ball.size());
    }
  }
  // transfer: post-adaptation detruncation
  std::vector<cplx> phi(ball.size(), cplx(0, 0));
  double mass = 0;
  for (int64_t i = 0; i < sim.S.size(); ++i) {
    int64_t r = find_key(ball, sim.S.at(i));
    if (r >= 0)
      phi[r] = sim.psi[i];
    else
      mass += weight(sim.psi[i]);
  }
  CSR H;
  build_csr(m, ball, H);
  std::vector<cplx> out;
  int terms = 0;
  double e_lo = H.emin, e_hi = H.emax;
  if (sim.p.taylor_order != 0) {
    if (taylor_expmv(H, sim.p.dt, sim.p.taylor_order, phi, out, terms))
      return 1;
  } else if (sim.p.krylov_order > 0) {
    KrylovOut ko;
    if (lanczos_expmv(H, sim.p.dt, sim.p.krylov_order, phi, out, ko)) return 1;
    terms = ko.dim;
    e_lo = ko.e_lo;
    e_hi = ko.e_hi;
  } else if (expmv(H, sim.p.dt, sim.p.max_terms, phi, out, terms)) {
    return 1;
  }
  sim.S = ball;
  sim.psi = out;
  sim.M = M;
  sim.frontier = frontier;
  sim.phi = phi;
  sim.H = H;
  sim.steps += 1;
  sim.t = sim.t + sim.p.dt;
  sim.mass_total += mass;
  sim.fresh = false;
  sim.prev_nS = ball.size();
  sim.prev_nM = M.size();
  // observables at the new time
  Obs o;
  o.pop.assign(m.N, 0.0);
  std::vector<cplx> hp;
  spmv(H, out, hp);
  double n2 = 0, en = 0;
  for (int64_t i = 0; i < H.n; ++i) {
    n2 += weight(out[i]);
    en += (std::conj(out[i]) * hp[i]).real();
    State s;
    decode(m, ball.at(i), s);
    o.pop[s.j] += weight(out[i]);
  }
  cplx a(0, 0);  // <psi0|psi(t)>, Eq. (init_state_spec) and below
  for (int64_t i = 0; i < sim.psi0_keys.size(); ++i) {
    int64_t r = find_key(ball, sim.psi0_keys.at(i));
    if (r >= 0) a += std::conj(sim.psi0[i]) * out[r];
  }
  o.f[ORC_OBS_T] = sim.t;
  o.f[ORC_OBS_NORM2] = n2;
  o.f[ORC_OBS_ENERGY] = en;
  o.f[ORC_OBS_A_RE] = a.real();
  o.f[ORC_OBS_A_IM] = a.imag();
  o.f[ORC_OBS_MASS_STEP] = mass;
  o.f[ORC_OBS_MASS_TOTAL] = sim.mass_total;
  o.f[ORC_OBS_NS] = double(ball.size());
  o.f[ORC_OBS_NM] = double(M.size());
  o.f[ORC_OBS_TERMS] = double(terms);
  o.f[ORC_OBS_EMIN] = e_lo;
  o.f[ORC_OBS_EMAX] = e_hi;
  sim.obs.push_back(o);
  return 0;
}

int load_state(const Model& m, int64_t n, const uint64_t* keys,
               const double* amps, Keys& S, std::vector<cplx>& psi) {
  Keys k;
  k.W = m.W;
  k.d.assign(keys, keys + n * m.W);
  std::vector<int64_t> idx = sort_order(k);
  S.W = m.W;
  S.d.clear();
  psi.clear();
  for (int64_t i = 0; i < n; ++i) {
    if (i > 0 && key_eq(k.at(idx[i]), k.at(idx[i - 1]), m.W))
      return fail("duplicate basis state in the input");
    S.push(k.at(idx[i]));
    psi.push_back(cplx(amps[2 * idx[i]], amps[2 * idx[i] + 1]));
  }
  return 0;
}

int check_keys(const Model& m, int64_t n, const uint64_t* keys) {
  // every field must decode to a valid value and no bit above B may be set
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t* k = keys + i * m.W;
    for (int pos = m.B; pos < 64 * m.W; ++pos)
      if (get_bit(k, m.W, pos)) return fail("key has bits above B set");
    State s;
    decode(m, k, s);
    if (s.j >= m.N) return fail("exciton site out of range");
    for (int f = 0; f < m.N * m.V; ++f)
      if (s.n[f] > m.cut[f % m.V]) return fail("occupation above cutoff");
  }
  return 0;
}


// ---------------------------------------------------------------------------
// Gradient of a loss of the autocorrelation (Form (3); the paper has no
// adjoint).  The sets S_0 (support of psi0), S_1, .., S_n of a recorded run
// are held fixed, and every step is the linear map
//     psi_{s+1} = U_s T_s psi_s,   U_s = exp(-i H_{s+1} dt) on S_{s+1},
// with T_s the restriction from S_s to S_{s+1} (post-adaptation
// detruncation).  For a real loss L of a_s = <psi0|psi_s> with
// gbar_s = dL/d conj(a_s), the discrete adjoint
//     lambda_n = gbar_n psi0,
//     lambda_s = T_s^T U_s^dag lambda_{s+1} + gbar_s psi0
// gives  dL/dtheta_p = sum_s 2 Re <lambda_{s+1} | (dU_s/dtheta_p) T_s psi_s>.
// H is linear in theta = (J_axis, g_nu, omega_nu, eps_n) (Eq. (holstein));
// dU/dtheta_p v is the Frechet derivative of exp at A = -i H dt in the
// direction E = -i dt dH/dtheta_p, the top block of
// exp([[A, E], [0, A]]) [0; v] (Van Loan 1978), evaluated with the same
// Taylor routine on the doubled system.
// ---------------------------------------------------------------------------

// Matrix elements of dH/dtheta_p between s and the states it couples to.
// Edges count whenever the lattice has them, whatever the parameter's
// value, so the derivative also exists at a parameter equal to zero.
void dH_entries(const Model& m, const State& s, int p,
                std::vector<std::pair<State, double>>& out) {
  out.clear();
  const int nJ = m.ndim, nG = m.V, nW = m.V;
  if (p < nJ) {  // J along axis p: 1 on both hops of that axis
    for (int dir = 0; dir < 2; ++dir) {
      const int jn = m.nbr[s.j * 2 * m.ndim + 2 * p + dir];
      if (jn < 0) continue;
      State t = s;
      t.j = jn;
      out.push_back({t, 1.0});
    }
    return;
  }
  p -= nJ;
  if (p < nG) {  // g_nu: sqrt(n) / sqrt(n+1) on the e-ph slots of mode nu
    const int n = s.n[s.j * m.V + p];
    if (n > 0) {
      State t = s;
      t.n[s.j * m.V + p] = n - 1;
      out.push_back({t, std::sqrt(double(n))});
    }
    if (n < m.cut[p]) {
      State t = s;
      t.n[s.j * m.V + p] = n + 1;
      out.push_back({t, std::sqrt(double(n + 1))});
    }
    return;
  }
  p -= nG;
  if (p < nW) {  // omega_nu: total occupation T_nu on the diagonal
    long T = 0;
    for (int i = 0; i < m.N; ++i) T += s.n[i * m.V + p];
    if (T) out.push_back({s, double(T)});
    return;
  }
  p -= nW;  // eps_p: 1 on the diagonal of rows with the exciton at site p
  if (s.j == p) out.push_back({s, 1.0});
}

int num_params(const Model& m) { return m.ndim + 2 * m.V + m.N; }

// CSR of dH/dtheta_p over the sorted set S.
void build_dH(const Model& m, const Keys& S, int p, CSR& E) {
  const int64_t n = S.size();
  E.n = n;
  E.rowptr.assign(n + 1, 0);
  E.cols.clear();
  E.vals.clear();
  std::vector<std::pair<State, double>> ent;
  std::vector<uint64_t> key(m.W);
  for (int64_t i = 0; i < n; ++i) {
    State s;
    decode(m, S.at(i), s);
    dH_entries(m, s, p, ent);
    std::vector<std::pair<int64_t, double>> row;
    for (auto& e : ent) {
      encode(m, e.first, key.data());
      const int64_t c = find_key(S, key.data());
      if (c >= 0) row.push_back({c, e.second});
    }
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      E.cols.push_back(e.first);
      E.vals.push_back(e.second);
    }
    E.rowptr[i + 1] = int64_t(E.cols.size());
  }
}

// (dU/dtheta_p) v for U = exp(-i H dt): top block of exp(-i dt [[H, E],
// [0, H]]) [0; v].  The doubled matrix is block triangular, so its
// spectrum is that of H and H's bounds serve the series' shift.
int frechet_apply(const CSR& H, const CSR& E, double dt, int max_terms,
                  const std::vector<cplx>& v, std::vector<cplx>& out) {
  const int64_t n = H.n;
  CSR B;
  B.n = 2 * n;
  B.rowptr.assign(2 * n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) {
      B.cols.push_back(H.cols[e]);
      B.vals.push_back(H.vals[e]);
    }
    for (int64_t e = E.rowptr[i]; e < E.rowptr[i + 1]; ++e) {
      B.cols.push_back(n + E.cols[e]);
      B.vals.push_back(E.vals[e]);
    }
    B.rowptr[i + 1] = int64_t(B.cols.size());
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = H.rowptr[i]; e < H.rowptr[i + 1]; ++e) {
      B.cols.push_back(n + H.cols[e]);
      B.vals.push_back(H.vals[e]);
    }
    B.rowptr[n + i + 1] = int64_t(B.cols.size());
  }
  B.emin = H.emin;
  B.emax = H.emax;
  std::vector<cplx> w(2 * n, cplx(0, 0)), r;
  for (int64_t i = 0; i < n; ++i) w[n + i] = v[i];
  int terms = 0;
  if (expmv(B, dt, max_terms, w, r, terms)) return 1;
  out.assign(r.begin(), r.begin() + n);
  return 0;
}

// A recorded run: the initial state and the set of every step.
struct Frozen {
  const Model* m = nullptr;
  Params p;
  Keys S0;                   // sorted support of psi0
  std::vector<cplx> psi0;    // aligned with S0
  std::vector<Keys> S;       // S[s] = set after step s+1
};

bool same_shape(const Model& a, const Model& b) {
  if (a.ndim != b.ndim || a.N != b.N || a.V != b.V) return false;
  for (int x = 0; x < 3; ++x)
    if (a.ext[x] != b.ext[x] || a.per[x] != b.per[x]) return false;
  for (int nu = 0; nu < a.V; ++nu)
    if (a.cut[nu] != b.cut[nu]) return false;
  return true;
}

// v on set `from` restricted to set `to` (both sorted).
std::vector<cplx> restrict_to(const Keys& from, const std::vector<cplx>& v,
                              const Keys& to) {
  std::vector<cplx> r(to.size(), cplx(0, 0));
  for (int64_t i = 0; i < from.size(); ++i) {
    const int64_t k = find_key(to, from.at(i));
    if (k >= 0) r[k] = v[i];
  }
  return r;
}

cplx overlap0(const Frozen& f, const Keys& S, const std::vector<cplx>& v) {
  cplx a(0, 0);
  for (int64_t i = 0; i < f.S0.size(); ++i) {
    const int64_t r = find_key(S, f.S0.at(i));
    if (r >= 0) a += std::conj(f.psi0[i]) * v[r];
  }
  return a;
}

// Replay of the recorded sets with model m: a[0..n] and, if wanted, every
// psi_s.
int frozen_forward(const Frozen& f, const Model& m, std::vector<cplx>& a,
                   std::vector<std::vector<cplx>>* states) {
  const int64_t n = int64_t(f.S.size());
  a.assign(n + 1, cplx(0, 0));
  std::vector<cplx> psi = f.psi0;
  a[0] = overlap0(f, f.S0, psi);
  if (states) states->assign(1, psi);
  const Keys* prev = &f.S0;
  for (int64_t s = 0; s < n; ++s) {
    std::vector<cplx> phi = restrict_to(*prev, psi, f.S[s]);
    CSR H;
    build_csr(m, f.S[s], H);
    int terms = 0;
    if (expmv(H, f.p.dt, f.p.max_terms, phi, psi, terms)) return 1;
    a[s + 1] = overlap0(f, f.S[s], psi);
    if (states) states->push_back(psi);
    prev = &f.S[s];
  }
  return 0;
}

int frozen_gradient(const Frozen& f, const Model& m,
                    const std::vector<cplx>& gbar, std::vector<cplx>& a,
                    std::vector<double>& grad) {
  std::vector<std::vector<cplx>> psi;
  if (frozen_forward(f, m, a, &psi)) return 1;
  const int64_t n = int64_t(f.S.size());
  const int P = num_params(m);
  grad.assign(P, 0.0);
  // lambda_n = gbar_n psi0 on S_n
  auto psi0_on = [&](const Keys& S, cplx c) {
    std::vector<cplx> r = restrict_to(f.S0, f.psi0, S);
    for (auto& z : r) z *= c;
    return r;
  };
  const Keys& last = n ? f.S[n - 1] : f.S0;
  std::vector<cplx> lam = psi0_on(last, gbar[n]);
  for (int64_t s = n - 1; s >= 0; --s) {
    const Keys& from = s ? f.S[s - 1] : f.S0;
    const Keys& to = f.S[s];
    const std::vector<cplx> phi = restrict_to(from, psi[s], to);
    CSR H;
    build_csr(m, to, H);
    for (int p = 0; p < P; ++p) {
      CSR E;
      build_dH(m, to, p, E);
      std::vector<cplx> x;
      if (frechet_apply(H, E, f.p.dt, f.p.max_terms, phi, x)) return 1;
      cplx ip(0, 0);
      for (int64_t i = 0; i < to.size(); ++i) ip += std::conj(lam[i]) * x[i];
      grad[p] += 2.0 * ip.real();
    }
    // mu = U^dag lambda = conj(U conj(lambda)) since H is real
    std::vector<cplx> cl(lam.size()), mu;
    for (size_t i = 0; i < lam.size(); ++i) cl[i] = std::conj(lam[i]);
    int terms = 0;
    if (expmv(H, f.p.dt, f.p.max_terms, cl, mu, terms)) return 1;
    for (auto& z : mu) z = std::conj(z);
    // lambda_s = T_s^T mu + gbar_s psi0 on S_s
    std::vector<cplx> back(from.size(), cplx(0, 0));
    for (int64_t i = 0; i < from.size(); ++i) {
      const int64_t k = find_key(to, from.at(i));
      if (k >= 0) back[i] = mu[k];
    }
    std::vector<cplx> add = psi0_on(from, gbar[s]);
    for (int64_t i = 0; i < from.size(); ++i) back[i] += add[i];
    lam.swap(back);
  }
  return 0;
}

}  // namespace

extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

// Threads of the row loops (results do not depend on them).
int orc_set_threads(int32_t n) {
  if (n < 1) return 1;
  omp_set_num_threads(n);
  return 0;
}
int32_t orc_threads(void) { return omp_get_max_threads(); }

int orc_pack_fields(int32_t nfields, const int32_t* widths,
                    const uint64_t* values, int32_t W, uint64_t* out) {
  if (nfields < 0 || W < 1) return fail("bad arguments");
  std::vector<int> wd(nfields), off(nfields);
  int pos = 0;
  for (int f = nfields - 1; f >= 0; --f) {
    if (widths[f] < 0 || widths[f] > 64) return fail("bad field width");
    if (widths[f] < 64 && (values[f] >> widths[f]) != 0)
      return fail("value does not fit its field");
    wd[f] = widths[f];
    off[f] = pos;
    pos += widths[f];
  }
  if (pos > 64 * W) return fail("fields do not fit in W words");
  pack_bits(nfields, wd.data(), off.data(), values, W, out);
  return 0;
}

int orc_model_create(const orc_model_desc* d, void** out) {
  if (!d || !out) return fail("null argument");
  Model* m = new Model();
  m->ndim = d->ndim;
  if (m->ndim < 1 || m->ndim > 3) {
    delete m;
    return fail("ndim must be 1..3");
  }
  m->N = 1;
  for (int a = 0; a < 3; ++a) {
    m->ext[a] = a < m->ndim ? d->extent[a] : 1;
    m->per[a] = a < m->ndim ? (d->periodic[a] != 0) : 0;
    m->J[a] = a < m->ndim ? d->J[a] : 0.0;
    if (m->ext[a] < 1 || (m->per[a] && m->ext[a] < 3)) {
      delete m;
      return fail("extent must be >= 1, and >= 3 when periodic");
    }
    m->N *= m->ext[a];
  }
  if (m->N >= 65536) {
    delete m;
    return fail("too many sites");
  }
  m->V = d->n_modes;
  if (m->V < 1 || m->V > 4) {
    delete m;
    return fail("n_modes must be 1..4");
  }
  for (int nu = 0; nu < m->V; ++nu) {
    m->cut[nu] = d->cutoff[nu];
    m->omega[nu] = d->omega[nu];
    m->g[nu] = d->g[nu];
    if (m->cut[nu] < 1 || m->cut[nu] > 255) {
      delete m;
      return fail("cutoff must be 1..255");
    }
    m->bnu[nu] = bits_for(m->cut[nu] + 1);
  }
  m->eps.assign(m->N, 0.0);
  if (d->eps)
    for (int i = 0; i < m->N; ++i) m->eps[i] = d->eps[i];
  m->bj = std::max(1, bits_for(m->N));
  // fields: occupations site-major most significant first, j last
  m->widths.clear();
  for (int i = 0; i < m->N; ++i)
    for (int nu = 0; nu < m->V; ++nu) m->widths.push_back(m->bnu[nu]);
  m->widths.push_back(m->bj);
  m->offsets.assign(m->widths.size(), 0);
  int pos = 0;
  for (int f = int(m->widths.size()) - 1; f >= 0; --f) {
    m->offsets[f] = pos;
    pos += m->widths[f];
  }
  m->B = pos;
  m->W = (m->B + 63) / 64;
  m->D = m->slot_count();
  // nearest neighbours per axis, +1 then -1
  m->nbr.assign(size_t(m->N) * 2 * m->ndim, -1);
  for (int i = 0; i < m->N; ++i) {
    int c[3] = {i % m->ext[0], (i / m->ext[0]) % m->ext[1],
                i / (m->ext[0] * m->ext[1])};
    for (int a = 0; a < m->ndim; ++a)
      for (int dir = 0; dir < 2; ++dir) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[a] += dir == 0 ? 1 : -1;
        if (cc[a] < 0 || cc[a] >= m->ext[a]) {
          if (!m->per[a]) continue;
          cc[a] = (cc[a] + m->ext[a]) % m->ext[a];
        }
        m->nbr[size_t(i) * 2 * m->ndim + 2 * a + dir] =
            cc[0] + m->ext[0] * (cc[1] + m->ext[1] * cc[2]);
      }
  }
  *out = m;
  return 0;
}

void orc_model_destroy(void* m) { delete static_cast<Model*>(m); }

int orc_model_info(const void* mp, int32_t* N, int32_t* W, int32_t* D,
                   int32_t* B) {
  const Model* m = static_cast<const Model*>(mp);
  if (!m) return fail("null model");
  if (N) *N = m->N;
  if (W) *W = m->W;
  if (D) *D = m->D;
  if (B) *B = m->B;
  return 0;
}

int orc_pack(const void* mp, int64_t n, const int32_t* exc,
             const uint16_t* occ, uint64_t* keys) {
  const Model* m = static_cast<const Model*>(mp);
  if (!m || n < 0) return fail("bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    State s;
    s.j = exc[i];
    if (s.j < 0 || s.j >= m->N) return fail("exciton site out of range");
    s.n.resize(m->N * m->V);
    for (int f = 0; f < m->N * m->V; ++f) {
      s.n[f] = occ[i * m->N * m->V + f];
      if (s.n[f] > m->cut[f % m->V]) return fail("occupation above cutoff");
    }
    encode(*m, s, keys + i * m->W);
  }
  return 0;
}

int orc_unpack(const void* mp, int64_t n, const uint64_t* keys, int32_t* exc,
               uint16_t* occ) {
  const Model* m = static_cast<const Model*>(mp);
  if (!m || n < 0) return fail("bad arguments");
  for (int64_t i = 0; i < n; ++i) {
    State s;
    decode(*m, keys + i * m->W, s);
    exc[i] = s.j;
    for (int f = 0; f < m->N * m->V; ++f)
      occ[i * m->N * m->V + f] = uint16_t(s.n[f]);
  }
  return 0;
}

int orc_neighbors(const void* mp, int64_t n, const uint64_t* keys,
                  uint64_t* keys_out, uint8_t* exists, double* vals,
                  double* diag) {
  const Model* m = static_cast<const Model*>(mp);
  if (!m || n < 0) return fail("bad arguments");
  if (check_keys(*m, n, keys)) return 1;
  const int D = m->D, W = m->W;
  for (int64_t i = 0; i < n; ++i) {
    State s;
    std::vector<Slot> sl;
    decode(*m, keys + i * W, s);
    slots_of(*m, s, sl);
    diag[i] = diagonal(*m, s);
    for (int q = 0; q < D; ++q) {
      exists[i * D + q] = sl[q].exists ? 1 : 0;
      vals[i * D + q] = sl[q].exists ? sl[q].val : 0.0;
      uint64_t* k = keys_out + (i * D + q) * W;
      for (int w = 0; w < W; ++w) k[w] = 0;
      if (sl[q].exists) encode(*m, sl[q].s, k);
    }
  }
  return 0;
}

int orc_sim_create(const void* mp, const orc_params* p, int64_t n,
                   const int32_t* exc, const uint16_t* occ,
                   const double* coef, void** out) {
  const Model* m = static_cast<const Model*>(mp);
  if (!m || !p || !out || n < 1) return fail("bad arguments");
  if (p->k < 0 || p->k_init < 0 || !(p->dt > 0) || !(p->theta >= 0))
    return fail("bad run parameters");
  std::vector<uint64_t> keys(size_t(n) * m->W);
  if (orc_pack(mp, n, exc, occ, keys.data())) return 1;
  Sim* s = new Sim();
  s->m = m;
  s->p.dt = p->dt;
  s->p.k = p->k;
  s->p.k_init = p->k_init;
  s->p.theta = p->theta;
  s->p.max_terms = p->max_terms > 0 ? p->max_terms : 200;
  if (p->max_states < 0) {
    delete s;
    return fail("bad state cap");
  }
  s->p.max_states = p->max_states;
  if (p->q_nom < 0 || (p->q_nom > 0 && p->max_states > 0)) {
    delete s;
    return fail("bad q_nom");
  }
  s->p.q_nom = p->q_nom;
  if (p->krylov_order < 0 || p->krylov_order > 63) {
    delete s;
    return fail("bad krylov_order");
  }
  s->p.krylov_order = p->krylov_order;
  if (p->taylor_order < -1 || p->taylor_order > 60 ||
      (p->taylor_order != 0 && p->krylov_order != 0)) {
    delete s;
    return fail("bad taylor_order");
  }
  s->p.taylor_order = p->taylor_order;
  if (load_state(*m, n, keys.data(), coef, s->S, s->psi)) {
    delete s;
    return 1;
  }
  s->psi0_keys = s->S;
  s->psi0 = s->psi;
  s->M.W = s->S.W = m->W;
  *out = s;
  return 0;
}

void orc_sim_destroy(void* s) { delete static_cast<Sim*>(s); }

int orc_sim_step(void* sp, int64_t n_steps) {
  Sim* s = static_cast<Sim*>(sp);
  if (!s || n_steps < 0) return fail("bad arguments");
  for (int64_t i = 0; i < n_steps; ++i)
    if (sim_step(*s)) return 1;
  return 0;
}

int orc_sim_set_state(void* sp, int64_t n, const uint64_t* keys,
                      const double* amps, double t) {
  Sim* s = static_cast<Sim*>(sp);
  if (!s || n < 0) return fail("bad arguments");
  if (check_keys(*s->m, n, keys)) return 1;
  Keys S;
  std::vector<cplx> psi;
  if (load_state(*s->m, n, keys, amps, S, psi)) return 1;
  s->S = S;
  s->psi = psi;
  s->t = t;
  s->fresh = false;
  return 0;
}

// Counts of the step before a loaded state (the state cap's q rule, App.
// "How to weight states for truncation" as read for a fixed cap): as if
// the state had been reached by a step with these |S| and |M|.
int orc_sim_set_prev_counts(void* sp, int64_t nS, int64_t nM) {
  Sim* s = static_cast<Sim*>(sp);
  if (!s || nS < 0 || nM < 0) return fail("bad arguments");
  s->prev_nS = nS;
  s->prev_nM = nM;
  return 0;
}

int orc_sim_size(const void* sp, int64_t* nS) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s || !nS) return fail("bad arguments");
  *nS = s->S.size();
  return 0;
}

int orc_sim_get_state(const void* sp, uint64_t* keys, double* amps) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s) return fail("bad arguments");
  if (keys) std::memcpy(keys, s->S.d.data(), s->S.d.size() * 8);
  if (amps)
    for (int64_t i = 0; i < s->S.size(); ++i) {
      amps[2 * i] = s->psi[i].real();
      amps[2 * i + 1] = s->psi[i].imag();
    }
  return 0;
}

int orc_sim_get_phi(const void* sp, double* amps) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s || !amps) return fail("bad arguments");
  for (size_t i = 0; i < s->phi.size(); ++i) {
    amps[2 * i] = s->phi[i].real();
    amps[2 * i + 1] = s->phi[i].imag();
  }
  return 0;
}

int orc_sim_get_set(const void* sp, int32_t which, int32_t round, int64_t* n,
                    uint64_t* keys) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s || !n) return fail("bad arguments");
  const Keys* k = nullptr;
  if (which == ORC_SET_M)
    k = &s->M;
  else if (which == ORC_SET_S)
    k = &s->S;
  else if (which == ORC_SET_FRONTIER) {
    if (round < 0 || round >= int(s->frontier.size()))
      return fail("no such round");
    k = &s->frontier[round];
  } else
    return fail("unknown set");
  *n = k->size();
  if (keys) std::memcpy(keys, k->d.data(), k->d.size() * 8);
  return 0;
}

int orc_sim_num_obs(const void* sp, int64_t* n) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s || !n) return fail("bad arguments");
  *n = int64_t(s->obs.size());
  return 0;
}

int orc_sim_obs(const void* sp, int64_t i, double* fields, double* pop) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s || i < 0 || i >= int64_t(s->obs.size()))
    return fail("bad arguments");
  if (fields)
    for (int f = 0; f < ORC_OBS_NFIELDS; ++f) fields[f] = s->obs[i].f[f];
  if (pop)
    for (size_t j = 0; j < s->obs[i].pop.size(); ++j) pop[j] = s->obs[i].pop[j];
  return 0;
}

int orc_sim_csr(const void* sp, int64_t* nrows, int64_t* nnz, int64_t* rowptr,
                int64_t* cols, double* vals) {
  const Sim* s = static_cast<const Sim*>(sp);
  if (!s) return fail("bad arguments");
  if (nrows) *nrows = s->H.n;
  if (nnz) *nnz = int64_t(s->H.cols.size());
  if (rowptr)
    std::memcpy(rowptr, s->H.rowptr.data(), s->H.rowptr.size() * 8);
  if (cols) std::memcpy(cols, s->H.cols.data(), s->H.cols.size() * 8);
  if (vals) std::memcpy(vals, s->H.vals.data(), s->H.vals.size() * 8);
  return 0;
}

int orc_expmv(int64_t n, const int64_t* rowptr, const int64_t* cols,
              const double* vals, double dt, double emin, double emax,
              int32_t max_terms, const double* v_in, double* v_out,
              int32_t* terms) {
  CSR H;
  H.n = n;
  H.rowptr.assign(rowptr, rowptr + n + 1);
  H.cols.assign(cols, cols + rowptr[n]);
  H.vals.assign(vals, vals + rowptr[n]);
  H.emin = emin;
  H.emax = emax;
  std::vector<cplx> v(n), out;
  for (int64_t i = 0; i < n; ++i) v[i] = cplx(v_in[2 * i], v_in[2 * i + 1]);
  int t = 0;
  if (expmv(H, dt, max_terms > 0 ? max_terms : 200, v, out, t)) return 1;
  for (int64_t i = 0; i < n; ++i) {
    v_out[2 * i] = out[i].real();
    v_out[2 * i + 1] = out[i].imag();
  }
  if (terms) *terms = t;
  return 0;
}

int orc_lanczos(int64_t n, const int64_t* rowptr, const int64_t* cols,
                const double* vals, double dt, int32_t order,
                const double* v_in, double* v_out, double* basis,
                double* alpha, double* beta, int32_t* dim, double* e_range) {
  if (n < 0 || !rowptr || !v_in || !v_out) return fail("bad arguments");
  CSR H;
  H.n = n;
  H.rowptr.assign(rowptr, rowptr + n + 1);
  H.cols.assign(cols, cols + rowptr[n]);
  H.vals.assign(vals, vals + rowptr[n]);
  std::vector<cplx> v(n), out;
  for (int64_t i = 0; i < n; ++i) v[i] = cplx(v_in[2 * i], v_in[2 * i + 1]);
  KrylovOut ko;
  if (lanczos_expmv(H, dt, order, v, out, ko)) return 1;
  for (int64_t i = 0; i < n; ++i) {
    v_out[2 * i] = out[i].real();
    v_out[2 * i + 1] = out[i].imag();
  }
  for (int j = 0; j < ko.dim; ++j) {
    if (basis)
      for (int64_t i = 0; i < n; ++i) {
        basis[2 * (int64_t(j) * n + i)] = ko.V[j][i].real();
        basis[2 * (int64_t(j) * n + i) + 1] = ko.V[j][i].imag();
      }
    if (alpha) alpha[j] = ko.alpha[j];
  }
  if (beta)
    for (size_t j = 0; j < ko.beta.size(); ++j) beta[j] = ko.beta[j];
  if (dim) *dim = ko.dim;
  if (e_range) {
    e_range[0] = ko.e_lo;
    e_range[1] = ko.e_hi;
  }
  return 0;
}

double orc_taylor_theta(int32_t m) {
  if (m < 1 || m > kTaylorMaxDeg) return -1.0;
  return taylor_thetas()[m];
}

int orc_taylor_select(double norm, int32_t* m, int32_t* s) {
  if (!(norm >= 0) || !m || !s) return fail("bad arguments");
  int mm = 0, ss = 0;
  taylor_select(norm, mm, ss);
  *m = mm;
  *s = ss;
  return 0;
}

int orc_taylor(int64_t n, const int64_t* rowptr, const int64_t* cols,
               const double* vals, double dt, double emin, double emax,
               int32_t order, const double* v_in, double* v_out,
               int32_t* mvs) {
  if (n < 0 || !rowptr || !v_in || !v_out) return fail("bad arguments");
  CSR H;
  H.n = n;
  H.rowptr.assign(rowptr, rowptr + n + 1);
  H.cols.assign(cols, cols + rowptr[n]);
  H.vals.assign(vals, vals + rowptr[n]);
  H.emin = emin;
  H.emax = emax;
  std::vector<cplx> v(n), out;
  for (int64_t i = 0; i < n; ++i) v[i] = cplx(v_in[2 * i], v_in[2 * i + 1]);
  int t = 0;
  if (taylor_expmv(H, dt, order, v, out, t)) return 1;
  for (int64_t i = 0; i < n; ++i) {
    v_out[2 * i] = out[i].real();
    v_out[2 * i + 1] = out[i].imag();
  }
  if (mvs) *mvs = t;
  return 0;
}

int orc_frozen_record(const void* mp, const orc_params* p, int64_t n,
                      const int32_t* exc, const uint16_t* occ,
                      const double* coef, int64_t n_steps, void** out) {
  if (!mp || !out || n_steps < 0) return fail("bad arguments");
  if (p && (p->krylov_order != 0 || p->taylor_order != 0))
    return fail("the adjoint gradient differentiates the series propagator");
  void* sp = nullptr;
  if (orc_sim_create(mp, p, n, exc, occ, coef, &sp)) return 1;
  Sim* sim = static_cast<Sim*>(sp);
  Frozen* f = new Frozen();
  f->m = sim->m;
  f->p = sim->p;
  f->S0 = sim->S;
  f->psi0 = sim->psi;
  for (int64_t s = 0; s < n_steps; ++s) {
    if (sim_step(*sim)) {
      delete sim;
      delete f;
      return 1;
    }
    f->S.push_back(sim->S);
  }
  delete sim;
  *out = f;
  return 0;
}

void orc_frozen_destroy(void* f) { delete static_cast<Frozen*>(f); }

int orc_sim_set_model(void* sp, const void* mp) {
  Sim* s = static_cast<Sim*>(sp);
  const Model* m = static_cast<const Model*>(mp);
  if (!s || !m) return fail("null argument");
  if (!same_shape(*s->m, *m)) return fail("model shape differs");
  s->m = m;
  return 0;
}

int orc_frozen_info(const void* fp, int64_t* n_steps, int32_t* n_params,
                    int64_t* sizes) {
  const Frozen* f = static_cast<const Frozen*>(fp);
  if (!f) return fail("null argument");
  if (n_steps) *n_steps = int64_t(f->S.size());
  if (n_params) *n_params = num_params(*f->m);
  if (sizes) {
    sizes[0] = f->S0.size();
    for (size_t s = 0; s < f->S.size(); ++s) sizes[s + 1] = f->S[s].size();
  }
  return 0;
}

int orc_frozen_get_set(const void* fp, int64_t step, uint64_t* keys) {
  const Frozen* f = static_cast<const Frozen*>(fp);
  if (!f || step < 0 || step > int64_t(f->S.size())) return fail("bad step");
  const Keys& k = step ? f->S[step - 1] : f->S0;
  std::copy(k.d.begin(), k.d.end(), keys);
  return 0;
}

int orc_frozen_eval(const void* fp, const void* mp, double* a_out) {
  const Frozen* f = static_cast<const Frozen*>(fp);
  const Model* m = static_cast<const Model*>(mp);
  if (!f || !m || !a_out) return fail("null argument");
  if (!same_shape(*f->m, *m)) return fail("model shape differs from the record");
  std::vector<cplx> a;
  if (frozen_forward(*f, *m, a, nullptr)) return 1;
  for (size_t s = 0; s < a.size(); ++s) {
    a_out[2 * s] = a[s].real();
    a_out[2 * s + 1] = a[s].imag();
  }
  return 0;
}

int orc_frozen_grad(const void* fp, const void* mp, const double* gbar,
                    double* a_out, double* grad) {
  const Frozen* f = static_cast<const Frozen*>(fp);
  const Model* m = static_cast<const Model*>(mp);
  if (!f || !m || !gbar || !grad) return fail("null argument");
  if (!same_shape(*f->m, *m)) return fail("model shape differs from the record");
  const size_t n = f->S.size() + 1;
  std::vector<cplx> gb(n), a;
  for (size_t s = 0; s < n; ++s) gb[s] = cplx(gbar[2 * s], gbar[2 * s + 1]);
  std::vector<double> g;
  if (frozen_gradient(*f, *m, gb, a, g)) return 1;
  if (a_out)
    for (size_t s = 0; s < n; ++s) {
      a_out[2 * s] = a[s].real();
      a_out[2 * s + 1] = a[s].imag();
    }
  std::copy(g.begin(), g.end(), grad);
  return 0;
}

}  // extern "C"
