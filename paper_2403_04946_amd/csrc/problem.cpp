// Host-side construction of the Burgers-Hopf operator in TT-matrix form.
//
// Paper: Sec. 3 eq. (hyper1) and eq. (coefficients) give the linear PDE
// for the characteristic function and its Galerkin coefficients; Sec. 5
// eq. (eqn:BHfde) gives the Burgers-Hopf FDE whose advective part is
// (i/2) d/dx of the second functional derivative and whose viscous part is
// nu d^2/dx^2 of the first.  On d orthonormal Fourier modes Gamma_k this is
//
//   dphi/dt = sum_k a_k [ (i/2) sum_{j,l} B_kjl d_j d_l phi + nu D_kk d_k phi ]
//   B_kjl = int Gamma_k (Gamma_j Gamma_l)',  D_kk = -kappa_k^2.
//
// B is computed here in closed form: every mode is a sum of two complex
// exponentials, so int_0^{2pi} of a product of three modes is 2*pi times the
// sum of the coefficient products whose frequencies cancel.
//
// The grid discretisation (Sec. 4 eq. (tt), (eqn:ode); Sec. 5) uses
// a_i = -L + 2L i/(n-1), centred second-order differences, and second-order
// one-sided boundary rows.
//
// An optional numerical-diffusion stabilisation (Sec. 5.2, explicit runs)
// adds kappa sum_k d^2/da_k^2: d one-site terms L2.
//
// The CDF equation (Sec. 5, eq. (eqn:cdf-burgers), the paper's own
// workload) is built by build_cdf_burgers below from the same automaton.
//
// TT-matrix form: the operator is a sum of products of one-axis operators
// on at most three sites (X = multiply by a, G = d/da, L2 = d^2/da^2, and
// the same-site compositions XG, XL2; multiplication by a_k acts after the
// derivatives).  It is written as a finite-state automaton over the sites:
// the channels on a bond are "nothing applied yet" (I), "term complete" (F),
// "a term has applied op o at site s < bond and waits for the rest" (A(s,o)),
// and "a term needs op o at site s >= bond to complete" (B(s,o)), with
// o in {X, G}.  A three-site term runs I -> A -> B -> F; a two-site term runs
// I -> A -> F or I -> B -> F; a one-site term runs I -> F.  There are at
// most 2 + 2d channels per bond.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <set>
#include <tuple>

#include "common.hpp"

namespace ttf {

namespace {

using cplx = std::complex<double>;

// A real Fourier mode as a combination of e^{i f x}: pairs (coef, f).
struct Exp2 {
  cplx c[2];
  int f[2];
};

int wavenumber(int k) { return (k + 2) / 2; }  // k 0-based -> ceil((k+1)/2)

Exp2 mode(int k, bool deriv) {
  const double s = 1.0 / std::sqrt(M_PI);
  const int m = wavenumber(k);
  Exp2 e;
  e.f[0] = m;
  e.f[1] = -m;
  const bool is_cos = (k % 2) == 0;
  if (!deriv) {
    if (is_cos) {  // cos = (e^{imx} + e^{-imx})/2
      e.c[0] = s * 0.5;
      e.c[1] = s * 0.5;
    } else {  // sin = (e^{imx} - e^{-imx})/(2i)
      e.c[0] = s * cplx(0, -0.5);
      e.c[1] = s * cplx(0, 0.5);
    }
  } else {
    if (is_cos) {  // (cos mx)' = -m sin mx
      e.c[0] = -m * s * cplx(0, -0.5);
      e.c[1] = -m * s * cplx(0, 0.5);
    } else {  // (sin mx)' = m cos mx
      e.c[0] = m * s * 0.5;
      e.c[1] = m * s * 0.5;
    }
  }
  return e;
}

// int_0^{2pi} p q r dx for three exponential pairs
double triple(const Exp2& p, const Exp2& q, const Exp2& r) {
  cplx acc = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c)
        if (p.f[a] + q.f[b] + r.f[c] == 0) acc += p.c[a] * q.c[b] * r.c[c];
  return (2.0 * M_PI * acc).real();
}

// Same-site composition of variables: x = multiply by a, p = d/da.
int compose(int nx, int np) {
  if (nx == 1 && np == 0) return OP_X;
  if (nx == 0 && np == 1) return OP_G;
  if (nx == 0 && np == 2) return OP_L2;
  if (nx == 1 && np == 1) return OP_XG;
  if (nx == 1 && np == 2) return OP_XL2;
  fail(TT_EINVAL, "unsupported local operator composition");
}

struct Term {
  cplx coef;
  std::vector<std::pair<int, int>> ops;  // (site, local op), sorted by site
};

// Rows of the local operators as lists of (column, weight); zero weights
// are dropped.  finish() packs them into the compressed rows of tt_op.
struct TapRows {
  int n;
  std::vector<std::vector<std::pair<int, double>>> rows;
  explicit TapRows(int n_) : n(n_), rows((size_t)NOPS * n_) {}
  void add(int o, int i, int col, double w) {
    if (w != 0.0) rows[(size_t)o * n + i].push_back({col, w});
  }
  void finish(tt_op* op) const {
    op->tap_ptr.assign(rows.size() + 1, 0);
    op->tap_col.clear();
    op->tap_w.clear();
    for (size_t r = 0; r < rows.size(); ++r) {
      for (const auto& cw : rows[r]) {
        op->tap_col.push_back(cw.first);
        op->tap_w.push_back(cw.second);
      }
      op->tap_ptr[r + 1] = (int)op->tap_col.size();
    }
  }
};

void build_automaton(tt_op* op, const std::vector<Term>& terms);

}  // namespace

void build_burgers_hopf(tt_op* op) {
  const int d = op->d, n = op->n;
  const double L = op->L, nu = op->nu;
  // ---- Galerkin coefficients
  op->B.assign((size_t)d * d * d, 0.0);
  op->D.assign((size_t)d * d, 0.0);
  std::vector<Exp2> g(d), gp(d);
  for (int k = 0; k < d; ++k) {
    g[k] = mode(k, false);
    gp[k] = mode(k, true);
  }
  for (int k = 0; k < d; ++k)
    for (int j = 0; j < d; ++j)
      for (int l = 0; l < d; ++l) {
        // int G_k (G_j G_l)' = int G_k G_j' G_l + int G_k G_j G_l'
        double v = triple(g[k], gp[j], g[l]) + triple(g[k], g[j], gp[l]);
        if (std::fabs(v) < 1e-13) v = 0.0;
        op->B[((size_t)k * d + j) * d + l] = v;
      }
  for (int k = 0; k < d; ++k) {
    const double m = wavenumber(k);
    op->D[(size_t)k * d + k] = -m * m;
  }
  // ---- grid and local operators as taps
  const double h = 2.0 * L / (n - 1);
  op->grid.resize(n);
  for (int i = 0; i < n; ++i) op->grid[i] = -L + 2.0 * L * i / (n - 1);
  TapRows taps(n);
  auto set = [&](int o, int i, int, int col, double w) { taps.add(o, i, col, w); };
  for (int i = 0; i < n; ++i) {
    set(OP_I, i, 0, i, 1.0);
    set(OP_X, i, 0, i, op->grid[i]);
    // first derivative
    int gc[3];
    double gw[3];
    if (i == 0) {
      gc[0] = 0; gc[1] = 1; gc[2] = 2;
      gw[0] = -3.0 / (2 * h); gw[1] = 4.0 / (2 * h); gw[2] = -1.0 / (2 * h);
    } else if (i == n - 1) {
      gc[0] = n - 3; gc[1] = n - 2; gc[2] = n - 1;
      gw[0] = 1.0 / (2 * h); gw[1] = -4.0 / (2 * h); gw[2] = 3.0 / (2 * h);
    } else {
      gc[0] = i - 1; gc[1] = i; gc[2] = i + 1;
      gw[0] = -1.0 / (2 * h); gw[1] = 0.0; gw[2] = 1.0 / (2 * h);
    }
    for (int t = 0; t < 3; ++t) {
      set(OP_G, i, t, gc[t], gw[t]);
      set(OP_XG, i, t, gc[t], op->grid[i] * gw[t]);
    }
    // second derivative
    int lc[4];
    double lw[4];
    const double h2 = h * h;
    if (i == 0) {
      for (int t = 0; t < 4; ++t) lc[t] = t;
      lw[0] = 2 / h2; lw[1] = -5 / h2; lw[2] = 4 / h2; lw[3] = -1 / h2;
    } else if (i == n - 1) {
      for (int t = 0; t < 4; ++t) lc[t] = n - 4 + t;
      lw[0] = -1 / h2; lw[1] = 4 / h2; lw[2] = -5 / h2; lw[3] = 2 / h2;
    } else {
      lc[0] = i - 1; lc[1] = i; lc[2] = i + 1; lc[3] = i;
      lw[0] = 1 / h2; lw[1] = -2 / h2; lw[2] = 1 / h2; lw[3] = 0.0;
    }
    for (int t = 0; t < 4; ++t) {
      set(OP_L2, i, t, lc[t], lw[t]);
      set(OP_XL2, i, t, lc[t], op->grid[i] * lw[t]);
    }
  }
  taps.finish(op);
  // ---- operator terms
  std::vector<Term> terms;
  const cplx half_i(0.0, 0.5);
  for (int k = 0; k < d; ++k)
    for (int j = 0; j < d; ++j)
      for (int l = j; l < d; ++l) {
        const double bjl = op->adv * op->B[((size_t)k * d + j) * d + l];
        if (bjl == 0.0) continue;
        // sum over ordered (j,l) of B_kjl d_j d_l = B_kjj d_j^2 + 2 B_kjl d_j d_l (j<l)
        const cplx c = half_i * (j == l ? bjl : 2.0 * bjl);
        std::map<int, std::pair<int, int>> cnt;  // site -> (#x, #p)
        cnt[k].first += 1;
        cnt[j].second += 1;
        cnt[l].second += 1;
        Term t;
        t.coef = c;
        for (auto& kv : cnt) t.ops.push_back({kv.first, compose(kv.second.first, kv.second.second)});
        terms.push_back(t);
      }
  for (int k = 0; k < d; ++k) {
    const double dk = op->D[(size_t)k * d + k];
    if (dk == 0.0 || nu == 0.0) continue;
    Term t;
    t.coef = cplx(nu * dk, 0.0);
    t.ops.push_back({k, OP_XG});
    terms.push_back(t);
  }
  if (op->ident != 0.0) {
    // ident * I as a one-site term (I at the first site): with no other
    // term the automaton has one channel per bond, R = 1
    Term t;
    t.coef = cplx(op->ident, 0.0);
    t.ops.push_back({0, OP_I});
    terms.push_back(t);
  }
  if (op->diff != 0.0)
    for (int k = 0; k < d; ++k) {
      Term t;
      t.coef = cplx(op->diff, 0.0);
      t.ops.push_back({k, OP_L2});
      terms.push_back(t);
    }
  build_automaton(op, terms);
}

namespace {

void build_automaton(tt_op* op, const std::vector<Term>& terms) {
  const int d = op->d;
  // ---- automaton
  // channel key: (kind, site, op); kind 0 = I, 1 = F, 2 = A, 3 = B
  using Key = std::tuple<int, int, int>;
  const Key KI{0, -1, -1}, KF{1, -1, -1};
  std::vector<std::set<Key>> live(d + 1);
  // transitions: (site, from key, to key, local op) -> coefficient
  std::map<std::tuple<int, Key, Key, int>, cplx> trans;
  auto is_xg = [](int o) { return o == OP_X || o == OP_G; };
  for (const Term& t : terms) {
    const int ns = (int)t.ops.size();
    const int s1 = t.ops[0].first, o1 = t.ops[0].second;
    // The automaton path of the term as (site, from, to, op, coef, shared).
    // Entry (I -> A) and exit (B -> F) transitions are shared by every term
    // through that channel and carry weight 1; the term's coefficient sits
    // on its one term-specific transition and accumulates.
    std::vector<std::tuple<int, Key, Key, int, cplx, bool>> path;
    if (ns == 1) {
      path.push_back({s1, KI, KF, o1, t.coef, false});
    } else if (ns == 2) {
      const int s2 = t.ops[1].first, o2 = t.ops[1].second;
      // the shared channel waits after an X or G end; a term with
      // composite ops at both ends waits after its first one
      if (is_xg(o1) || !is_xg(o2)) {
        Key a{2, s1, o1};
        path.push_back({s1, KI, a, o1, 1.0, true});
        path.push_back({s2, a, KF, o2, t.coef, false});
      } else {
        Key b{3, s2, o2};
        path.push_back({s1, KI, b, o1, t.coef, false});
        path.push_back({s2, b, KF, o2, 1.0, true});
      }
    } else {
      const int s2 = t.ops[1].first, o2 = t.ops[1].second;
      const int s3 = t.ops[2].first, o3 = t.ops[2].second;
      if (!is_xg(o1) || !is_xg(o2) || !is_xg(o3)) fail(TT_EINVAL, "three-site term with composite op");
      Key a{2, s1, o1}, b{3, s3, o3};
      path.push_back({s1, KI, a, o1, 1.0, true});
      path.push_back({s2, a, b, o2, t.coef, false});
      path.push_back({s3, b, KF, o3, 1.0, true});
    }
    // every intermediate channel is live on the bonds it spans, I before the
    // first site, F after the last
    for (int c = 0; c <= s1; ++c) live[c].insert(KI);
    for (size_t p = 0; p < path.size(); ++p) {
      const int s = std::get<0>(path[p]);
      const Key to = std::get<2>(path[p]);
      const int next = (p + 1 < path.size()) ? std::get<0>(path[p + 1]) : d;
      for (int c = s + 1; c <= next; ++c) live[c].insert(to);
      const auto key = std::make_tuple(s, std::get<1>(path[p]), to, std::get<3>(path[p]));
      if (std::get<5>(path[p]))
        trans[key] = 1.0;
      else
        trans[key] += std::get<4>(path[p]);
    }
  }
  // identity pass-throughs for channels live on both sides of a site
  for (int s = 0; s < d; ++s)
    for (const Key& k : live[s])
      if (live[s + 1].count(k)) trans[{s, k, k, OP_I}] += 1.0;
  // index channels per bond: I, F, A's, B's in key order
  std::vector<std::map<Key, int>> index(d + 1);
  op->R.assign(d + 1, 0);
  for (int c = 0; c <= d; ++c) {
    int idx = 0;
    for (const Key& k : live[c]) index[c][k] = idx++;
    op->R[c] = idx;
  }
  if (op->R[0] != 1 || op->R[d] != 1) fail(TT_EINVAL, "operator automaton must start and end in one state");
  op->site.assign(d, {});
  for (const auto& kv : trans) {
    const int s = std::get<0>(kv.first);
    const Key& from = std::get<1>(kv.first);
    const Key& to = std::get<2>(kv.first);
    if (!index[s].count(from) || !index[s + 1].count(to)) fail(TT_EINVAL, "automaton transition on a dead channel");
    if (std::abs(kv.second) == 0.0) continue;
    Entry e;
    e.alpha = index[s].at(from);
    e.beta = index[s + 1].at(to);
    e.lop = std::get<3>(kv.first);
    e.cre = kv.second.real();
    e.cim = kv.second.imag();
    op->site[s].push_back(e);
  }
}

}  // namespace

// The CDF equation of the stochastic Burgers equation with reaction
// R(u) = alpha sin(pi u) (Sec. 5, eq. (eqn:burgers-rxn) and
// eq. (eqn:cdf-burgers)) on N = d evenly spaced points of the circle.  With
// D1, D2 the periodic second-order first- and second-difference matrices
// (spacing 2 pi / N), the semi-discrete velocity of point i is
// v_i = -u_i (D1 u)_i + gamma (D2 u)_i + R(u_i); integrating the Liouville
// equation over the phase variables up to u gives
//
//   dF/dt = sum_i [ -gamma D2_ii u_i - R(u_i) ] dF/du_i
//         + sum_{i != j} [ D1_ij u_i - gamma D2_ij ] (u_j - J_j) dF/du_i,
//
// J_j being the cumulative integral along u_j from the lower end of the
// box.  The reaction enters once, as in the velocity (the equation as
// printed repeats it in a separate last sum).  Phase space: [-box, box]^N,
// n points per axis (ends included); centred second-order differences with
// outflow boundaries (dF/du = 0: the boundary rows of G are zero), the
// trapezoid rule for J.  Local operators: X, G, XG, SG = sin(pi u) G and
// K = X - J; the terms are one-site (XG, SG) and two-site (XG or G at i,
// K at j = i +- 1 mod N).  op->L is the box half-width, op->gamma and
// op->alpha the coefficients, op->diff an optional kappa sum_k d2F/du_k^2
// (interior rows of L2; the boundary rows are zero).
void build_cdf_burgers(tt_op* op) {
  const int d = op->d, n = op->n;
  const double box = op->L, gamma = op->gamma, alpha = op->alpha;
  const double h = 2.0 * box / (n - 1);
  op->grid.resize(n);
  for (int i = 0; i < n; ++i) op->grid[i] = -box + 2.0 * box * i / (n - 1);
  TapRows taps(n);
  for (int i = 0; i < n; ++i) {
    const double u = op->grid[i];
    taps.add(OP_I, i, i, 1.0);
    taps.add(OP_X, i, i, u);
    if (i > 0 && i < n - 1) {
      const double w = 1.0 / (2 * h), w2 = 1.0 / (h * h);
      taps.add(OP_G, i, i - 1, -w);
      taps.add(OP_G, i, i + 1, w);
      taps.add(OP_XG, i, i - 1, -u * w);
      taps.add(OP_XG, i, i + 1, u * w);
      const double sn = std::sin(M_PI * u);
      taps.add(OP_SG, i, i - 1, -sn * w);
      taps.add(OP_SG, i, i + 1, sn * w);
      taps.add(OP_L2, i, i - 1, w2);
      taps.add(OP_L2, i, i, -2.0 * w2);
      taps.add(OP_L2, i, i + 1, w2);
      taps.add(OP_XL2, i, i - 1, u * w2);
      taps.add(OP_XL2, i, i, -2.0 * u * w2);
      taps.add(OP_XL2, i, i + 1, u * w2);
    }
    // K = X - J, (J g)_i = h (g_0 / 2 + g_1 + ... + g_{i-1} + g_i / 2)
    for (int c = 0; c <= i; ++c) {
      double w = 0.0;
      if (i > 0) w = -h * ((c == 0 || c == i) ? 0.5 : 1.0);
      if (c == i) w += u;
      taps.add(OP_K, i, c, w);
    }
  }
  taps.finish(op);
  // periodic difference matrices on the circle
  const double dx = 2.0 * M_PI / d;
  std::vector<double> D1((size_t)d * d, 0.0), D2((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) {
    const int ip = (i + 1) % d, im = (i + d - 1) % d;
    D1[(size_t)i * d + ip] += 1.0 / (2 * dx);
    D1[(size_t)i * d + im] -= 1.0 / (2 * dx);
    D2[(size_t)i * d + i] -= 2.0 / (dx * dx);
    D2[(size_t)i * d + ip] += 1.0 / (dx * dx);
    D2[(size_t)i * d + im] += 1.0 / (dx * dx);
  }
  for (double& v : D1)
    if (std::fabs(v) < 1e-12) v = 0.0;
  for (double& v : D2)
    if (std::fabs(v) < 1e-12) v = 0.0;
  op->B.clear();
  op->D = D2;
  std::vector<Term> terms;
  auto one = [&](int i, int o, double c) {
    if (c == 0.0) return;
    Term t;
    t.coef = cplx(c, 0.0);
    t.ops.push_back({i, o});
    terms.push_back(t);
  };
  auto two = [&](int i, int oi, int j, int oj, double c) {
    if (c == 0.0) return;
    Term t;
    t.coef = cplx(c, 0.0);
    if (i < j) {
      t.ops.push_back({i, oi});
      t.ops.push_back({j, oj});
    } else {
      t.ops.push_back({j, oj});
      t.ops.push_back({i, oi});
    }
    terms.push_back(t);
  };
  for (int i = 0; i < d; ++i) {
    one(i, OP_XG, -gamma * D2[(size_t)i * d + i]);
    one(i, OP_SG, -alpha);
    if (op->diff != 0.0) one(i, OP_L2, op->diff);
    for (int j = 0; j < d; ++j) {
      if (j == i) continue;
      two(i, OP_XG, j, OP_K, D1[(size_t)i * d + j]);
      two(i, OP_G, j, OP_K, -gamma * D2[(size_t)i * d + j]);
    }
  }
  if (terms.empty()) fail(TT_EINVAL, "CDF operator without terms (gamma, alpha and the advection all vanish)");
  build_automaton(op, terms);
}

}  // namespace ttf
