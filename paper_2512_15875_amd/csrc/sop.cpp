// Host-side operator compiler: sum-of-products Hamiltonian -> TTNO (FP64).
//
// The paper compiles Eq. sum_of_tp into a TTNO through a compressed state
// diagram (Sec. II.A.3).  Any exact TTNO represents the same operator; this
// compiler builds one from a channel automaton and then compresses every bond
// to the operator Schmidt rank with SVDs:
//
//  * across the edge above node u, a term is either untouched inside the
//    subtree of u ("identity" channel), finished inside it ("done" channel,
//    carrying its coefficient), or split, in which case the channel is the
//    distinct partial operator product inside the subtree;
//  * node tensors route channels (identity -> identity, one child's done ->
//    done, children partials x local factor -> parent partial, or -> done with
//    the coefficient at the lowest node holding the whole term);
//  * compression: Householder QR from the leaves to the root, then a
//    root-to-leaves sweep of one-sided Jacobi SVDs that keeps singular values
//    above rel_tol * sigma_max, moving the orthogonality centre with the sweep.
//
// Per-mode operators live in the harmonic-oscillator basis |0>..|d-1>:
// n = diag(0..d-1) (the on-site term omega*n is the harmonic part with the
// zero-point energy removed) and q^k = the d x d block of (Q_{d+k})^k with
// Q_m the position matrix in a basis of size m (an exact projection).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "internal.h"

struct ttn_sop {
  int n = 0;
  std::vector<int> bond;                // per edge e(u)
  std::vector<std::vector<int>> shape;  // legs of W[u]
  std::vector<std::vector<double>> W;
};

namespace {

typedef std::vector<double> Vec;

struct Mat {  // row-major dense matrix
  int r = 0, c = 0;
  Vec a;
  Mat() {}
  Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      const double x = A(i, k);
      if (x == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += x * B(k, j);
    }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

// ---- per-mode operators
Mat pos_matrix(int m) {
  Mat q(m, m);
  for (int k = 1; k < m; ++k) q(k - 1, k) = q(k, k - 1) = std::sqrt(k / 2.0);
  return q;
}

Mat qpow(int d, int k) {
  Mat Q = pos_matrix(d + k);
  Mat P(d + k, d + k);
  for (int i = 0; i < d + k; ++i) P(i, i) = 1.0;
  for (int t = 0; t < k; ++t) P = matmul(P, Q);
  Mat out(d, d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) out(i, j) = P(i, j);
  return out;
}

// ---- thin Householder QR: A (m x n, m >= n) = Q (m x n) R (n x n), diag(R) >= 0
void householder_qr(const Mat& A, Mat& Q, Mat& R) {
  const int m = A.r, n = A.c;
  Mat W = A;
  std::vector<Vec> vs;
  std::vector<double> taus;
  const int kmax = std::min(m, n);
  for (int k = 0; k < kmax; ++k) {
    double nrm = 0;
    for (int i = k; i < m; ++i) nrm += W(i, k) * W(i, k);
    nrm = std::sqrt(nrm);
    Vec v(m, 0.0);
    if (nrm == 0.0) {
      vs.push_back(v);
      taus.push_back(0.0);
      continue;
    }
    const double alpha = W(k, k) >= 0 ? -nrm : nrm;
    for (int i = k; i < m; ++i) v[i] = W(i, k);
    v[k] -= alpha;
    double vn = 0;
    for (int i = k; i < m; ++i) vn += v[i] * v[i];
    const double tau = vn > 0 ? 2.0 / vn : 0.0;
    for (int j = k; j < n; ++j) {
      double s = 0;
      for (int i = k; i < m; ++i) s += v[i] * W(i, j);
      s *= tau;
      for (int i = k; i < m; ++i) W(i, j) -= s * v[i];
    }
    vs.push_back(v);
    taus.push_back(tau);
  }
  R = Mat(kmax, n);
  for (int i = 0; i < kmax; ++i)
    for (int j = i; j < n; ++j) R(i, j) = W(i, j);
  // Q = H_0 H_1 ... applied to the first kmax unit columns
  Q = Mat(m, kmax);
  for (int j = 0; j < kmax; ++j) Q(j, j) = 1.0;
  for (int k = kmax - 1; k >= 0; --k) {
    const Vec& v = vs[k];
    const double tau = taus[k];
    if (tau == 0.0) continue;
    for (int j = 0; j < kmax; ++j) {
      double s = 0;
      for (int i = k; i < m; ++i) s += v[i] * Q(i, j);
      s *= tau;
      for (int i = k; i < m; ++i) Q(i, j) -= s * v[i];
    }
  }
  for (int i = 0; i < kmax; ++i)
    if (R(i, i) < 0) {
      for (int j = 0; j < n; ++j) R(i, j) = -R(i, j);
      for (int r = 0; r < m; ++r) Q(r, i) = -Q(r, i);
    }
}

// ---- one-sided Jacobi SVD: A (m x n) = U diag(s) V^T, s descending
void jacobi_svd(const Mat& Ain, Mat& U, Vec& s, Mat& Vt) {
  const bool tr = Ain.r < Ain.c;
  Mat A = tr ? transpose(Ain) : Ain;  // m >= n
  const int m = A.r, n = A.c;
  Mat V(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  // work on columns: store A column-major for locality
  std::vector<Vec> col(n, Vec(m));
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) col[j][i] = A(i, j);
  std::vector<Vec> vcol(n, Vec(n, 0.0));
  for (int j = 0; j < n; ++j) vcol[j][j] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0, b = 0, g = 0;
        for (int i = 0; i < m; ++i) {
          a += col[p][i] * col[p][i];
          b += col[q][i] * col[q][i];
          g += col[p][i] * col[q][i];
        }
        if (std::fabs(g) <= 1e-15 * std::sqrt(a * b) || g == 0.0) continue;
        off = std::max(off, std::fabs(g) / std::sqrt(a * b));
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = col[p][i], y = col[q][i];
          col[p][i] = c * x - sn * y;
          col[q][i] = sn * x + c * y;
        }
        for (int i = 0; i < n; ++i) {
          const double x = vcol[p][i], y = vcol[q][i];
          vcol[p][i] = c * x - sn * y;
          vcol[q][i] = sn * x + c * y;
        }
      }
    if (off < 1e-15) break;
  }
  std::vector<std::pair<double, int>> sv(n);
  for (int j = 0; j < n; ++j) {
    double nn = 0;
    for (int i = 0; i < m; ++i) nn += col[j][i] * col[j][i];
    sv[j] = {std::sqrt(nn), j};
  }
  std::sort(sv.begin(), sv.end(), [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
    return x.first > y.first;
  });
  Mat Uo(m, n), Vo(n, n);
  s.assign(n, 0.0);
  for (int r = 0; r < n; ++r) {
    const int j = sv[r].second;
    s[r] = sv[r].first;
    for (int i = 0; i < m; ++i) Uo(i, r) = s[r] > 0 ? col[j][i] / s[r] : 0.0;
    for (int i = 0; i < n; ++i) Vo(i, r) = vcol[j][i];
  }
  if (!tr) {
    U = Uo;
    Vt = transpose(Vo);
  } else {  // A^T = Uo s Vo^T  ->  A = Vo s Uo^T
    U = Vo;
    Vt = transpose(Uo);
  }
}

// ---- dense tensor helpers (row-major, shape vector)
struct Tens {
  std::vector<int> sh;
  Vec a;
  int64_t size() const {
    int64_t s = 1;
    for (int x : sh) s *= x;
    return s;
  }
};

// move axis `ax` to the last position
Tens move_last(const Tens& T, int ax) {
  const int nd = (int)T.sh.size();
  std::vector<int> perm;
  for (int i = 0; i < nd; ++i)
    if (i != ax) perm.push_back(i);
  perm.push_back(ax);
  Tens O;
  for (int p : perm) O.sh.push_back(T.sh[p]);
  O.a.assign(T.a.size(), 0.0);
  std::vector<int64_t> st(nd, 1);
  for (int i = nd - 2; i >= 0; --i) st[i] = st[i + 1] * T.sh[i + 1];
  std::vector<int> idx(nd, 0);
  const int64_t n = T.size();
  for (int64_t o = 0; o < n; ++o) {
    int64_t src = 0;
    for (int i = 0; i < nd; ++i) src += (int64_t)idx[i] * st[perm[i]];
    O.a[(size_t)o] = T.a[(size_t)src];
    for (int i = nd - 1; i >= 0; --i) {
      if (++idx[i] < O.sh[i]) break;
      idx[i] = 0;
    }
  }
  return O;
}

// inverse of move_last: last axis back to position ax
Tens move_from_last(const Tens& T, int ax) {
  const int nd = (int)T.sh.size();
  // build perm such that output axis i takes input axis perm[i]
  std::vector<int> perm;
  for (int i = 0, j = 0; i < nd; ++i) {
    if (i == ax) perm.push_back(nd - 1);
    else perm.push_back(j++);
  }
  Tens O;
  for (int p : perm) O.sh.push_back(T.sh[p]);
  O.a.assign(T.a.size(), 0.0);
  std::vector<int64_t> st(nd, 1);
  for (int i = nd - 2; i >= 0; --i) st[i] = st[i + 1] * T.sh[i + 1];
  std::vector<int> idx(nd, 0);
  const int64_t n = T.size();
  for (int64_t o = 0; o < n; ++o) {
    int64_t src = 0;
    for (int i = 0; i < nd; ++i) src += (int64_t)idx[i] * st[perm[i]];
    O.a[(size_t)o] = T.a[(size_t)src];
    for (int i = nd - 1; i >= 0; --i) {
      if (++idx[i] < O.sh[i]) break;
      idx[i] = 0;
    }
  }
  return O;
}

// contract axis ax of T (dim old) with R[new][old]  -> axis ax has dim new
Tens absorb(const Tens& T, int ax, const Mat& R) {
  Tens L = move_last(T, ax);
  const int old = L.sh.back();
  const int64_t rows = L.size() / old;
  Tens O;
  O.sh = L.sh;
  O.sh.back() = R.r;
  O.a.assign((size_t)rows * R.r, 0.0);
  for (int64_t i = 0; i < rows; ++i)
    for (int nw = 0; nw < R.r; ++nw) {
      double s = 0;
      for (int o = 0; o < old; ++o) s += L.a[(size_t)(i * old + o)] * R(nw, o);
      O.a[(size_t)(i * R.r + nw)] = s;
    }
  return move_from_last(O, ax);
}

}  // namespace

extern "C" ttn_status ttn_sop_build(const ttn_tree* t, const int32_t* node_mode, int32_t n_modes, const double* omega,
                                    const int32_t* dims, int32_t n_mono, const int32_t* mono_ptr,
                                    const int32_t* mono_mode, const int32_t* mono_pow, const double* coef,
                                    double rel_tol, ttn_sop** out) {
  if (!t || !node_mode || !omega || !dims || !out || n_modes < 1 || n_mono < 0 || (n_mono > 0 && (!mono_ptr || !mono_mode || !mono_pow || !coef)))
    return TTN_E_ARG;
  const int n = t->n;
  std::vector<int> node_of(n_modes, -1);
  for (int u = 0; u < n; ++u) {
    const int m = node_mode[u];
    if (m >= n_modes) return TTN_E_ARG;
    if (m >= 0) {
      if (node_of[m] >= 0 || t->phys[u] != dims[m]) return TTN_E_SHAPE;
      node_of[m] = u;
    } else if (t->phys[u] != 1) {
      return TTN_E_SHAPE;
    }
  }
  for (int m = 0; m < n_modes; ++m)
    if (node_of[m] < 0) return TTN_E_ARG;
  // terms: (coef, sorted list of (mode, key)); key -1 = number operator, k>0 = q^k
  struct Term {
    double c;
    std::vector<std::pair<int, int>> f;
  };
  std::vector<Term> terms;
  for (int m = 0; m < n_modes; ++m) terms.push_back({omega[m], {{m, -1}}});
  for (int i = 0; i < n_mono; ++i) {
    Term tm;
    tm.c = coef[i];
    for (int j = mono_ptr[i]; j < mono_ptr[i + 1]; ++j) {
      if (mono_mode[j] < 0 || mono_mode[j] >= n_modes || mono_pow[j] < 1) return TTN_E_ARG;
      tm.f.push_back({mono_mode[j], mono_pow[j]});
    }
    std::sort(tm.f.begin(), tm.f.end());
    for (size_t j = 1; j < tm.f.size(); ++j)
      if (tm.f[j].first == tm.f[j - 1].first) return TTN_E_ARG;  // one factor per mode
    if (tm.f.empty()) return TTN_E_ARG;
    terms.push_back(tm);
  }
  // subtree membership
  std::vector<std::vector<char>> in_sub(n, std::vector<char>(n, 0));
  for (int u = 0; u < n; ++u) {
    int x = u;
    while (x >= 0) {
      in_sub[x][u] = 1;
      x = t->parent[x];
    }
  }
  typedef std::vector<std::pair<int, int>> Part;
  auto restrict_to = [&](const Part& f, int u) {
    Part p;
    for (auto& x : f)
      if (in_sub[u][node_of[x.first]]) p.push_back(x);
    return p;
  };
  // channel dictionaries per edge e(u)
  std::vector<std::map<Part, int>> chan(n);
  for (int u = 0; u < n; ++u) {
    if (u == t->root) continue;
    std::set<Part> parts;
    for (auto& tm : terms) {
      Part p = restrict_to(tm.f, u);
      if (!p.empty() && p.size() != tm.f.size()) parts.insert(p);
    }
    int id = 2;
    for (auto& p : parts) chan[u][p] = id++;
  }
  auto label = [&](const Term& tm, int c) -> int {  // channel of a term on the edge above c
    Part p = restrict_to(tm.f, c);
    if (p.empty()) return 0;
    if (p.size() == tm.f.size()) return 1;
    return chan[c].at(p);
  };
  auto lowest_holder = [&](const Term& tm) {
    int u = node_of[tm.f[0].first];
    for (;;) {
      bool all = true;
      for (auto& x : tm.f)
        if (!in_sub[u][node_of[x.first]]) all = false;
      if (all) return u;
      u = t->parent[u];
    }
  };
  std::map<std::pair<int, int>, Mat> opcache;
  auto local_op = [&](int mode, int key) -> const Mat& {
    auto k = std::make_pair(mode, key);
    auto it = opcache.find(k);
    if (it != opcache.end()) return it->second;
    const int d = dims[mode];
    Mat M(d, d);
    if (key < 0) {
      for (int i = 0; i < d; ++i) M(i, i) = (double)i;  // number operator (omega is the term coefficient)
    } else {
      M = qpow(d, key);
    }
    return opcache[k] = M;
  };
  // automaton tensors
  std::vector<Tens> W(n);
  for (int u = 0; u < n; ++u) {
    Tens T;
    const bool hp = u != t->root;
    if (hp) T.sh.push_back((int)chan[u].size() + 2);
    for (int c : t->ch[u]) T.sh.push_back((int)chan[c].size() + 2);
    const int d = t->phys[u];
    T.sh.push_back(d);
    T.sh.push_back(d);
    T.a.assign((size_t)T.size(), 0.0);
    std::vector<int64_t> st(T.sh.size(), 1);
    for (int i = (int)T.sh.size() - 2; i >= 0; --i) st[i] = st[i + 1] * T.sh[i + 1];
    const int nch = (int)t->ch[u].size();
    const int coff = hp ? 1 : 0;
    auto put = [&](int par, const std::vector<int>& chs, const Mat* op, double cf) {
      int64_t base = 0;
      if (hp) base += (int64_t)par * st[0];
      for (int i = 0; i < nch; ++i) base += (int64_t)chs[i] * st[coff + i];
      const int64_t sp = st[coff + nch], sq = st[coff + nch + 1];
      for (int p = 0; p < d; ++p)
        for (int q = 0; q < d; ++q) {
          const double v = op ? (*op)(p, q) : (p == q ? 1.0 : 0.0);
          T.a[(size_t)(base + p * sp + q * sq)] += cf * v;
        }
    };
    std::vector<int> zeros(nch, 0);
    if (hp) put(0, zeros, nullptr, 1.0);
    for (int i = 0; i < nch; ++i) {
      std::vector<int> chs(zeros);
      chs[i] = 1;
      put(1, chs, nullptr, 1.0);
    }
    const int my = node_mode[u];
    for (auto& tm : terms) {
      if (lowest_holder(tm) != u) continue;
      std::vector<int> chs;
      for (int c : t->ch[u]) chs.push_back(label(tm, c));
      const Mat* op = nullptr;
      for (auto& x : tm.f)
        if (x.first == my) op = &local_op(my, x.second);
      put(1, chs, op, tm.c);
    }
    if (hp) {
      for (auto& kv : chan[u]) {
        std::vector<int> chs;
        for (int c : t->ch[u]) {
          Part p;
          for (auto& x : kv.first)
            if (in_sub[c][node_of[x.first]]) p.push_back(x);
          chs.push_back(p.empty() ? 0 : chan[c].at(p));
        }
        const Mat* op = nullptr;
        for (auto& x : kv.first)
          if (x.first == my) op = &local_op(my, x.second);
        put(kv.second, chs, op, 1.0);
      }
    }
    W[u] = T;
  }
  // compression: post-order QR toward the root
  std::vector<int> post;
  {
    std::vector<std::pair<int, int>> stk{{t->root, 0}};
    while (!stk.empty()) {
      auto& top = stk.back();
      if (top.second < (int)t->ch[top.first].size()) {
        const int c = t->ch[top.first][top.second++];
        stk.push_back({c, 0});
      } else {
        post.push_back(top.first);
        stk.pop_back();
      }
    }
  }
  auto leg_in_parent = [&](int p, int c) {
    const int off = p != t->root ? 1 : 0;
    for (size_t i = 0; i < t->ch[p].size(); ++i)
      if (t->ch[p][i] == c) return off + (int)i;
    return -1;
  };
  auto qr_toward_parent = [&](int u) {
    Tens L = move_last(W[u], 0);
    const int Mp = L.sh.back();
    const int rows = (int)(L.size() / Mp);
    Mat A(rows, Mp);
    A.a = L.a;
    Mat Q, R;
    if (rows >= Mp) {
      householder_qr(A, Q, R);
    } else {  // wide: keep as is (Q = A, R = I) with the smaller bond
      Mat U, Vt;
      Vec s;
      jacobi_svd(A, U, s, Vt);
      Q = U;
      R = Mat(U.c, Mp);
      for (int i = 0; i < U.c; ++i)
        for (int j = 0; j < Mp; ++j) R(i, j) = s[i] * Vt(i, j);
    }
    Tens N;
    N.sh = L.sh;
    N.sh.back() = Q.c;
    N.a = Q.a;
    W[u] = move_from_last(N, 0);
    const int p = t->parent[u];
    W[p] = absorb(W[p], leg_in_parent(p, u), R);
  };
  for (int u : post)
    if (u != t->root) qr_toward_parent(u);
  // sweep down with SVD truncation (iterative DFS)
  std::vector<int> bond(n, 0);
  std::vector<std::pair<int, int>> stk{{t->root, 0}};
  while (!stk.empty()) {
    auto& top = stk.back();
    const int u = top.first;
    if (top.second < (int)t->ch[u].size()) {
      const int c = t->ch[u][top.second++];
      const int leg = leg_in_parent(u, c);
      Tens L = move_last(W[u], leg);
      const int Mc = L.sh.back();
      const int rows = (int)(L.size() / Mc);
      Mat A(rows, Mc);
      A.a = L.a;
      Mat U, Vt;
      Vec s;
      jacobi_svd(A, U, s, Vt);
      int keep = 0;
      for (double x : s)
        if (s[0] > 0 && x > rel_tol * s[0]) ++keep;
      keep = std::max(keep, 1);
      Tens N;
      N.sh = L.sh;
      N.sh.back() = keep;
      N.a.assign((size_t)rows * keep, 0.0);
      for (int i = 0; i < rows; ++i)
        for (int j = 0; j < keep; ++j) N.a[(size_t)i * keep + j] = U(i, j);
      W[u] = move_from_last(N, leg);
      Mat SV(keep, Mc);
      for (int i = 0; i < keep; ++i)
        for (int j = 0; j < Mc; ++j) SV(i, j) = s[i] * Vt(i, j);
      W[c] = absorb(W[c], 0, SV);
      bond[c] = keep;
      stk.push_back({c, 0});
    } else {
      stk.pop_back();
      if (u != t->root) {
        // centre back to the parent
        const int p = t->parent[u];
        Tens L = move_last(W[u], 0);
        const int Mp = L.sh.back();
        const int rows = (int)(L.size() / Mp);
        Mat A(rows, Mp);
        A.a = L.a;
        if (rows >= Mp) {
          Mat Q, R;
          householder_qr(A, Q, R);
          Tens N;
          N.sh = L.sh;
          N.a = Q.a;
          W[u] = move_from_last(N, 0);
          W[p] = absorb(W[p], leg_in_parent(p, u), R);
        }
      }
    }
  }
  ttn_sop* S = new (std::nothrow) ttn_sop();
  if (!S) return TTN_E_ARG;
  S->n = n;
  S->bond = bond;
  for (int u = 0; u < n; ++u) {
    S->shape.push_back(W[u].sh);
    S->W.push_back(W[u].a);
  }
  *out = S;
  return TTN_OK;
}

// ---------------------------------------------------------------- state diagram
//
// The state-diagram construction of Sec. II.A.3: leaves to root, every item (a
// term, or a group of terms merged further down) is an edge of the bipartite
// graph between its descriptor inside the subtree (operator at the node, or the
// identity, and its channel on each child edge) and its operator string outside
// the subtree.  A minimum vertex cover (Konig's construction from a maximum
// matching by augmenting paths; left vertices in order of first appearance,
// neighbours in order) gives the edge's channels: a covered descriptor is a
// coefficient-free channel, a covered outside string carries the sum of
// coefficient x descriptor of its items, which merge there into one item of
// coefficient 1 (the coefficients are placed once).  Items merged in another
// branch must reach the edge through a coefficient-free channel (forced into the
// cover).  Channels: covered descriptors in order of first appearance, then
// covered strings.  The root sums what is left.  No compression: the tensors
// keep the diagram's sparsity.

namespace {

// minimum vertex cover containing the forced left vertices (returns sorted lists)
void min_vertex_cover(int nl, int nr, const std::vector<std::vector<int>>& adj, const std::vector<char>& forced,
                      std::vector<int>& cl, std::vector<int>& cr) {
  std::vector<std::vector<int>> a2(nl);
  for (int l = 0; l < nl; ++l)
    if (!forced[l]) a2[l] = adj[l];
  std::vector<int> ml(nl, -1), mr(nr, -1);
  for (int l0 = 0; l0 < nl; ++l0) {
    if (a2[l0].empty()) continue;
    std::vector<char> seen(nr, 0);
    std::vector<std::pair<int, int>> stk{{l0, 0}}, path;
    bool found = false;
    while (!stk.empty() && !found) {
      const int l = stk.back().first, i = stk.back().second;
      if (i >= (int)a2[l].size()) {
        stk.pop_back();
        if (!path.empty()) path.pop_back();
        continue;
      }
      stk.back().second = i + 1;
      const int r = a2[l][i];
      if (seen[r]) continue;
      seen[r] = 1;
      path.push_back({l, r});
      if (mr[r] < 0) found = true;
      else stk.push_back({mr[r], 0});
    }
    if (found)
      for (auto& pr : path) {
        ml[pr.first] = pr.second;
        mr[pr.second] = pr.first;
      }
  }
  std::vector<char> vl(nl, 0), vr(nr, 0);
  std::vector<int> stk;
  for (int l = 0; l < nl; ++l)
    if (ml[l] < 0 && !a2[l].empty()) {
      vl[l] = 1;
      stk.push_back(l);
    }
  while (!stk.empty()) {
    const int l = stk.back();
    stk.pop_back();
    for (int r : a2[l])
      if (!vr[r] && ml[l] != r) {
        vr[r] = 1;
        const int l2 = mr[r];
        if (l2 >= 0 && !vl[l2]) {
          vl[l2] = 1;
          stk.push_back(l2);
        }
      }
  }
  cl.clear();
  cr.clear();
  for (int l = 0; l < nl; ++l)
    if (forced[l] || (!a2[l].empty() && !vl[l])) cl.push_back(l);
  for (int r = 0; r < nr; ++r)
    if (vr[r]) cr.push_back(r);
}

}  // namespace

extern "C" ttn_status ttn_sop_build_sd(const ttn_tree* t, const int32_t* node_mode, int32_t n_modes,
                                       const double* omega, const int32_t* dims, int32_t n_mono,
                                       const int32_t* mono_ptr, const int32_t* mono_mode, const int32_t* mono_pow,
                                       const double* coef, ttn_sop** out) {
  if (!t || !node_mode || !omega || !dims || !out || n_modes < 1 || n_mono < 0 ||
      (n_mono > 0 && (!mono_ptr || !mono_mode || !mono_pow || !coef)))
    return TTN_E_ARG;
  const int n = t->n;
  std::vector<int> node_of(n_modes, -1);
  for (int u = 0; u < n; ++u) {
    const int m = node_mode[u];
    if (m >= n_modes) return TTN_E_ARG;
    if (m >= 0) {
      if (node_of[m] >= 0 || t->phys[u] != dims[m]) return TTN_E_SHAPE;
      node_of[m] = u;
    } else if (t->phys[u] != 1) {
      return TTN_E_SHAPE;
    }
  }
  for (int m = 0; m < n_modes; ++m)
    if (node_of[m] < 0) return TTN_E_ARG;
  typedef std::vector<std::pair<int, int>> Part;  // sorted (mode, key); key -1 = n, k > 0 = q^k
  struct Item {
    Part ops;
    double c;
    int merged_at;
    std::map<int, int> chan;
  };
  std::vector<Item> items;
  // the on-site term of mode m: coefficient 1, operator omega_m n (as the oracle writes it)
  for (int m = 0; m < n_modes; ++m) items.push_back({{{m, -1}}, 1.0, -1, {}});
  for (int i = 0; i < n_mono; ++i) {
    Item it;
    it.c = coef[i];
    it.merged_at = -1;
    for (int j = mono_ptr[i]; j < mono_ptr[i + 1]; ++j) {
      if (mono_mode[j] < 0 || mono_mode[j] >= n_modes || mono_pow[j] < 1) return TTN_E_ARG;
      it.ops.push_back({mono_mode[j], mono_pow[j]});
    }
    std::sort(it.ops.begin(), it.ops.end());
    for (size_t j = 1; j < it.ops.size(); ++j)
      if (it.ops[j].first == it.ops[j - 1].first) return TTN_E_ARG;
    if (it.ops.empty()) return TTN_E_ARG;
    items.push_back(it);
  }
  std::vector<std::vector<char>> in_sub(n, std::vector<char>(n, 0));
  for (int u = 0; u < n; ++u)
    for (int x = u; x >= 0; x = t->parent[x]) in_sub[x][u] = 1;
  std::vector<int> post;
  {
    std::vector<std::pair<int, int>> stk{{t->root, 0}};
    while (!stk.empty()) {
      auto& top = stk.back();
      if (top.second < (int)t->ch[top.first].size()) {
        const int c = t->ch[top.first][top.second++];
        stk.push_back({c, 0});
      } else {
        post.push_back(top.first);
        stk.pop_back();
      }
    }
  }
  std::map<std::pair<int, int>, Mat> opcache;
  auto local_op = [&](int mode, int key) -> const Mat& {
    auto k = std::make_pair(mode, key);
    auto it = opcache.find(k);
    if (it != opcache.end()) return it->second;
    const int d = dims[mode];
    Mat M(d, d);
    if (key < 0) {
      for (int i = 0; i < d; ++i) M(i, i) = omega[mode] * (double)i;
    } else {
      M = qpow(d, key);
    }
    return opcache[k] = M;
  };
  const int NOKEY = INT32_MIN;
  std::vector<int> bond(n, 0);
  std::vector<Tens> W(n);
  typedef std::pair<int, std::vector<int>> Desc;
  for (int u : post) {
    const auto& ch = t->ch[u];
    const int d = t->phys[u], my = node_mode[u];
    const bool hp = u != t->root;
    std::vector<Desc> desc(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
      int key = NOKEY;
      if (my >= 0)
        for (auto& x : items[i].ops)
          if (x.first == my) key = x.second;
      std::vector<int> chs;
      for (int c : ch) chs.push_back(items[i].chan.at(c));
      desc[i] = {key, chs};
    }
    // the tensor: [parent channel?, children channels..., p, q]
    auto alloc_tensor = [&](int M) {
      Tens T;
      if (hp) T.sh.push_back(M);
      for (int c : ch) T.sh.push_back(bond[c]);
      T.sh.push_back(d);
      T.sh.push_back(d);
      T.a.assign((size_t)T.size(), 0.0);
      return T;
    };
    auto put = [&](Tens& T, int par, const Desc& ds, double cf) {
      std::vector<int64_t> st(T.sh.size(), 1);
      for (int i = (int)T.sh.size() - 2; i >= 0; --i) st[i] = st[i + 1] * T.sh[i + 1];
      const int off = hp ? 1 : 0;
      int64_t base = hp ? (int64_t)par * st[0] : 0;
      for (size_t i = 0; i < ch.size(); ++i) base += (int64_t)ds.second[i] * st[off + i];
      const int64_t sp = st[off + ch.size()], sq = st[off + ch.size() + 1];
      const Mat* op = ds.first == NOKEY ? nullptr : &local_op(my, ds.first);
      for (int p = 0; p < d; ++p)
        for (int q = 0; q < d; ++q) {
          const double v = op ? (*op)(p, q) : (p == q ? 1.0 : 0.0);
          T.a[(size_t)(base + p * sp + q * sq)] += cf * v;
        }
    };
    if (!hp) {
      Tens T = alloc_tensor(0);
      for (size_t i = 0; i < items.size(); ++i) put(T, 0, desc[i], items[i].c);
      W[u] = T;
      break;
    }
    std::vector<Part> rights(items.size());
    for (size_t i = 0; i < items.size(); ++i)
      for (auto& x : items[i].ops)
        if (!in_sub[u][node_of[x.first]]) rights[i].push_back(x);
    std::map<Desc, int> lid;
    std::map<Part, int> rid;
    std::vector<const Desc*> lvec;
    std::vector<int> li(items.size()), ri(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
      auto a = lid.emplace(desc[i], (int)lid.size());
      if (a.second) lvec.push_back(&a.first->first);
      li[i] = a.first->second;
      ri[i] = rid.emplace(rights[i], (int)rid.size()).first->second;
    }
    const int nl = (int)lid.size(), nr = (int)rid.size();
    std::vector<std::vector<int>> adj(nl);
    for (size_t i = 0; i < items.size(); ++i)
      if (std::find(adj[li[i]].begin(), adj[li[i]].end(), ri[i]) == adj[li[i]].end()) adj[li[i]].push_back(ri[i]);
    std::vector<char> forced(nl, 0);
    for (size_t i = 0; i < items.size(); ++i)
      if (items[i].merged_at >= 0 && !in_sub[u][items[i].merged_at]) forced[li[i]] = 1;
    std::vector<int> cl, cr;
    min_vertex_cover(nl, nr, adj, forced, cl, cr);
    std::vector<int> chan_l(nl, -1), chan_r(nr, -1);
    for (size_t i = 0; i < cl.size(); ++i) chan_l[cl[i]] = (int)i;
    for (size_t i = 0; i < cr.size(); ++i) chan_r[cr[i]] = (int)(cl.size() + i);
    const int M = (int)(cl.size() + cr.size());
    bond[u] = M;
    Tens T = alloc_tensor(M);
    for (int l : cl) put(T, chan_l[l], *lvec[l], 1.0);
    std::vector<Item> next;
    std::map<int, size_t> merged;  // right vertex -> index in next
    for (size_t i = 0; i < items.size(); ++i) {
      if (chan_l[li[i]] >= 0) {
        Item it = items[i];
        it.chan[u] = chan_l[li[i]];
        next.push_back(std::move(it));
        continue;
      }
      const int r = ri[i];
      if (chan_r[r] < 0) return TTN_E_ARG;  // not a cover (cannot happen)
      put(T, chan_r[r], desc[i], items[i].c);
      if (!merged.count(r)) {
        Item g;
        g.ops = rights[i];
        g.c = 1.0;
        g.merged_at = u;
        for (auto& kv : items[i].chan)
          if (!in_sub[u][kv.first]) g.chan[kv.first] = kv.second;
        g.chan[u] = chan_r[r];
        merged[r] = next.size();
        next.push_back(std::move(g));
      }
    }
    items.swap(next);
    W[u] = T;
  }
  ttn_sop* S = new (std::nothrow) ttn_sop();
  if (!S) return TTN_E_ARG;
  S->n = n;
  S->bond = bond;
  for (int u = 0; u < n; ++u) {
    S->shape.push_back(W[u].sh);
    S->W.push_back(W[u].a);
  }
  *out = S;
  return TTN_OK;
}

extern "C" ttn_status ttn_sop_bonds(const ttn_sop* s, int32_t* op_bond) {
  if (!s || !op_bond) return TTN_E_ARG;
  for (int u = 0; u < s->n; ++u) op_bond[u] = s->bond[u];
  return TTN_OK;
}

extern "C" ttn_status ttn_sop_tensor(const ttn_sop* s, int32_t u, double* out, int64_t cap) {
  if (!s || !out || u < 0 || u >= s->n) return TTN_E_ARG;
  if ((int64_t)s->W[u].size() > cap) return TTN_E_SHAPE;
  std::memcpy(out, s->W[u].data(), s->W[u].size() * sizeof(double));
  return TTN_OK;
}

extern "C" ttn_status ttn_sop_destroy(ttn_sop* s) {
  delete s;
  return TTN_OK;
}
