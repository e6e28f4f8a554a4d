// Contraction planner: minimum-flop pairwise order for the small tensor
// networks of the hot path (a node's operands: state tensor(s), TTNO tensor,
// up to four environments), then one offset-table GEMM per pairwise stage.
//
// Cost model: a pairwise contraction of operands with index sets I and J
// costs 2 * prod(dims of I u J) per batch item when either operand is batched
// (depends on the state or pair), or once per call when both are shared.
// Every index of these networks appears in exactly two places (two operands,
// or one operand and the output), so the indices shared by a pair are exactly
// the contracted ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdlib>
#include <limits>

#include "internal.h"

namespace ttn {

namespace {

struct Node {
  std::vector<int> lab;  // sorted labels
  int batched;
};

std::vector<int> sym_diff(const std::vector<int>& a, const std::vector<int>& b) {
  std::vector<int> out;
  std::set_symmetric_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}
std::vector<int> uni(const std::vector<int>& a, const std::vector<int>& b) {
  std::vector<int> out;
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}

struct Search {
  const std::map<int, int>* dims;
  double batch;
  double best = std::numeric_limits<double>::infinity();
  double best_mem = std::numeric_limits<double>::infinity();
  std::vector<std::pair<int, int>> best_seq, cur;

  double prodd(const std::vector<int>& l) const {
    double p = 1;
    for (int x : l) p *= dims->at(x);
    return p;
  }
  void rec(std::vector<Node>& ns, double cost, double mem) {
    if (cost > best * (1 + 1e-12)) return;
    if (ns.size() == 1) {
      if (cost < best * (1 - 1e-12) || (cost <= best * (1 + 1e-12) && mem < best_mem)) {
        best = cost;
        best_mem = mem;
        best_seq = cur;
      }
      return;
    }
    for (size_t i = 0; i < ns.size(); ++i)
      for (size_t j = i + 1; j < ns.size(); ++j) {
        Node a = ns[i], b = ns[j];
        const bool bat = a.batched || b.batched;
        const double c = 2.0 * prodd(uni(a.lab, b.lab)) * (bat ? batch : 1.0);
        Node r{sym_diff(a.lab, b.lab), bat ? 1 : 0};
        const double m2 = std::max(mem, prodd(r.lab) * (bat ? batch : 1.0));
        std::vector<Node> nx;
        for (size_t t = 0; t < ns.size(); ++t)
          if (t != i && t != j) nx.push_back(ns[t]);
        nx.push_back(r);
        cur.push_back({(int)i, (int)j});
        rec(nx, cost + c, m2);
        cur.pop_back();
      }
  }
};

// mixed-radix offsets of a label group: last label fastest
void group_offsets(const std::vector<int>& labs, const std::map<int, int>& dims,
                   const std::map<int, int64_t>& stride, std::vector<int32_t>& out) {
  int64_t n = 1;
  for (int l : labs) n *= dims.at(l);
  out.assign((size_t)n, 0);
  std::vector<int> digit(labs.size(), 0);
  for (int64_t t = 0; t < n; ++t) {
    int64_t off = 0;
    for (size_t i = 0; i < labs.size(); ++i) off += (int64_t)digit[i] * stride.at(labs[i]);
    out[(size_t)t] = (int32_t)off;
    for (int i = (int)labs.size() - 1; i >= 0; --i) {
      if (++digit[i] < dims.at(labs[i])) break;
      digit[i] = 0;
    }
  }
}

int pick_tile(int M, int N, int K, double nblocks_other, bool tn) {
  // tiny per-item products over many items: one wave per item (tile id 7).
  // Measured on the fitting environments it does not beat the 32x32 tile
  // (those stages are bound by their intermediates' memory traffic), so it is
  // only used when requested.
  static const int wave_on = getenv("TTN_WAVE_KERNEL") ? 1 : 0;
  if (wave_on && nblocks_other >= 256 && (double)M * N <= 64.0 * 64.0 && K <= 4096) return 7;
  // a short contraction (K <= 64) whose output is at least 32 x 33: the
  // general 64 x 64 tile.  The autotuner picks it on both benchmark
  // workloads over the unit-stride-k tiles (1600 x 40 x 40 stages of the
  // 12-mode tree: 2.05 -> 1.58 ms; 1600 x 720 x 40: 1.07 -> 0.81 ms) and over
  // the 64 x 32 tile that fits N = 96 or 216 without padding (576 x 96 x 24:
  // 440 -> 390 us): such a stage is bound by writing its output, and the
  // padded columns are masked rather than written (12-mode step, FP32
  // storage 2.49 -> 2.42 s, FP64 storage with FP32 arithmetic 3.36 -> 3.28 s;
  // TTN_NO_SHORTK_TILE=1 turns the rule off for comparisons)
  static const bool shortk_on = !getenv("TTN_NO_SHORTK_TILE");
  if (shortk_on && K <= 64 && M >= 32 && N > 32) return 1;
  // prefer big tiles when the grid stays large enough to fill 256 CUs
  struct C {
    int id, bm, bn;
  };
  static const std::vector<C> general{{0, 128, 128}, {2, 128, 64}, {3, 64, 128}, {1, 64, 64},
                                      {5, 64, 32},   {4, 32, 64},  {6, 32, 32}};
  // unit-stride-k operands: the 16-byte-run tiles (no 32-row tiles there)
  static const std::vector<C> unit_k{{10, 128, 128}, {11, 128, 64}, {12, 64, 128}, {14, 96, 96},
                                     {13, 64, 64},   {16, 128, 32}, {15, 64, 32}};
  static const bool unit_k_on = !getenv("TTN_NO_UNIT_K_TILES");
  tn = tn && unit_k_on;
  const std::vector<C>& cs = tn ? unit_k : general;
  int best = tn ? 15 : 6;
  double best_score = -1;
  for (auto& c : cs) {
    // a short contraction (K <= 64) is bound by writing its output, not by
    // operand reuse: tiles up to 64 x 64 keep more workgroups per CU in flight
    // (measured on the 24-deep and 63-deep H_eff stages of the binary tree)
    if (K <= 64 && c.bm * c.bn > 64 * 64) continue;
    const double tm = std::ceil((double)M / c.bm), tn = std::ceil((double)N / c.bn);
    const double eff = (double)M * N / (tm * c.bm * tn * c.bn);  // useful fraction of the tile area
    const double wgs = tm * tn * nblocks_other;
    const double fill = std::min(1.0, wgs / 512.0);
    const double score = eff * fill * (1.0 + 0.15 * std::log2((double)c.bm * c.bn / 1024.0));
    if (score > best_score) {
      best_score = score;
      best = c.id;
    }
  }
  return best;
}

}  // namespace

double min_flops(const std::vector<Tensor>& in, const std::map<int, int>& dims, const std::vector<int>& out_lab,
                 double batch) {
  std::vector<Node> ns;
  for (auto& t : in) {
    Node n;
    n.lab = t.lab;
    std::sort(n.lab.begin(), n.lab.end());
    n.batched = t.batched;
    ns.push_back(n);
  }
  if (ns.size() == 1) return 0.0;
  Search s;
  s.dims = &dims;
  s.batch = batch;
  s.rec(ns, 0.0, 0.0);
  (void)out_lab;
  return s.best;
}

std::unique_ptr<Plan> make_plan(const std::vector<Tensor>& in, const std::map<int, int>& dims,
                                const std::vector<int>& out_lab, const std::vector<int64_t>& out_str,
                                double batch, int ctype, Status& st) {
  auto plan = std::make_unique<Plan>();
  plan->n_in = (int)in.size();
  std::vector<Node> ns;
  for (auto& t : in) {
    Node n;
    n.lab = t.lab;
    std::sort(n.lab.begin(), n.lab.end());
    n.batched = t.batched;
    ns.push_back(n);
  }
  if (ns.size() < 2) {
    st = {TTN_E_ARG, "contraction network needs at least two operands"};
    return nullptr;
  }
  Search s;
  s.dims = &dims;
  s.batch = batch;
  s.rec(ns, 0.0, 0.0);

  // replay the chosen sequence, assigning layouts
  struct Live {
    int id;
    std::vector<int> lab;  // memory order
    std::map<int, int64_t> str;
    int batched;
  };
  std::vector<Live> live;
  for (size_t i = 0; i < in.size(); ++i) {
    Live l;
    l.id = (int)i;
    l.lab = in[i].lab;
    for (size_t j = 0; j < in[i].lab.size(); ++j) l.str[in[i].lab[j]] = in[i].str[j];
    l.batched = in[i].batched;
    live.push_back(l);
  }
  int next_id = (int)in.size();      // intermediate ids of the contraction sequence (lookahead keys)
  int next_actual = (int)in.size();  // ids of the plan's stage outputs (relayout stages included)
  std::map<int, int> act;            // sequence id -> stage output id
  for (size_t i = 0; i < in.size(); ++i) act[(int)i] = (int)i;
  // Lookahead: which step consumes each intermediate, and with which other
  // operand.  An intermediate stores the legs its consumer contracts last, in
  // the other operand's order, so both operands of the consumer run
  // contiguously along k (what the split-K and narrow kernels need).
  std::map<int, int> consumer_other;           // intermediate id -> id of the other operand of its consumer
  std::map<int, std::vector<int>> label_set;  // id -> sorted labels
  {
    std::vector<int> ids;
    for (size_t i = 0; i < in.size(); ++i) {
      ids.push_back((int)i);
      label_set[(int)i] = ns[i].lab;
    }
    int nid = (int)in.size();
    for (size_t si = 0; si < s.best_seq.size(); ++si) {
      const int ia = ids[s.best_seq[si].first], ib = ids[s.best_seq[si].second];
      if (ia >= (int)in.size()) consumer_other[ia] = ib;
      if (ib >= (int)in.size()) consumer_other[ib] = ia;
      // output labels: symmetric difference of the operands' labels
      const auto &xa = label_set[ia], &xb = label_set[ib];
      std::vector<int> o;
      std::set_symmetric_difference(xa.begin(), xa.end(), xb.begin(), xb.end(), std::back_inserter(o));
      label_set[nid] = o;
      std::vector<int> nx;
      for (size_t t = 0; t < ids.size(); ++t)
        if ((int)t != s.best_seq[si].first && (int)t != s.best_seq[si].second) nx.push_back(ids[t]);
      nx.push_back(nid++);
      ids = nx;
    }
  }
  std::vector<int32_t> all_tabs;
  std::vector<Plan::TabRef> refs;
  int64_t ws_item = 0, ws_shared = 0;
  std::vector<int64_t> inter_off;  // by intermediate id - n_in
  std::vector<int> inter_shared;

  for (size_t si = 0; si < s.best_seq.size(); ++si) {
    const auto pr = s.best_seq[si];
    Live la = live[pr.first], lb = live[pr.second];
    const bool last = (si + 1 == s.best_seq.size());
    // contracted labels
    std::vector<int> sa(la.lab), sb(lb.lab);
    std::sort(sa.begin(), sa.end());
    std::sort(sb.begin(), sb.end());
    std::vector<int> kl;
    std::set_intersection(sa.begin(), sa.end(), sb.begin(), sb.end(), std::back_inserter(kl));
    // choose A = the operand with the larger free part (rows), B the other
    auto freeprod = [&](const Live& l) {
      double p = 1;
      for (int x : l.lab)
        if (!std::binary_search(kl.begin(), kl.end(), x)) p *= dims.at(x);
      return p;
    };
    bool swap_ab = freeprod(lb) > freeprod(la);
    if (last) {
      // rows of the final output should hold its slowest labels: keep A =
      // the operand that owns out_lab[0] when possible
      if (!out_lab.empty()) {
        const bool a_has = std::find(la.lab.begin(), la.lab.end(), out_lab[0]) != la.lab.end();
        const bool b_has = std::find(lb.lab.begin(), lb.lab.end(), out_lab[0]) != lb.lab.end();
        if (a_has) swap_ab = false;
        else if (b_has) swap_ab = true;
      }
    }
    if (swap_ab) std::swap(la, lb);
    auto by_stride_desc = [&](const Live& l, std::vector<int> labs) {
      std::stable_sort(labs.begin(), labs.end(), [&](int x, int y) { return l.str.at(x) > l.str.at(y); });
      return labs;
    };
    std::vector<int> ml, nl, kk;
    for (int x : la.lab)
      if (!std::binary_search(kl.begin(), kl.end(), x)) ml.push_back(x);
    for (int x : lb.lab)
      if (!std::binary_search(kl.begin(), kl.end(), x)) nl.push_back(x);
    ml = by_stride_desc(la, ml);
    nl = by_stride_desc(lb, nl);
    kk = by_stride_desc(la, kl);

    Step stp;
    stp.a = act.at(la.id);
    stp.b = act.at(lb.id);
    stp.batched = la.batched || lb.batched;
    double un = 1;
    for (int x : uni(sa, sb)) un *= dims.at(x);
    stp.flops = 2.0 * un;
    GemmDesc& g = stp.g;
    auto prod = [&](const std::vector<int>& l) {
      int64_t p = 1;
      for (int x : l) p *= dims.at(x);
      return p;
    };
    const int64_t M = prod(ml), N = prod(nl), K = prod(kk);
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) {
      st = {TTN_E_SHAPE, "contraction stage too large for 32-bit offsets"};
      return nullptr;
    }
    g.M = (int)M;
    g.N = (int)N;
    g.K = (int)K;

    // output layout
    Live lo;
    lo.batched = stp.batched ? 1 : 0;
    std::map<int, int64_t> ostr;
    if (last) {
      for (size_t j = 0; j < out_lab.size(); ++j) ostr[out_lab[j]] = out_str[j];
      lo.id = -1;
    } else {
      std::vector<int> ol(ml);
      ol.insert(ol.end(), nl.begin(), nl.end());
      static const bool lookahead = !getenv("TTN_PLAN_NO_LOOKAHEAD");
      auto co = consumer_other.find(next_id);
      if (lookahead && co != consumer_other.end()) {
        // labels the consumer contracts = shared with its other operand
        const Live* other = nullptr;
        for (auto& l : live)
          if (l.id == co->second) other = &l;
        std::vector<int> kc;
        if (other) {
          // other operand already laid out: its memory order (slowest first)
          std::vector<int> ord = other->lab;
          std::stable_sort(ord.begin(), ord.end(),
                           [&](int x, int y) { return other->str.at(x) > other->str.at(y); });
          for (int x : ord)
            if (std::find(ol.begin(), ol.end(), x) != ol.end()) kc.push_back(x);
        } else {
          // produced later: ascending label order; that operand will then
          // follow this one's order
          for (int x : label_set[co->second])
            if (std::find(ol.begin(), ol.end(), x) != ol.end()) kc.push_back(x);
        }
        if (!kc.empty()) {
          std::vector<int> re;
          for (int x : ol)
            if (std::find(kc.begin(), kc.end(), x) == kc.end()) re.push_back(x);
          re.insert(re.end(), kc.begin(), kc.end());
          ol = re;
        }
      }
      int64_t acc = 1;
      for (int j = (int)ol.size() - 1; j >= 0; --j) {
        ostr[ol[j]] = acc;
        acc *= dims.at(ol[j]);
      }
      lo.lab = ol;
      lo.id = next_id++;
      stp.out_size = acc;
      if (acc > INT32_MAX) {
        st = {TTN_E_SHAPE, "intermediate too large for 32-bit offsets"};
        return nullptr;
      }
    }
    lo.str = ostr;
    // Row and column order.  The matrix rows run over ml in the order listed
    // (last label fastest), likewise the columns over nl; they start sorted by
    // the operand's own strides.  The output's unit-stride label f should be
    // the fastest row (or column) index, or the kernels write one element per
    // memory run; it is moved there unless that breaks an m-fast (n-fast) read
    // of a larger operand (A read M*K against C written M*N).
    auto smallest = [&](const std::map<int, int64_t>& str, const std::vector<int>& labs) {
      int best = -1;
      int64_t bs = INT64_MAX;
      for (int x : labs) {
        auto it = str.find(x);
        if (it != str.end() && it->second < bs) {
          bs = it->second;
          best = x;
        }
      }
      return best;
    };
    {
      std::vector<int> mn(ml);
      mn.insert(mn.end(), nl.begin(), nl.end());
      const int f = smallest(ostr, mn);
      auto move_last = [&](std::vector<int>& v, int x) {
        v.erase(std::find(v.begin(), v.end(), x));
        v.push_back(x);
      };
      const int sa = smallest(la.str, la.lab), sb = smallest(lb.str, lb.lab);
      if (f >= 0 && std::find(ml.begin(), ml.end(), f) != ml.end() && ml.back() != f) {
        const bool a_rows_fast = ml.back() == sa;
        if (!a_rows_fast || N >= K) move_last(ml, f);
      } else if (f >= 0 && std::find(nl.begin(), nl.end(), f) != nl.end() && nl.back() != f) {
        const bool b_cols_fast = nl.back() == sb;
        if (!b_cols_fast || M >= K) move_last(nl, f);
      }
      // fast flags: is an operand's unit-stride label its fastest row / column
      g.a_mfast = !ml.empty() && ml.back() == sa;
      g.b_nfast = !nl.empty() && nl.back() == sb;
      g.c_mfast = !ml.empty() && (nl.empty() || ml.back() == f);
    }
    // A small shared input (an operator tensor) read neither along its unit
    // stride nor contiguously along k is first copied, once per call, into
    // [k][rows] order, so that the GEMM reads it row-fast and coalesced; the
    // same for B ([k][columns]).
    auto vmax = [](const std::vector<int32_t>& v) {
      int64_t m = 0;
      for (int32_t x : v) m = std::max<int64_t>(m, x);
      return m;
    };
    auto relayout = [&](Live& l, const std::vector<int>& rows, int64_t R) {
      std::vector<int32_t> t_r, t_k;
      group_offsets(rows, dims, l.str, t_r);
      group_offsets(kk, dims, l.str, t_k);
      bool ku = true, al = true;
      for (int i = 0; i < (int)t_k.size() && ku; ++i) ku = t_k[i] == i;
      for (int32_t x : t_r) al = al && x % 4 == 0;
      if ((ku && al) || R * K > (int64_t)1 << 24) return -1;  // already contiguous along k, or too big
      Step rs;
      rs.kind = 1;
      rs.a = act.at(l.id);
      rs.b = -1;
      rs.batched = false;
      rs.g.M = (int)R;
      rs.g.N = 1;
      rs.g.K = (int)K;
      rs.out_size = R * K;
      rs.max_a = vmax(t_r) + vmax(t_k);
      rs.max_b = 0;
      rs.max_c = R * K - 1;
      refs.push_back({plan->steps.size(), 0, all_tabs.size()});
      all_tabs.insert(all_tabs.end(), t_r.begin(), t_r.end());
      while (all_tabs.size() % 16) all_tabs.push_back(0);
      refs.push_back({plan->steps.size(), 1, all_tabs.size()});
      all_tabs.insert(all_tabs.end(), t_k.begin(), t_k.end());
      while (all_tabs.size() % 16) all_tabs.push_back(0);
      rs.out = next_actual++;
      inter_off.push_back(ws_shared);
      inter_shared.push_back(1);
      ws_shared += (R * K + 63) / 64 * 64;
      plan->steps.push_back(rs);
      // the copy's strides: rows in the listed order (last fastest), then k * R
      std::map<int, int64_t> ns;
      int64_t acc = 1;
      for (int j = (int)rows.size() - 1; j >= 0; --j) {
        ns[rows[j]] = acc;
        acc *= dims.at(rows[j]);
      }
      for (int j = (int)kk.size() - 1; j >= 0; --j) {
        ns[kk[j]] = acc;
        acc *= dims.at(kk[j]);
      }
      l.str = ns;
      return rs.out;
    };
    static const bool relayout_on = !getenv("TTN_PLAN_NO_RELAYOUT");
    if (relayout_on && !g.a_mfast && la.id < (int)in.size() && !la.batched && !ml.empty()) {
      const int r = relayout(la, ml, M);
      if (r >= 0) {
        stp.a = r;
        g.a_mfast = true;
      }
    }
    if (relayout_on && !g.b_nfast && lb.id < (int)in.size() && !lb.batched && !nl.empty()) {
      const int r = relayout(lb, nl, N);
      if (r >= 0) {
        stp.b = r;
        g.b_nfast = true;
      }
    }
    // the stage's own output slot (after any relayout slots: stage outputs
    // are numbered in stage order)
    if (!last) {
      stp.out = next_actual++;
      act[lo.id] = stp.out;
      const int64_t acc = stp.out_size;
      if (stp.batched) {
        inter_off.push_back(ws_item);
        inter_shared.push_back(0);
        ws_item += (acc + 63) / 64 * 64;
      } else {
        inter_off.push_back(ws_shared);
        inter_shared.push_back(1);
        ws_shared += (acc + 63) / 64 * 64;
      }
    } else {
      stp.out = -1;
    }
    // tables
    std::vector<int32_t> t_am, t_ak, t_bk, t_bn, t_cm, t_cn;
    group_offsets(ml, dims, la.str, t_am);
    group_offsets(kk, dims, la.str, t_ak);
    group_offsets(kk, dims, lb.str, t_bk);
    group_offsets(nl, dims, lb.str, t_bn);
    group_offsets(ml, dims, ostr, t_cm);
    group_offsets(nl, dims, ostr, t_cn);
    std::vector<int32_t>* tabs6[6] = {&t_am, &t_ak, &t_bk, &t_bn, &t_cm, &t_cn};
    for (int w = 0; w < 6; ++w) {
      std::vector<int32_t>* v = tabs6[w];
      refs.push_back({plan->steps.size(), w, all_tabs.size()});
      all_tabs.insert(all_tabs.end(), v->begin(), v->end());
      // pad each table to 16 entries for alignment
      while (all_tabs.size() % 16) all_tabs.push_back(0);
    }
    stp.max_a = vmax(t_am) + vmax(t_ak);
    stp.max_b = vmax(t_bk) + vmax(t_bn);
    stp.max_c = vmax(t_cm) + vmax(t_cn);
    {
      bool ku = true, al = true;
      for (int i = 0; i < (int)t_ak.size() && ku; ++i) ku = t_ak[i] == i && t_bk[i] == i;
      for (int32_t x : t_am) al = al && x % 4 == 0;
      for (int32_t x : t_bn) al = al && x % 4 == 0;
      g.k_unit = ku;
      g.rows_al4 = al;
    }
    g.tile = splitk_eligible(g, ctype)   ? 8
             : narrow_eligible(g, ctype) ? 9
                                         : pick_tile(g.M, g.N, g.K, stp.batched ? batch : 1.0, tn_eligible(g, ctype));
    // a tile forced for tests and tuning experiments (read at planning time),
    // taken where the stage admits it
    if (const char* ft = getenv("TTN_FORCE_TILE")) {
      const int t = atoi(ft);
      const bool ok = (t >= 0 && t <= 6) || (t == 8 && splitk_eligible(g, ctype)) ||
                      (t == 9 && narrow_eligible(g, ctype)) || (t >= 10 && t <= 16 && tn_eligible(g, ctype));
      if (ok) g.tile = t;
    }
    if (stp.batched) plan->flops_per_item += stp.flops;
    else plan->flops_shared += stp.flops;
    plan->steps.push_back(stp);
    // update the live list
    std::vector<Live> nx;
    for (size_t t = 0; t < live.size(); ++t)
      if ((int)t != pr.first && (int)t != pr.second) nx.push_back(live[t]);
    nx.push_back(lo);
    live = nx;
  }
  plan->inter_off = inter_off;
  plan->ws_per_item = ws_item;
  plan->ws_shared = ws_shared;
  (void)inter_shared;
  (void)ctype;
  // the tables go to the device when the context binds the plan (table pool)
  plan->h_tabs = std::move(all_tabs);
  plan->tab_refs = std::move(refs);
  return plan;
}

void bind_plan_tables(Plan& plan, const int32_t* d_tabs) {
  for (const auto& r : plan.tab_refs) {
    GemmDesc& g = plan.steps[r.step].g;
    const int32_t* p = d_tabs + r.off;
    switch (r.which) {
      case 0: g.a_om = p; break;
      case 1: g.a_ok = p; break;
      case 2: g.b_ok = p; break;
      case 3: g.b_on = p; break;
      case 4: g.c_om = p; break;
      default: g.c_on = p; break;
    }
  }
}

bool check_plan_bounds(const Plan& P, const std::vector<int64_t>& in_elems, int64_t out_elems, std::string& why) {
  if ((int)in_elems.size() != P.n_in) {
    why = "operand count mismatch";
    return false;
  }
  std::map<int, int64_t> size;
  for (int i = 0; i < P.n_in; ++i) size[i] = in_elems[i];
  for (const Step& s : P.steps)
    if (s.out >= 0) size[s.out] = s.out_size;
  for (const Step& s : P.steps) {
    const int64_t cs = s.out >= 0 ? s.out_size : out_elems;
    if (s.max_a >= size.at(s.a) || (s.b >= 0 && s.max_b >= size.at(s.b)) || s.max_c >= cs) {
      why = "contraction stage would address outside its operands";
      return false;
    }
  }
  return true;
}

}  // namespace ttn
