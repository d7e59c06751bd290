// Nested dissection symbolic analysis (Section 2.2 and Section 3.2 of the
// paper name nested dissection and the multifrontal method without further
// detail; George 1973 / Duff & Reid 1983 are the cited sources).
//
// The 3^d stencil couples grid points at infinity-distance <= 1, so a plane
// of width one along any axis separates the two sides of a box.  Boxes are
// split along their longest axis at the middle until every extent is at
// most the leaf side.  A front eliminates its separator (or, for a leaf,
// its whole box); its boundary set B is the halo of the box (points at
// infinity-distance exactly 1, inside the grid), which lies on ancestor
// separators.  Fronts are ordered by height so that one level of fronts can
// be factorised in one batched launch.
#include "plan.h"

#include <algorithm>
#include <functional>
#include <unordered_map>

namespace lsp {

namespace {

struct Node {
  int lo[3], hi[3];
  bool leaf;
  int axis, sep;
  int child[2];
  int nchild;
  int height;
  std::vector<int> I, B;
};

int lin(const int* i, int n, int d) {
  int l = 0, s = 1;
  for (int a = 0; a < d; ++a) { l += i[a] * s; s *= n; }
  return l;
}

}  // namespace

void build_plan(Plan& P, int n, int d, int max_nrhs, const lsp_options& opts) {
  LSP_REQUIRE(d == 2 || d == 3, "d must be 2 or 3");
  LSP_REQUIRE(n >= 4 && n <= 4096, "n must be in [4, 4096]");
  LSP_REQUIRE(max_nrhs >= 1 && max_nrhs <= 256, "max_nrhs must be in [1, 256]");
  long long NN = 1;
  for (int a = 0; a < d; ++a) NN *= n;
  LSP_REQUIRE(NN <= (1LL << 28), "grid too large");
  P.n = n; P.d = d; P.N = (int)NN; P.L = 2 * n; P.max_nrhs = max_nrhs; P.opts = opts;

  // FFT radices of L = 2^a 3^b (largest radices first).
  {
    int L = P.L, r = L;
    int c3 = 0, c2 = 0;
    while (r % 3 == 0) { r /= 3; ++c3; }
    while (r % 2 == 0) { r /= 2; ++c2; }
    LSP_REQUIRE(r == 1, "2n must factor as 2^a 3^b (n = 2^a' 3^b)");
    std::vector<int> rad;
    while (c2 >= 3) { rad.push_back(8); c2 -= 3; }
    if (c2 == 2) rad.push_back(4);
    if (c2 == 1) rad.push_back(2);
    for (int k = 0; k < c3; ++k) rad.push_back(3);
    P.radices = rad;
  }

  int leaf = opts.leaf > 0 ? opts.leaf : (d == 2 ? 8 : 4);
  LSP_REQUIRE(leaf >= 2, "leaf side must be >= 2");

  std::vector<Node> nodes;
  nodes.reserve(1024);
  std::function<int(const int*, const int*)> build = [&](const int* lo, const int* hi) -> int {
    Node nd;
    for (int a = 0; a < 3; ++a) { nd.lo[a] = a < d ? lo[a] : 0; nd.hi[a] = a < d ? hi[a] : 1; }
    int ax = 0, ext = 0;
    for (int a = 0; a < d; ++a) {
      int e = hi[a] - lo[a];
      if (e > ext) { ext = e; ax = a; }
    }
    nd.leaf = ext <= leaf;
    nd.nchild = 0;
    nd.child[0] = nd.child[1] = -1;
    nd.axis = ax;
    nd.sep = lo[ax] + ext / 2;
    nd.height = 0;
    int id = (int)nodes.size();
    nodes.push_back(nd);
    if (!nd.leaf) {
      int l2[3], h2[3];
      for (int a = 0; a < d; ++a) { l2[a] = lo[a]; h2[a] = hi[a]; }
      h2[ax] = nd.sep;
      int c0 = (h2[ax] > l2[ax]) ? build(l2, h2) : -1;
      for (int a = 0; a < d; ++a) { l2[a] = lo[a]; h2[a] = hi[a]; }
      l2[ax] = nd.sep + 1;
      int c1 = (h2[ax] > l2[ax]) ? build(l2, h2) : -1;
      Node& me = nodes[id];
      if (c0 >= 0) me.child[me.nchild++] = c0;
      if (c1 >= 0) me.child[me.nchild++] = c1;
      int h = 0;
      for (int c = 0; c < me.nchild; ++c) h = std::max(h, nodes[me.child[c]].height + 1);
      me.height = h;
    }
    return id;
  };
  int lo0[3] = {0, 0, 0}, hi0[3] = {n, n, n};
  int root = build(lo0, hi0);
  (void)root;

  // Index sets.
  for (auto& nd : nodes) {
    int i[3];
    if (nd.leaf) {
      for (i[2] = nd.lo[2]; i[2] < nd.hi[2]; ++i[2])
        for (i[1] = nd.lo[1]; i[1] < nd.hi[1]; ++i[1])
          for (i[0] = nd.lo[0]; i[0] < nd.hi[0]; ++i[0]) nd.I.push_back(lin(i, n, d));
    } else {
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) { lo[a] = nd.lo[a]; hi[a] = nd.hi[a]; }
      lo[nd.axis] = nd.sep; hi[nd.axis] = nd.sep + 1;
      for (i[2] = lo[2]; i[2] < hi[2]; ++i[2])
        for (i[1] = lo[1]; i[1] < hi[1]; ++i[1])
          for (i[0] = lo[0]; i[0] < hi[0]; ++i[0]) nd.I.push_back(lin(i, n, d));
    }
    int elo[3], ehi[3];
    for (int a = 0; a < 3; ++a) {
      if (a < d) { elo[a] = std::max(nd.lo[a] - 1, 0); ehi[a] = std::min(nd.hi[a] + 1, n); }
      else { elo[a] = 0; ehi[a] = 1; }
    }
    for (i[2] = elo[2]; i[2] < ehi[2]; ++i[2])
      for (i[1] = elo[1]; i[1] < ehi[1]; ++i[1])
        for (i[0] = elo[0]; i[0] < ehi[0]; ++i[0]) {
          bool inside = true;
          for (int a = 0; a < d; ++a) inside = inside && i[a] >= nd.lo[a] && i[a] < nd.hi[a];
          if (!inside) nd.B.push_back(lin(i, n, d));
        }
  }

  // Order by height, stable in creation order.
  std::vector<int> order(nodes.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return nodes[a].height < nodes[b].height; });
  std::vector<int> newid(nodes.size());
  for (size_t k = 0; k < order.size(); ++k) newid[order[k]] = (int)k;

  int H = 0;
  for (auto& nd : nodes) H = std::max(H, nd.height);
  P.nlevels = H + 1;
  P.level_ptr.assign(P.nlevels + 1, 0);
  P.level_maxp.assign(P.nlevels, 0);
  P.level_maxpq.assign(P.nlevels, 0);
  P.fronts.resize(nodes.size());
  P.idx.clear();
  long long f_off = 0, piv_off = 0, dinv_off = 0;
  P.nb = opts.panel > 0 ? opts.panel : 32;
  P.flops = 0.0; P.factor_entries = 0.0; P.max_front = 0; P.max_p = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    const Node& nd = nodes[order[k]];
    FrontDev& f = P.fronts[k];
    f.p = (int)nd.I.size();
    LSP_REQUIRE(f.p > 0, "empty separator in the dissection");
    f.q = (int)nd.B.size();
    f.child0 = nd.nchild > 0 ? newid[nd.child[0]] : -1;
    f.child1 = nd.nchild > 1 ? newid[nd.child[1]] : -1;
    f.idx_off = (long long)P.idx.size();
    f.f_off = f_off;
    f.piv_off = piv_off;
    f.dinv_off = dinv_off;
    dinv_off += (long long)((f.p + P.nb - 1) / P.nb) * 2 * P.nb * P.nb;
    f.level = nd.height;
    f.pad = 0;
    P.idx.insert(P.idx.end(), nd.I.begin(), nd.I.end());
    P.idx.insert(P.idx.end(), nd.B.begin(), nd.B.end());
    long long m = f.p + f.q;
    f_off += m * m;
    piv_off += f.p;
    P.level_ptr[nd.height + 1]++;
    P.level_maxp[nd.height] = std::max(P.level_maxp[nd.height], f.p);
    P.level_maxpq[nd.height] = std::max(P.level_maxpq[nd.height], (int)m);
    P.max_front = std::max(P.max_front, (int)m);
    P.max_p = std::max(P.max_p, f.p);
    // complex multiply-adds of the partial LU: pivot j updates the trailing
    // (m - j - 1)^2 block; 8 real flops per complex multiply-add.
    double cm = 0.0;
    for (long long j = 0; j < f.p; ++j) cm += (double)(m - j - 1) * (double)(m - j - 1);
    P.flops += 8.0 * cm;
    P.factor_entries += (double)m * m - (double)f.q * f.q;
    for (int k0 = 0; k0 < f.p; k0 += P.nb) {
      int kb = std::min(P.nb, f.p - k0);
      P.sweep_entries += (double)(m - k0 - kb) * kb + (double)P.nb * P.nb;
      P.update_flops += 8.0 * (double)(m - k0 - kb) * (double)(m - k0 - kb) * kb;
      P.panel_blocks += 1.0;
    }
  }
  for (FrontDev& f : P.fronts) {
    const int kids[2] = {f.child0, f.child1};
    for (int c = 0; c < 2; ++c) {
      const bool has = kids[c] >= 0;
      f.cidx[c] = has ? P.fronts[kids[c]].idx_off : -1;
      f.cfoff[c] = has ? P.fronts[kids[c]].f_off : -1;
      f.cm[c] = has ? P.fronts[kids[c]].p + P.fronts[kids[c]].q : 0;
    }
  }
  for (int l = 0; l < P.nlevels; ++l) P.level_ptr[l + 1] += P.level_ptr[l];
  // default trailing-update tiles by front order; an autotuner may replace them
  // (measured with the autotuner on 2D n = 256 and 1024 and 3D n = 64:
  // complex128 factors run fastest with 32-wide tiles everywhere; complex64
  // ones with 64-wide tiles, except in 2D up to 160 rows and above 512 rows
  // (the two-panel levels), where 32-wide ones win, and a single 2D root
  // front of 1024 rows or more, which takes 128-wide ones)
  P.level_tile.assign(P.nlevels, 64);
  for (int l = 0; l < P.nlevels; ++l) {
    const int cnt = P.level_ptr[l + 1] - P.level_ptr[l], mq = P.level_maxpq[l];
    if (opts.precision == LSP_FP64 || (d == 2 && mq <= 160)) P.level_tile[l] = 32;
    else if (d == 2 && mq >= 1024 && cnt == 1) P.level_tile[l] = 128;
    else if (d == 2 && mq > 512) P.level_tile[l] = 32;
    else P.level_tile[l] = 64;
  }
  // Dense sweep levels: few fronts (a front's panel chain runs on one
  // workgroup per right-hand-side group, so with few fronts the chain's
  // latency is the level's time), at least two panels, at most 1024 rows.
  P.level_dense.assign(P.nlevels, 0);
  P.dense_elems = 0;
  P.dense_entries = 0.0;
  P.dense_levels = 0;
  for (int l = 0; l < P.nlevels; ++l) {
    const int cnt = P.level_ptr[l + 1] - P.level_ptr[l];
    if (opts.dense_sweeps != 0 && cnt <= 16 && P.level_maxp[l] > P.nb && P.level_maxpq[l] <= 1024) {
      P.level_dense[l] = 1;
      ++P.dense_levels;
    }
  }
  for (FrontDev& f : P.fronts) {
    const long long m = f.p + f.q;
    f.g_off = -1;
    if (!P.level_dense[f.level]) continue;
    f.g_off = P.dense_elems;
    P.dense_elems += 2 * m * f.p;
    P.dense_entries += (double)m * f.p;
    for (int k0 = 0; k0 < f.p; k0 += P.nb) {  // these panels are not read by the sweeps
      const int kb = std::min(P.nb, f.p - k0);
      P.sweep_entries -= (double)(m - k0 - kb) * kb + (double)P.nb * P.nb;
    }
  }
  P.level_small_sweep.assign(P.nlevels, 0);
  for (int l = 0; l < P.nlevels; ++l) {
    bool ok = !P.level_dense[l] && P.level_maxp[l] <= 2 * P.nb && P.level_maxpq[l] <= 160;
    for (int i = P.level_ptr[l]; ok && i < P.level_ptr[l + 1]; ++i)
      ok = P.fronts[i].q + P.fronts[i].p - std::min(P.fronts[i].p, P.nb) <= 128;
    P.level_small_sweep[l] = ok;
  }
  // small-front levels (more than 16 fronts of at most two panels and 256
  // rows) of plans for blocks of right-hand sides: panel chains with the
  // right-hand sides on the matrix cores
  P.level_mchain.assign(P.nlevels, 0);
  P.mchain_levels = 0;
  P.mchain_entries = 0.0;
  P.mchain_pivots = P.mchain_rows = P.mchain_child_rows = 0.0;
  for (int l = 0; l < P.nlevels; ++l) {
    const int cnt = P.level_ptr[l + 1] - P.level_ptr[l];
    const bool want = opts.dense_sweeps == 2 || (opts.dense_sweeps == 1 && max_nrhs >= 4);
    if (!want || P.level_dense[l] || cnt <= 16 || P.level_maxp[l] > 2 * P.nb || P.level_maxpq[l] > 256) continue;
    P.level_mchain[l] = 1;
    ++P.mchain_levels;
  }
  P.level_blocked.assign(P.nlevels, 0);
  for (int l = 0; l < P.nlevels; ++l) {
    const int cnt = P.level_ptr[l + 1] - P.level_ptr[l];
    if (opts.blocked_sweeps == 0 || P.level_dense[l] || P.level_mchain[l] || P.level_small_sweep[l]) continue;
    P.level_blocked[l] = opts.blocked_sweeps == 2 || P.level_maxpq[l] > 1024 ||
                         (cnt <= 32 && P.level_maxp[l] > 2 * P.nb);
  }
  // storage of the blocked levels' super-block operators (forward then
  // backward, SB x SB each), after the dense levels' operators
  {
    const long long SB = kSweepRows;
    P.blocked_levels = 0;
    P.blocked_entries = 0.0;
    P.bsweep_ystride = 0;
    P.bsweep_chunks = 0;
    for (int l = 0; l < P.nlevels; ++l) {
      if (!P.level_blocked[l]) continue;
      ++P.blocked_levels;
      const long long cnt = P.level_ptr[l + 1] - P.level_ptr[l];
      int maxq = 0;
      for (int i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
        FrontDev& f = P.fronts[i];
        const long long nsb = (f.p + SB - 1) / SB;
        f.g_off = P.dense_elems;
        P.dense_elems += 2 * nsb * SB * SB;
        P.blocked_entries += (double)(nsb * SB * SB);
        maxq = std::max(maxq, f.q);
      }
      P.bsweep_ystride = std::max(P.bsweep_ystride, cnt * std::max<long long>(SB, P.level_maxp[l]));
      P.bsweep_chunks = std::max(P.bsweep_chunks, (maxq + kSweepCols - 1) / kSweepCols);
    }
    P.chain_entries = 0.0;
    P.blocked_panel_entries = 0.0;
    P.assemble_entries = 0.0;
    for (const FrontDev& f : P.fronts) {
      const long long m = f.p + f.q;
      P.assemble_entries += (double)m * m;
      if (f.child0 >= 0) P.assemble_entries += (double)P.fronts[f.child0].q * P.fronts[f.child0].q;
      if (f.child1 >= 0) P.assemble_entries += (double)P.fronts[f.child1].q * P.fronts[f.child1].q;
      if (P.level_dense[f.level]) continue;
      if (P.level_mchain[f.level]) {
        P.mchain_pivots += f.p;
        P.mchain_rows += (double)m;
        if (f.child0 >= 0) P.mchain_child_rows += P.fronts[f.child0].q;
        if (f.child1 >= 0) P.mchain_child_rows += P.fronts[f.child1].q;
        for (int k0 = 0; k0 < f.p; k0 += P.nb) {
          const int kb = std::min(P.nb, f.p - k0);
          P.mchain_entries += (double)(m - k0 - kb) * kb + (double)P.nb * P.nb;
        }
      } else if (P.level_blocked[f.level]) {
        for (long long s0 = 0; s0 < f.p; s0 += SB) {
          const long long s1 = std::min<long long>(s0 + SB, f.p);
          P.blocked_panel_entries += (double)(m - s1) * (double)(s1 - s0);
        }
      } else {
        for (int k0 = 0; k0 < f.p; k0 += P.nb) {
          const int kb = std::min(P.nb, f.p - k0);
          P.chain_entries += (double)(m - k0 - kb) * kb + (double)P.nb * P.nb;
        }
      }
    }
  }
  P.front_elems = f_off;
  P.dinv_elems = dinv_off;
  P.sum_p = piv_off;
  P.sum_pq = (long long)P.idx.size();
  LSP_REQUIRE((long long)P.max_front * P.max_front < (1LL << 31), "front too large for 32-bit entry indices");
  {
    const int sh = gpos_shift(d);
    P.gpos.resize(P.idx.size());
    for (size_t k = 0; k < P.idx.size(); ++k) {
      long long g = P.idx[k];
      unsigned packed = 0;
      for (int a = 0; a < d; ++a) {
        packed |= (unsigned)(g % n) << (sh * a);
        g /= n;
      }
      P.gpos[k] = packed;
    }
  }
  LSP_REQUIRE(P.sum_p == P.N, "nested dissection lost grid points");

  // Extend-add maps: for each front position, where the same grid point sits
  // in each child's front (only the child's B part can match).
  P.cpos.assign(2 * P.idx.size(), -1);
  std::vector<int> where(P.N, -1);
  for (size_t k = 0; k < P.fronts.size(); ++k) {
    const FrontDev& f = P.fronts[k];
    int kids[2] = {f.child0, f.child1};
    for (int c = 0; c < 2; ++c) {
      if (kids[c] < 0) continue;
      const FrontDev& ch = P.fronts[kids[c]];
      for (int j = 0; j < ch.q; ++j) where[P.idx[ch.idx_off + ch.p + j]] = ch.p + j;
      int matched = 0;
      for (int r = 0; r < f.p + f.q; ++r) {
        int g = P.idx[f.idx_off + r];
        if (where[g] >= 0) { P.cpos[2 * (f.idx_off + r) + c] = where[g]; ++matched; }
      }
      LSP_REQUIRE(matched == ch.q, "child boundary not contained in parent front");
      for (int j = 0; j < ch.q; ++j) where[P.idx[ch.idx_off + ch.p + j]] = -1;
    }
  }
}

void build_general(Plan& P, const unsigned char* mask, int r) {
  LSP_REQUIRE(mask != nullptr, "null domain mask");
  LSP_REQUIRE(r >= 1 && r <= 4096, "sketch columns must be in [1, 4096]");
  const int n = P.n, d = P.d, ns = d == 2 ? 9 : 27;
  P.general = true;
  P.sketch_r = r;
  P.ptab.assign(P.N, -2);
  P.bpts.clear();
  P.bslots.clear();
  P.domain_points = 0;
  for (int pt = 0; pt < P.N; ++pt) {
    if (!mask[pt]) continue;
    ++P.domain_points;
    const int i[3] = {pt % n, (pt / n) % n, d == 3 ? pt / (n * n) : 0};
    unsigned bits = 0;
    for (int q = 0; q < ns; ++q) {
      const int o[3] = {q % 3 - 1, (q / 3) % 3 - 1, q / 9 - 1};
      bool in = true;
      long long nb = 0, st = 1;
      for (int a = 0; a < d; ++a) {
        const int j = i[a] + o[a];
        in = in && j >= 0 && j < n;
        nb += (long long)j * st;
        st *= n;
      }
      if (in && mask[nb]) bits |= 1u << q;
    }
    if (bits == (ns == 32 ? ~0u : (1u << ns) - 1)) {
      P.ptab[pt] = -1;
    } else {
      P.ptab[pt] = (int)P.bpts.size();
      P.bpts.push_back(pt);
      P.bslots.push_back(bits);
    }
  }
  LSP_REQUIRE(P.domain_points > 0, "empty domain mask");
}

}  // namespace lsp
