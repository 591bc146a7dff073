// Host-side level structure (integer work): see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <map>
#include <numeric>

namespace ambddc {

static int lower_index(const std::vector<int>& v, int x, int lo, int hi) {
  auto it = std::lower_bound(v.begin() + lo, v.begin() + hi, x);
  if (it == v.begin() + hi || *it != x) return -1;
  return int(it - v.begin()) - lo;
}

std::string level1_input(int n_nodes, int n_elems, int dof, const int32_t* elem_nodes,
                         const uint8_t* dirichlet, const int32_t* elem_to_sub, LevelInput& in,
                         std::vector<int>& free_of_full) {
  in = LevelInput();
  in.dof_per_node = dof;
  in.n_rb = dof == 1 ? 1 : 6;
  in.n_node = n_nodes;
  in.n_elem = n_elems;
  const int64_t nfull = int64_t(n_nodes) * dof;
  free_of_full.assign(nfull, -1);
  int nf = 0;
  for (int64_t j = 0; j < nfull; ++j)
    if (!dirichlet[j]) free_of_full[j] = nf++;
  in.n_dof = nf;
  in.dof_comp.resize(nf);
  in.node_dof_ptr.assign(n_nodes + 1, 0);
  for (int n = 0; n < n_nodes; ++n) {
    int c = 0;
    for (int q = 0; q < dof; ++q) c += free_of_full[int64_t(n) * dof + q] >= 0;
    in.node_dof_ptr[n + 1] = in.node_dof_ptr[n] + c;
  }
  in.node_dofs.resize(in.node_dof_ptr[n_nodes]);
  for (int n = 0; n < n_nodes; ++n) {
    int p = in.node_dof_ptr[n];
    for (int q = 0; q < dof; ++q) {
      int f = free_of_full[int64_t(n) * dof + q];
      if (f >= 0) {
        in.node_dofs[p++] = f;
        in.dof_comp[f] = q;
      }
    }
  }
  int n_sub = 0;
  for (int e = 0; e < n_elems; ++e) {
    if (elem_to_sub[e] < 0) return "elem_to_sub has a negative entry";
    n_sub = std::max(n_sub, elem_to_sub[e] + 1);
  }
  in.n_sub = n_sub;
  in.elem_sub.assign(elem_to_sub, elem_to_sub + n_elems);
  in.elem_node_ptr.resize(n_elems + 1);
  in.elem_dof_ptr.resize(n_elems + 1);
  in.elem_nodes.resize(size_t(n_elems) * 8);
  in.elem_dofs.resize(size_t(n_elems) * 8 * dof);
  in.sub_floating.assign(n_sub, 1);
  for (int e = 0; e < n_elems; ++e) {
    in.elem_node_ptr[e] = int64_t(e) * 8;
    in.elem_dof_ptr[e] = int64_t(e) * 8 * dof;
    for (int a = 0; a < 8; ++a) {
      int n = elem_nodes[int64_t(e) * 8 + a];
      if (n < 0 || n >= n_nodes) return "elem_nodes out of range";
      in.elem_nodes[int64_t(e) * 8 + a] = n;
      for (int q = 0; q < dof; ++q) {
        int f = free_of_full[int64_t(n) * dof + q];
        in.elem_dofs[int64_t(e) * 8 * dof + a * dof + q] = f;
        if (f < 0) in.sub_floating[elem_to_sub[e]] = 0;
      }
    }
  }
  in.elem_node_ptr[n_elems] = int64_t(n_elems) * 8;
  in.elem_dof_ptr[n_elems] = int64_t(n_elems) * 8 * dof;
  return "";
}

std::string build_level_plan(LevelPlan& L, int init, bool keep_edges) {
  if (init != INIT_CE && init != INIT_CEF && init != INIT_C) return "unknown initial constraint set";
  const bool face_averages = init == INIT_CEF, edge_averages = init != INIT_C;
  LevelInput& in = L.in;
  const int nn = in.n_node, ns = in.n_sub;
  // node -> sorted set of subdomains (via sorted (node, sub) keys)
  std::vector<uint64_t> keys;
  keys.reserve(in.elem_nodes.size());
  for (int e = 0; e < in.n_elem; ++e)
    for (int64_t p = in.elem_node_ptr[e]; p < in.elem_node_ptr[e + 1]; ++p)
      keys.push_back(uint64_t(in.elem_nodes[p]) * uint64_t(ns + 1) + uint64_t(in.elem_sub[e]));
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  std::vector<int> nptr(nn + 1, 0), nsub;
  nsub.reserve(keys.size());
  for (uint64_t k : keys) {
    int n = int(k / uint64_t(ns + 1));
    nptr[n + 1]++;
    nsub.push_back(int(k % uint64_t(ns + 1)));
  }
  for (int n = 0; n < nn; ++n) nptr[n + 1] += nptr[n];
  // globs: interface nodes grouped by their subdomain set, in order of first node
  std::map<std::vector<int>, int> gid;
  L.globs.clear();
  std::vector<int> node_glob(nn, -1);
  for (int n = 0; n < nn; ++n) {
    int c = nptr[n + 1] - nptr[n];
    if (c < 2) continue;
    std::vector<int> key(nsub.begin() + nptr[n], nsub.begin() + nptr[n + 1]);
    auto it = gid.find(key);
    int g;
    if (it == gid.end()) {
      g = int(L.globs.size());
      gid.emplace(key, g);
      Glob gl;
      gl.subs = key;
      L.globs.push_back(gl);
    } else {
      g = it->second;
    }
    L.globs[g].nodes.push_back(n);
    node_glob[n] = g;
  }
  std::vector<Glob> kept;
  std::vector<int> remap(L.globs.size(), -1);
  for (size_t g = 0; g < L.globs.size(); ++g) {
    Glob& gl = L.globs[g];
    for (int n : gl.nodes)
      for (int p = in.node_dof_ptr[n]; p < in.node_dof_ptr[n + 1]; ++p) gl.dofs.push_back(in.node_dofs[p]);
    std::sort(gl.dofs.begin(), gl.dofs.end());
    if (gl.dofs.empty()) continue;
    gl.type = gl.subs.size() == 2 ? GLOB_FACE : (gl.nodes.size() == 1 ? GLOB_CORNER : GLOB_EDGE);
    remap[g] = int(kept.size());
    kept.push_back(gl);
  }
  L.globs.swap(kept);
  // DOF -> node, interface flag
  L.dof_node.assign(in.n_dof, -1);
  for (int n = 0; n < nn; ++n)
    for (int p = in.node_dof_ptr[n]; p < in.node_dof_ptr[n + 1]; ++p) L.dof_node[in.node_dofs[p]] = n;
  for (int j = 0; j < in.n_dof; ++j)
    if (L.dof_node[j] < 0) return "a level DOF belongs to no node";
  // subdomain DOFs: interior then interface, each ascending
  std::vector<std::vector<int>> sd(ns);
  for (int e = 0; e < in.n_elem; ++e) {
    auto& v = sd[in.elem_sub[e]];
    for (int64_t p = in.elem_dof_ptr[e]; p < in.elem_dof_ptr[e + 1]; ++p)
      if (in.elem_dofs[p] >= 0) v.push_back(in.elem_dofs[p]);
  }
  L.subs.assign(ns, Sub());
  for (int s = 0; s < ns; ++s) {
    auto& v = sd[s];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    if (v.empty()) return "subdomain " + std::to_string(s) + " has no free DOF";
    Sub& S = L.subs[s];
    for (int j : v) {
      int n = L.dof_node[j];
      if (nptr[n + 1] - nptr[n] < 2) S.dofs.push_back(j);
    }
    S.nI = int(S.dofs.size());
    for (int j : v) {
      int n = L.dof_node[j];
      if (nptr[n + 1] - nptr[n] >= 2) S.dofs.push_back(j);
    }
    S.nG = int(S.dofs.size()) - S.nI;
  }
  // initial constraints
  L.cons.clear();
  for (size_t g = 0; g < L.globs.size(); ++g) {
    const Glob& gl = L.globs[g];
    if (gl.type == GLOB_CORNER) {
      for (int j : gl.dofs) {
        Constraint c;
        c.glob = int(g);
        c.kind = CONS_UNIT;
        c.dofs = {j};
        L.cons.push_back(c);
      }
    } else if ((gl.type == GLOB_EDGE && edge_averages) || (gl.type == GLOB_FACE && face_averages)) {
      std::vector<int> comps;
      for (int j : gl.dofs) comps.push_back(in.dof_comp[j]);
      std::vector<int> uc = comps;
      std::sort(uc.begin(), uc.end());
      uc.erase(std::unique(uc.begin(), uc.end()), uc.end());
      for (int cc : uc) {
        Constraint c;
        c.glob = int(g);
        c.kind = CONS_AVG;
        for (size_t q = 0; q < gl.dofs.size(); ++q)
          if (comps[q] == cc) c.dofs.push_back(gl.dofs[q]);
        L.cons.push_back(c);
      }
    }
  }
  L.n_cons_initial = int(L.cons.size());
  // pairs: one per face glob
  L.pairs.clear();
  for (size_t g = 0; g < L.globs.size(); ++g) {
    const Glob& gl = L.globs[g];
    if (gl.type != GLOB_FACE) continue;
    Pair P;
    P.s = gl.subs[0];
    P.t = gl.subs[1];
    P.glob = int(g);
    P.face_dofs = gl.dofs;
    L.pairs.push_back(P);
  }
  L.sub_npairs.assign(ns, 0);
  for (auto& P : L.pairs) {
    P.slot_s = L.sub_npairs[P.s]++;
    P.slot_t = L.sub_npairs[P.t]++;
    P.both_floating = in.sub_floating[P.s] && in.sub_floating[P.t];
    const Sub& S = L.subs[P.s];
    const Sub& T = L.subs[P.t];
    // shared interface DOFs (both interface lists are ascending)
    int a = S.nI, b = T.nI;
    const int ae = S.nI + S.nG, be = T.nI + T.nG;
    while (a < ae && b < be) {
      if (S.dofs[a] < T.dofs[b]) ++a;
      else if (S.dofs[a] > T.dofs[b]) ++b;
      else {
        P.sh_s.push_back(a - S.nI);
        P.sh_t.push_back(b - T.nI);
        ++a;
        ++b;
      }
    }
    if (keep_edges) {
      // rows on every shared DOF (ascending level ids, like the intersection)
      P.face_dofs.clear();
      for (int q : P.sh_s) P.face_dofs.push_back(S.dofs[S.nI + q]);
      P.face_s = P.sh_s;
      P.face_t = P.sh_t;
    } else {
      for (int j : P.face_dofs) {
        int is = lower_index(S.dofs, j, S.nI, S.nI + S.nG);
        int it = lower_index(T.dofs, j, T.nI, T.nI + T.nG);
        if (is < 0 || it < 0) return "face DOF missing from a subdomain interface";
        P.face_s.push_back(is);
        P.face_t.push_back(it);
      }
    }
  }
  add_adaptive_constraints(L, std::vector<int>(L.pairs.size(), 0));
  return "";
}

void add_adaptive_constraints(LevelPlan& L, const std::vector<int>& k) {
  for (size_t p = 0; p < L.pairs.size(); ++p) {
    for (int r = 0; r < k[p]; ++r) {
      Constraint c;
      c.glob = L.pairs[p].glob;
      c.kind = CONS_ADAPT;
      c.dofs = L.pairs[p].face_dofs;
      c.pair = int(p);
      c.row = r;
      L.cons.push_back(c);
    }
  }
  for (auto& S : L.subs) S.cons.clear();
  for (size_t c = 0; c < L.cons.size(); ++c)
    for (int s : L.globs[L.cons[c].glob].subs) L.subs[s].cons.push_back(int(c));
  for (auto& P : L.pairs) {
    const auto& cs = L.subs[P.s].cons;
    const auto& ct = L.subs[P.t].cons;
    P.dr_s.clear();
    P.dr_t.clear();
    // shared coarse DOFs of the initial set (rows of D); adaptive ones are
    // only used once the pair problems are solved
    size_t a = 0, b = 0;
    while (a < cs.size() && b < ct.size()) {
      if (cs[a] < ct[b]) ++a;
      else if (cs[a] > ct[b]) ++b;
      else {
        if (L.cons[cs[a]].kind != CONS_ADAPT) {
          P.dr_s.push_back(int(a));
          P.dr_t.push_back(int(b));
        }
        ++a;
        ++b;
      }
    }
    std::vector<int> uni(cs);
    uni.insert(uni.end(), ct.begin(), ct.end());
    std::sort(uni.begin(), uni.end());
    uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
    P.n_cp = int(uni.size());
    P.pc_s.resize(cs.size());
    P.pc_t.resize(ct.size());
    for (size_t r = 0; r < cs.size(); ++r)
      P.pc_s[r] = int(std::lower_bound(uni.begin(), uni.end(), cs[r]) - uni.begin());
    for (size_t r = 0; r < ct.size(); ++r)
      P.pc_t[r] = int(std::lower_bound(uni.begin(), uni.end(), ct[r]) - uni.begin());
  }
}

std::string next_level_input(const LevelPlan& L, const std::vector<int>& parent, LevelInput& out) {
  const LevelInput& in = L.in;
  if (int(parent.size()) != in.n_sub) return "parent map size differs from the subdomain count";
  out = LevelInput();
  out.dof_per_node = in.dof_per_node;
  out.n_rb = in.n_rb;
  out.n_dof = int(L.cons.size());
  std::vector<std::vector<int>> gcons(L.globs.size());
  for (size_t c = 0; c < L.cons.size(); ++c) gcons[L.cons[c].glob].push_back(int(c));
  std::vector<int> node_of_glob(L.globs.size(), -1);
  out.node_dof_ptr.push_back(0);
  for (size_t g = 0; g < L.globs.size(); ++g) {
    if (gcons[g].empty()) continue;
    node_of_glob[g] = out.n_node++;
    for (int c : gcons[g]) out.node_dofs.push_back(c);
    out.node_dof_ptr.push_back(int(out.node_dofs.size()));
  }
  out.dof_comp.assign(out.n_dof, -1);
  for (size_t c = 0; c < L.cons.size(); ++c) {
    const Constraint& C = L.cons[c];
    if (C.kind == CONS_ADAPT) continue;
    int c0 = in.dof_comp[C.dofs[0]];
    bool same = true;
    for (int j : C.dofs) same = same && in.dof_comp[j] == c0;
    if (same) out.dof_comp[c] = c0;
  }
  out.n_elem = in.n_sub;
  int np = 0;
  for (int s = 0; s < in.n_sub; ++s) {
    if (parent[s] < 0) return "negative parent id";
    np = std::max(np, parent[s] + 1);
  }
  out.n_sub = np;
  out.elem_sub = parent;
  out.elem_dof_ptr.push_back(0);
  out.elem_node_ptr.push_back(0);
  for (int s = 0; s < in.n_sub; ++s) {
    const auto& cs = L.subs[s].cons;
    for (int c : cs) out.elem_dofs.push_back(c);
    out.elem_dof_ptr.push_back(int64_t(out.elem_dofs.size()));
    std::vector<int> nodes;
    for (int c : cs) nodes.push_back(node_of_glob[L.cons[c].glob]);
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    for (int n : nodes) out.elem_nodes.push_back(n);
    out.elem_node_ptr.push_back(int64_t(out.elem_nodes.size()));
  }
  out.sub_floating.assign(np, 1);
  for (int s = 0; s < in.n_sub; ++s)
    if (!in.sub_floating[s]) out.sub_floating[parent[s]] = 0;
  return "";
}

}  // namespace ambddc
