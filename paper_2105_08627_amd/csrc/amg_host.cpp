// Aggregation multigrid for the Schur complement S = A_F Y^-1 A_F^T of the
// preconditioner (eqs. 12-15), host setup.  The paper inverts S with an
// aggregation-based algebraic multigrid (AGMG); this is an own implementation
// of pairwise aggregation as published by Notay: each level pairs every node
// with its strongest negatively coupled unpaired neighbour, twice; the coarse
// matrix is the Galerkin product P^T S P with the piecewise-constant
// prolongation P.  Coarsening stops at kAmgCoarse nodes or when a level no
// longer shrinks.
//
// With the linear basis functions S has positive couplings (between opposite
// faces of a voxel) and its coarse graphs turn star-shaped (many nodes whose
// only coupling is to one hub): strict pairing stalls, since a hub takes one
// partner per pass and the rest stay single.  For such an S a node left
// single by a pass joins the pair of its dominant neighbour (at least half of
// its total negative coupling); its smooth-mode value follows that
// neighbour's, so the merge keeps the coarse space's quality.  An S without
// positive couplings (piecewise-constant functions only) is paired strictly.
//
// Rows without couplings (Dirichlet nodes, which keep identity rows, and the
// one-node remainders of isolated lines) are solved exactly by their diagonal
// on their level and left out of the coarser ones.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "host_math.h"

namespace svh {

namespace {

bool decoupled_row(const AmgLevel& L, int i) {
  for (int q = L.rptr[i]; q < L.rptr[i + 1]; ++q)
    if (L.col[q] != i && L.val[q] != 0) return false;
  return true;
}

// Pairwise matching on the CSR matrix of one level: agg[i] = aggregate of i,
// or -1 for a decoupled row when drop is set (its diagonal solves it exactly,
// so it is left out of the coarser levels).  Candidates of i: unmatched j with
// -a_ij >= beta * max_k(-a_ik); i is paired with the candidate of the most
// negative coupling, else left single (and may then join a neighbour's pair).
int pair_once(const AmgLevel& L, std::vector<int>& agg, bool drop, bool join) {
  const int n = L.n;
  agg.assign(n, -2);  // -2 unvisited
  int nc = 0;
  const double beta = 0.25, kJoinDominance = 0.5;
  for (int i = 0; i < n; ++i) {
    if (agg[i] != -2) continue;
    if (drop && decoupled_row(L, i)) {
      agg[i] = -1;
      continue;
    }
    double strongest = 0;
    for (int q = L.rptr[i]; q < L.rptr[i + 1]; ++q)
      if (L.col[q] != i) strongest = std::max(strongest, -L.val[q]);
    int best = -1;
    double bv = 0;
    if (strongest > 0)
      for (int q = L.rptr[i]; q < L.rptr[i + 1]; ++q) {
        const int j = L.col[q];
        if (j == i || agg[j] != -2) continue;
        const double s = -L.val[q];
        if (s >= beta * strongest && s > bv) {
          bv = s;
          best = j;
        }
      }
    agg[i] = nc;
    if (best >= 0) agg[best] = nc;
    ++nc;
  }
  if (!join) return nc;
  // single nodes join the pair of their dominant neighbour (pairs formed in
  // this pass only, so no chains), then aggregates are renumbered densely
  std::vector<int> size(nc, 0), into(nc, -1);
  for (int i = 0; i < n; ++i)
    if (agg[i] >= 0) size[agg[i]]++;
  for (int i = 0; i < n; ++i) {
    if (agg[i] < 0 || size[agg[i]] != 1) continue;
    double total = 0, bv = 0;
    int bj = -1;
    for (int q = L.rptr[i]; q < L.rptr[i + 1]; ++q)
      if (L.col[q] != i && L.val[q] < 0) {
        total -= L.val[q];
        if (-L.val[q] > bv) {
          bv = -L.val[q];
          bj = L.col[q];
        }
      }
    if (bj >= 0 && agg[bj] >= 0 && size[agg[bj]] >= 2 && bv >= kJoinDominance * total) into[agg[i]] = agg[bj];
  }
  std::vector<int> label(nc, -1);
  int m = 0;
  for (int a = 0; a < nc; ++a)
    if (into[a] < 0) label[a] = m++;
  for (int i = 0; i < n; ++i)
    if (agg[i] >= 0) agg[i] = label[into[agg[i]] >= 0 ? into[agg[i]] : agg[i]];
  return m;
}

// Galerkin product of a piecewise-constant prolongation: C = P^T A P (rows
// and columns with agg < 0 are left out).
AmgLevel galerkin(const AmgLevel& A, const std::vector<int>& agg, int nc) {
  AmgLevel C;
  C.n = nc;
  std::vector<std::vector<int>> members(nc);
  for (int i = 0; i < A.n; ++i)
    if (agg[i] >= 0) members[agg[i]].push_back(i);
  C.rptr.assign(nc + 1, 0);
  std::vector<double> acc(nc, 0.0);
  std::vector<int> mark(nc, -1), cols;
  for (int I = 0; I < nc; ++I) {
    cols.clear();
    for (int i : members[I])
      for (int q = A.rptr[i]; q < A.rptr[i + 1]; ++q) {
        const int J = agg[A.col[q]];
        if (J < 0) continue;
        if (mark[J] != I) {
          mark[J] = I;
          acc[J] = 0;
          cols.push_back(J);
        }
        acc[J] += A.val[q];
      }
    std::sort(cols.begin(), cols.end());
    for (int J : cols) {
      C.col.push_back(J);
      C.val.push_back(acc[J]);
    }
    C.rptr[I + 1] = (int)C.col.size();
  }
  return C;
}

}  // namespace

// S over all M nodes: rows of free nodes from the incidence matrix (CSR rows
// of A, CSC columns), identity rows for Dirichlet nodes.
AmgLevel schur_matrix(const Topology& t, const std::vector<char>& dirichlet, const std::vector<double>& ydiag) {
  AmgLevel S;
  const int M = t.M;
  S.n = M;
  S.rptr.assign(M + 1, 0);
  std::vector<double> acc(M, 0.0);
  std::vector<int> mark(M, -1), cols;
  for (int m = 0; m < M; ++m) {
    cols.clear();
    if (dirichlet[m]) {
      cols.push_back(m);
      acc[m] = 1.0;
    } else {
      for (int q = t.rptr[m]; q < t.rptr[m + 1]; ++q) {
        const int b = t.rcol[q];
        const double am = t.rval[q] / ydiag[b];
        for (int k = t.cptr[b]; k < t.cptr[b + 1]; ++k) {
          const int n = t.crow[k];
          if (dirichlet[n]) continue;
          if (mark[n] != m) {
            mark[n] = m;
            acc[n] = 0;
            cols.push_back(n);
          }
          acc[n] += am * t.cval[k];
        }
      }
      if (cols.empty()) {  // isolated free node (cannot occur for a connected grid)
        cols.push_back(m);
        acc[m] = 1.0;
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int n : cols) {
      S.col.push_back(n);
      S.val.push_back(acc[n]);
    }
    S.rptr[m + 1] = (int)S.col.size();
  }
  return S;
}

bool has_positive_coupling(const AmgLevel& A) {
  for (int i = 0; i < A.n; ++i)
    for (int q = A.rptr[i]; q < A.rptr[i + 1]; ++q)
      if (A.col[q] != i && A.val[q] > 0) return true;
  return false;
}

int amg_setup(AmgLevel fine, std::vector<AmgLevel>& levels, std::vector<std::vector<int>>& aggs,
              std::vector<double>& coarse_inv) {
  levels.clear();
  aggs.clear();
  levels.push_back(std::move(fine));
  const bool join = has_positive_coupling(levels[0]);
  while (levels.back().n > kAmgCoarse && (int)levels.size() < kAmgMaxLevels) {
    const AmgLevel& A = levels.back();
    int coupled = 0;
    for (int i = 0; i < A.n; ++i) coupled += decoupled_row(A, i) ? 0 : 1;
    // two pairing passes: aggregates of up to four nodes; decoupled rows drop out
    std::vector<int> a1, a2;
    const int n1 = pair_once(A, a1, true, join);
    AmgLevel A1 = galerkin(A, a1, n1);
    const int n2 = pair_once(A1, a2, false, join);
    std::vector<int> agg(A.n);
    for (int i = 0; i < A.n; ++i) agg[i] = a1[i] >= 0 ? a2[a1[i]] : -1;
    if (n2 == 0 || n2 > 0.9 * coupled) break;  // nothing left, or no longer coarsening
    levels.push_back(galerkin(A, agg, n2));
    aggs.push_back(std::move(agg));
  }
  // coarsest level: diagonal (the piecewise-constant functions alone couple
  // only the faces along one line, so coarsening ends with one node per line)
  // -> solved by its diagonal; small -> dense inverse; else damped Jacobi
  const AmgLevel& C = levels.back();
  const int n = C.n;
  bool diagonal = true;
  for (int i = 0; i < n && diagonal; ++i)
    for (int q = C.rptr[i]; q < C.rptr[i + 1]; ++q)
      if (C.col[q] != i && C.val[q] != 0) {
        diagonal = false;
        break;
      }
  coarse_inv.clear();
  if (diagonal) return kAmgCoarseDiagonal;
  if (n > kAmgCoarseMax) return kAmgCoarseJacobi;
  // exact inverse of the coarsest matrix (dense Gauss-Jordan with partial pivoting)
  std::vector<double> a((size_t)n * n, 0.0), inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int q = C.rptr[i]; q < C.rptr[i + 1]; ++q) a[(size_t)i * n + C.col[q]] = C.val[q];
    inv[(size_t)i * n + i] = 1.0;
  }
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[(size_t)i * n + k]) > std::fabs(a[(size_t)piv * n + k])) piv = i;
    if (a[(size_t)piv * n + k] == 0) return -1;
    if (piv != k)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)k * n + j], a[(size_t)piv * n + j]);
        std::swap(inv[(size_t)k * n + j], inv[(size_t)piv * n + j]);
      }
    const double d = 1.0 / a[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      a[(size_t)k * n + j] *= d;
      inv[(size_t)k * n + j] *= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[(size_t)i * n + k];
      if (f == 0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
        inv[(size_t)i * n + j] -= f * inv[(size_t)k * n + j];
      }
    }
  }
  coarse_inv = std::move(inv);
  return kAmgCoarseDense;
}

}  // namespace svh
