// Face-node topology of the saddle system (eq. 7), host side.
//
// Nodes sit at the centres of the faces of non-empty voxels (Sec. II.A); a
// face shared by two non-empty voxels is one node.  Entry A[m, (k, a)] is the
// current the piecewise-constant basis f^a of voxel k (total current 1) draws
// from node m into the voxel: +1 at its -a face, -1 at its +a face, so that
// A I = 0 is current conservation (eq. 2) at every node and the first block
// row of eq. 7 reads Z I - A^T Phi = V.  The linear functions of eqs. 5-6
// (same normalisation) have zero net flux: f^2D draws -1/2 through each x face
// and +1/2 through each y face, f^3D draws -1/2 through each of the four x
// and y faces and +1 through each z face.
#include <algorithm>
#include <numeric>
#include <vector>

#include "host_math.h"

namespace svh {

namespace {
struct FaceIndex {
  int K[3];
  long long off[3];
  long long id(int axis, int x, int y, int z) const {
    // face grid of `axis` has K[axis] + 1 positions along that axis
    if (axis == 0) return off[0] + ((long long)z * K[1] + y) * (K[0] + 1) + x;
    if (axis == 1) return off[1] + ((long long)z * (K[1] + 1) + y) * K[0] + x;
    return off[2] + ((long long)z * K[1] + y) * K[0] + x;
  }
};
}  // namespace

int build_topology(const int K[3], const int32_t* vidx, int nvox, int basis, Topology& t) {
  if (basis != 3 && basis != 5) return -1;
  FaceIndex fi;
  for (int a = 0; a < 3; ++a) fi.K[a] = K[a];
  fi.off[0] = 0;
  fi.off[1] = (long long)(K[0] + 1) * K[1] * K[2];
  fi.off[2] = fi.off[1] + (long long)K[0] * (K[1] + 1) * K[2];
  const long long nfaces = fi.off[2] + (long long)K[0] * K[1] * (K[2] + 1);
  std::vector<int32_t> node(nfaces, -1);
  t.coords.assign((size_t)3 * nvox, 0);
  for (int z = 0; z < K[2]; ++z)
    for (int y = 0; y < K[1]; ++y)
      for (int x = 0; x < K[0]; ++x) {
        const int k = vidx[((size_t)z * K[1] + y) * K[0] + x];
        if (k < 0) continue;
        t.coords[3 * (size_t)k] = x;
        t.coords[3 * (size_t)k + 1] = y;
        t.coords[3 * (size_t)k + 2] = z;
      }
  // number nodes in face-grid order (x faces, then y faces, then z faces)
  std::vector<char> used(nfaces, 0);
  for (int k = 0; k < nvox; ++k) {
    const int x = t.coords[3 * k], y = t.coords[3 * k + 1], z = t.coords[3 * k + 2];
    used[fi.id(0, x, y, z)] = used[fi.id(0, x + 1, y, z)] = 1;
    used[fi.id(1, x, y, z)] = used[fi.id(1, x, y + 1, z)] = 1;
    used[fi.id(2, x, y, z)] = used[fi.id(2, x, y, z + 1)] = 1;
  }
  int M = 0;
  for (long long f = 0; f < nfaces; ++f)
    if (used[f]) node[f] = M++;
  t.M = M;
  t.C = basis;
  t.nvox = nvox;
  // voxel face -> node, face code 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z
  t.face_node.assign((size_t)6 * nvox, -1);
  for (int k = 0; k < nvox; ++k) {
    const int x = t.coords[3 * k], y = t.coords[3 * k + 1], z = t.coords[3 * k + 2];
    t.face_node[6 * (size_t)k + 0] = node[fi.id(0, x, y, z)];
    t.face_node[6 * (size_t)k + 1] = node[fi.id(0, x + 1, y, z)];
    t.face_node[6 * (size_t)k + 2] = node[fi.id(1, x, y, z)];
    t.face_node[6 * (size_t)k + 3] = node[fi.id(1, x, y + 1, z)];
    t.face_node[6 * (size_t)k + 4] = node[fi.id(2, x, y, z)];
    t.face_node[6 * (size_t)k + 5] = node[fi.id(2, x, y, z + 1)];
  }
  // CSC (one column per basis function, column index a * nvox + k)
  const int ncol = basis * nvox;
  t.cptr.assign(ncol + 1, 0);
  t.crow.clear();
  t.cval.clear();
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < nvox; ++k) {
      const int col = a * nvox + k;
      t.crow.push_back(t.face_node[6 * (size_t)k + 2 * a]);
      t.cval.push_back(1.0);
      t.crow.push_back(t.face_node[6 * (size_t)k + 2 * a + 1]);
      t.cval.push_back(-1.0);
      t.cptr[col + 1] = (int)t.crow.size();
    }
  if (basis == 5) {
    // face code f: axis f / 2; 2D: -1/2 on x faces, +1/2 on y faces;
    // 3D: -1/2 on x and y faces, +1 on z faces
    const double w2d[3] = {-0.5, 0.5, 0.0}, w3d[3] = {-0.5, -0.5, 1.0};
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < nvox; ++k) {
        const int col = (3 + b) * nvox + k;
        const double* wt = b == 0 ? w2d : w3d;
        for (int f = 0; f < 6; ++f) {
          if (wt[f / 2] == 0.0) continue;
          t.crow.push_back(t.face_node[6 * (size_t)k + f]);
          t.cval.push_back(wt[f / 2]);
        }
        t.cptr[col + 1] = (int)t.crow.size();
      }
  }
  // CSR from CSC
  t.rptr.assign(M + 1, 0);
  for (int r : t.crow) t.rptr[r + 1]++;
  std::partial_sum(t.rptr.begin(), t.rptr.end(), t.rptr.begin());
  t.rcol.assign(t.crow.size(), 0);
  t.rval.assign(t.crow.size(), 0.0);
  std::vector<int> fill(t.rptr.begin(), t.rptr.end() - 1);
  for (int col = 0; col < ncol; ++col)
    for (int q = t.cptr[col]; q < t.cptr[col + 1]; ++q) {
      const int r = t.crow[q];
      t.rcol[fill[r]] = col;
      t.rval[fill[r]] = t.cval[q];
      fill[r]++;
    }
  return 0;
}

// Dirichlet mask: the given port nodes plus one grounded node for every
// connected region (through basis functions) that has no Dirichlet node; the
// conservation rows of such a region sum to zero.
void ground_floating(const Topology& t, std::vector<char>& dirichlet) {
  std::vector<int> parent(t.M);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int i) {
    while (parent[i] != i) {
      parent[i] = parent[parent[i]];
      i = parent[i];
    }
    return i;
  };
  const int ncol = (int)t.cptr.size() - 1;
  for (int col = 0; col < ncol; ++col) {
    const int a = t.crow[t.cptr[col]];
    for (int q = t.cptr[col] + 1; q < t.cptr[col + 1]; ++q) {
      const int ra = find(a), rb = find(t.crow[q]);
      if (ra != rb) parent[rb] = ra;
    }
  }
  std::vector<char> has(t.M, 0);
  for (int m = 0; m < t.M; ++m)
    if (dirichlet[m]) has[find(m)] = 1;
  for (int m = 0; m < t.M; ++m) {
    const int r = find(m);
    if (!has[r]) {
      dirichlet[m] = 1;
      has[r] = 1;
    }
  }
}

}  // namespace svh
