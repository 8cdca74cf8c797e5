// Host-side data structures: geometry tables in cluster-tree order, the
// cluster tree and the block partition of the hierarchical matrix.
#pragma once

#include <cstdint>
#include <vector>

namespace ewbem {

struct HostGeom {
  int ne = 0;
  std::vector<int> perm;      // perm[tree index] = caller's element index
  std::vector<int> iperm;     // iperm[caller index] = tree index
  std::vector<double> cen;    // [ne][3]
  std::vector<double> nrm;    // [ne][3]
  std::vector<double> area;   // [ne]
  std::vector<double> qp;     // [ne][7][3]
  std::vector<double> qw;     // [ne][7]
  std::vector<double> vtx;    // [ne][3][3]
};

struct Cluster {
  int begin = 0, end = 0;     // element range in tree order
  double lo[3], hi[3];        // bounding box of the elements' vertices
  int child[2] = {-1, -1};
  int level = 0;
  bool leaf() const { return child[0] < 0; }
  int size() const { return end - begin; }
};

struct BlockPair {
  int row, col;               // cluster indices
};

struct Partition {
  std::vector<Cluster> clusters;
  std::vector<int> leaves;    // leaf cluster indices in tree order
  std::vector<BlockPair> near, far;
};

// Degree-5 seven-point rule on a triangle: barycentric points and weights
// (summing to one).
void radon7(double bary[7][3], double w[7]);

// n-point Gauss-Legendre nodes and weights on [0, 1].
void gauss_legendre01(int n, double* x, double* w);

// Geometry of a flat-triangle mesh.  ``exterior``: the solid lies outside
// the closed surface(s) (cavities), so normals point into the enclosed
// volume.  Element order is permuted into cluster-tree order by ``tree``.
void build_geometry(int nv, const double* xyz, int nt, const int32_t* tri, bool exterior,
                    const std::vector<int>& perm, HostGeom& g);

// Cluster tree: recursive median bisection of element centroids along the
// longest side of their bounding box, down to at most ``leaf_size`` elements.
// Returns the permutation (tree index -> caller index).
std::vector<int> build_tree(int nv, const double* xyz, int nt, const int32_t* tri, int leaf_size,
                            std::vector<Cluster>& clusters);

// Block partition: (tau, sigma) is admissible (low rank) when
// min(diam tau, diam sigma) <= eta * dist(tau, sigma) with bounding-box
// diameters and distances; eta <= 0 makes every block near (dense).  An
// admissible pair with more than max_far elements on a side is split into
// its child pairs (admissible as well) until both sides fit.
void build_partition(double eta, Partition& p, int max_far);

}  // namespace ewbem
