// Static build of the HBS (hierarchically block separable) compressed
// inverse of A_oo = -1/2 I + D + N on the reference wall.  The paper uses the
// HBS compression and inverse of its cited fast direct solver (Gillman, Young
// & Martinsson) as the black-box solver of the reference discretization that
// Algorithm 1 takes as input (Sec. 3.2); this is a from-scratch version of
// that scheme for the Stokes double-layer system.
//
// Tree of contiguous arcs; root = level 0, leaves = level L.  The arcs are
// those of a perfect binary tree, and each tree level takes `merge` binary
// levels at once (merge = 1: binary tree; 2: four children per node; the
// level nearest the root takes what is left), so an apply has fewer
// dependent level sweeps.  Per non-root node tau with input size n (2 * leaf
// nodes at the leaves, the children's skeleton sizes above) and skeleton
// size k:
//   E (n x k), F* (k x n), G (n x n);  root: G_root = D_root^{-1}.
// Apply of A_oo^{-1} b: upward b^ = F* b and g = G b per node (children's
// b^ concatenated form the parent's input), x_root = G_root b_root, downward
// x = E x^ + g.
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"

struct HbsNodeGen {
  int nin = 0, k = 0;
  std::vector<double> E;    // nin x k, column-major
  std::vector<double> Ft;   // k x nin, column-major
  std::vector<double> G;    // nin x nin, column-major
};

struct HbsInverse {
  int L = 0;                                 // leaf level
  std::vector<std::vector<HbsNodeGen>> lev;  // lev[l], l = 1..L (lev[0] unused)
  int nroot = 0;
  std::vector<double> Groot;                 // nroot x nroot, column-major
  int max_rank = 0;
  int64_t entries = 0;                       // sum of |E| + |F| + |G| over all nodes
};

struct HbsParams {
  int leaf_nodes = 64;
  double tol = 1e-10;
  int n_proxy = 48;          // proxy points per circle
  double proxy_ratio = 2.0;  // proxy radius / node radius
  int threads = 0;
  int merge = 1;             // binary levels per tree level (1..4)
};

// Throws RwError(RW_ESINGULAR) on a singular node block.
void hbs_build_inverse(const std::vector<NodeRec>& nodes, const HbsParams& prm, HbsInverse& out);

// Folds tree level 1 into the root: the new root block is the map
// blockdiag(E_1) G_root blockdiag(F*_1) + blockdiag(G_1) from the level-1
// nodes' inputs to their down-sweep outputs (the same operator, one dense
// block), so an apply has two dependent sweeps less.  Only when the new
// root has at most max_root rows and the tree has at least two levels;
// returns whether it folded.
bool hbs_fold_top(HbsInverse& H, int max_root);
