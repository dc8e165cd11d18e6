// Binary tree over the cubic lattice and its U(1) leg sectors.
#pragma once

#include <map>
#include <vector>

#include "common.h"
#include "model.h"

namespace qed {

// Tree (Methods, "Tensor Networks"): bottom nodes merge x-neighbours,
// the next layer y-neighbours, then z, cyclically (an axis is skipped
// once a block spans the lattice).  Site s is link s; node n's parent leg
// is link N + n; the root's parent leg ("top") has dimension 1 and
// carries the total charge.  Nodes are numbered layer by layer, inside a
// layer by the (z, y, x) order of the block origin (the sweep order).
struct Tree {
    int N = 0;
    struct Node {
        int l, r, p;      // links
        int layer;
        int origin[3];
    };
    std::vector<Node> nodes;
    std::vector<std::vector<int>> sites_of;   // per link, ascending
    std::vector<int> parent_node;             // per link: node holding it as child, or -1
    std::vector<int> parent_side;             // 0 = l, 1 = r
    int root = -1, top = -1;
    void build(const Lattice& lat);
    std::vector<int> path(int a, int b) const;
    int nlinks() const { return N + (int)nodes.size(); }
};

// Deterministic sector allocation (exact caps, proportional split of chi
// with integer largest remainder, consistency with every QR of the tree).
std::vector<Leg> allocate_sectors(const Tree& tree, const std::vector<Leg>& site_legs,
                                  int Q, int chi);

}  // namespace qed
