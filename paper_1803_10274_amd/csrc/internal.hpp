// Internal types shared by the libkrr translation units.
#pragma once

#include <array>
#include <vector>

#include "common.hpp"

struct krr_tree_s {
    int64_t n = 0;
    // n_nodes rows of (begin, end, left, right, parent), postorder, root last.
    std::vector<int64_t> nodes;
    std::array<int64_t, 4> stats{{0, 0, 0, 0}};
    int64_t n_nodes() const { return (int64_t)nodes.size() / 5; }
    int64_t b(int64_t i) const { return nodes[5 * i]; }
    int64_t e(int64_t i) const { return nodes[5 * i + 1]; }
    int64_t left(int64_t i) const { return nodes[5 * i + 2]; }
    int64_t right(int64_t i) const { return nodes[5 * i + 3]; }
    int64_t parent(int64_t i) const { return nodes[5 * i + 4]; }
    bool leaf(int64_t i) const { return nodes[5 * i + 2] < 0; }
};

namespace krr {

// Per-node bookkeeping of a compressed HSS matrix (host side).
struct HNode {
    int64_t b, e, left, right, parent;
    int32_t height;   // 0 at leaves, 1 + max(children) above
    int32_t m;        // rows of U: leaf size, or k_left + k_right
    int32_t k;        // rank (columns of U); 0 at the root
    int64_t offU;     // into U pool (m * k doubles), -1 at the root
    int64_t offD;     // into D pool (leaf: m * m doubles), -1 otherwise
    int64_t offB;     // into B pool (k_left * k_right), -1 at leaves
    int64_t offJ;     // into J pool (k int32 positions), -1 at the root
};

// Nodes grouped by height: every node's children have smaller height, so a
// level is a batch of independent nodes for bottom-up sweeps.
std::vector<std::vector<int>> levels_by_height(std::vector<HNode> &nodes);

void validate_tree(const krr_tree_s *t);

// Diagnostic logging to stderr when the environment sets KRR_VERBOSE.
bool verbose();

}  // namespace krr

struct hss_s {
    int64_t n = 0;
    int32_t d = 0;
    double h = 0;
    std::vector<krr::HNode> node;
    std::vector<std::vector<int>> levels;
    krr::DBuf U, D, B, J;     // generator pools (FP64, FP64, FP64, int32)
    int64_t nU = 0, nD = 0, nB = 0, nJ = 0;
    int32_t r_final = 0, regrowths = 0, max_rank = 0, truncated = 0;
};

struct hss_ulv_s {
    int64_t n = 0;
    double lambda = 0;
    std::vector<krr::HNode> node;       // copy of the HSS node table
    std::vector<std::vector<int>> levels;
    // Per node: Householder vectors of U's QR (m x k, column j = reflector j),
    // tau (k), Cholesky factor L of the eliminated block ((m-k)^2), and
    // W = A_ce L^{-T} (k x (m-k)).  The root holds the Cholesky factor of its
    // whole reduced block in L.
    std::vector<int64_t> offV, offT, offL, offW;
    krr::DBuf V, T, L, W;
    int64_t nV = 0, nT = 0, nL = 0, nW = 0;
};
