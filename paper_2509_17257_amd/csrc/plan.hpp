// Internal host-side structures of the h2x library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/h2x.h"

namespace h2x {

// Row length of the transposed near blocks and leaf bases of a leaf of nt points: zero-padded
// to a multiple of kRowPad entries, so that the kernels can read two neighbouring rows with
// one load.  (Padding to 16, so that a 16-row tile of an FP64 row is one aligned 128-byte
// line, read with non-temporal loads, measured 2 % faster in the FP64 leaf stage and 1.5 %
// slower in the low-precision one, for 16 % more stored entries.)
constexpr int64_t kRowPad = 2;
constexpr int64_t pad_rows(int64_t nt) { return (nt + kRowPad - 1) / kRowPad * kRowPad; }

// Host topology produced by the planner.  Clusters are numbered in pre-order,
// so the points of every cluster occupy one contiguous range of tree positions.
struct Plan {
    int64_t n = 0;
    h2x_params prm{};
    int32_t p = 0, k = 0;

    std::vector<int64_t> perm;      // tree position -> original index
    std::vector<double> pts_tree;   // n x 3, tree order

    int32_t C = 0;                  // clusters
    std::vector<int32_t> first, size, parent, son0, son1, depth;
    std::vector<double> box;        // C x 6: interpolation box lo[3], hi[3]
    int32_t depth_max = 0;

    std::vector<int32_t> leaves;    // leaf cluster ids, pre-order (= tree-position order)
    std::vector<int32_t> leaf_index;  // cluster id -> leaf index or -1

    // clusters grouped by depth (all clusters) for the level-synchronous passes
    std::vector<int32_t> lvl_ptr;   // depth_max + 2
    std::vector<int32_t> lvl_all;   // cluster ids by depth
    std::vector<int32_t> lvl_inner_ptr;  // depth_max + 2
    std::vector<int32_t> lvl_inner;      // inner cluster ids by depth
    // shallowest depth of a cluster in an admissible block: x-hat above it is
    // never read and y-hat above it stays zero, so the transfer passes stop there
    int32_t adm_depth = 0;

    // admissible leaves, CSR by row cluster
    std::vector<int64_t> adm_ptr;   // C + 1
    std::vector<int32_t> adm_col;   // n_adm
    // near-field leaves, CSR by row leaf (indexed by leaf index)
    std::vector<int64_t> near_ptr;  // L + 1
    std::vector<int32_t> near_col;  // column cluster id
    std::vector<int64_t> near_off;  // offset of the block in the near-field array
    int64_t near_entries = 0;
    // matrix-core layout: near blocks stored transposed with rows padded to pad_rows(|t|),
    // and a per-leaf transposed copy of the leaf basis (k x pad_rows(|t|))
    std::vector<int64_t> near_off_t;
    int64_t near_entries_t = 0;
    std::vector<int64_t> vt_off;    // L
    int64_t vt_entries = 0;
    int32_t max_leaf = 0;           // largest leaf size
    int32_t max_near_rows = 0;      // largest sum of |s| over the near blocks of one leaf

    // column lists for the adjoint: admissible blocks by column cluster (entries are
    // indices into the row-ordered arrays), near-field blocks by column leaf
    std::vector<int64_t> adm_cptr;  // C + 1
    std::vector<int64_t> adm_cblk;  // n_adm
    std::vector<int64_t> near_cptr; // L + 1
    std::vector<int64_t> near_cblk; // n_near

    // launch order of the row clusters in the coupling stage: the rows are cut
    // into 8 contiguous eighths (one per XCD), longest list first within each
    std::vector<int32_t> cpl_order; // C
    // launch order of the leaves in the leaf stage (one contraction per leaf): 8 contiguous
    // eighths (one per XCD), the leaves with the most work first within each, so that the
    // longest leaves do not start last
    std::vector<int32_t> leaf_order; // L
    // positions of each eighth of leaf_order whose near-field entries add up to about half
    // of all (the first half of the near field when it runs in two halves)
    int32_t leaf_half = 0;
    // the same rows in two parts, so that the coupling of the deep part can run beside the
    // upper transfer levels: "deep" rows lie at depth >= split_depth and every inner
    // cluster of their lists too (their x-hat is complete once the upward pass has done
    // split_depth); the other rows form the second part.  Each part in the XCD order of
    // cpl_order.  split_depth 0: no split (too little work in the deep part).
    int32_t split_depth = 0;
    std::vector<int32_t> cpl_deep, cpl_shallow;

    // independent systems (a merged plan is the block-diagonal union of several
    // cluster trees; a plan from build_plan holds one system).  System i owns
    // tree positions / original rows [sys_row[i], sys_row[i+1]), clusters
    // [sys_C[i], sys_C[i+1]), admissible blocks [sys_adm[i], sys_adm[i+1]) and
    // near-field blocks [sys_near[i], sys_near[i+1]); its kernel parameters are sys_prm[i].
    std::vector<h2x_params> sys_prm;
    std::vector<int64_t> sys_row, sys_C, sys_adm, sys_near;
    int32_t nsys() const { return (int32_t)sys_prm.size(); }
};

Plan *build_plan(const double *pts, int64_t n, const h2x_params &prm, std::string &err);
// Block-diagonal union of plans with one Chebyshev order (any sizes, kernels,
// length scales, shifts, leaf sizes and eta): the systems keep their own trees,
// blocks and lists; every per-level array holds the clusters of all systems.
Plan *merge_plans(const std::vector<const Plan *> &parts, std::string &err);

void set_error(const std::string &msg);

}  // namespace h2x
