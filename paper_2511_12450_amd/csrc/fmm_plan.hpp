// FMM plan shared by the matvec and the preconditioner.
#pragma once
#include <vector>

#include "lm_internal.hpp"

constexpr int MAXP = 31;  // 2p+1 <= 63 fits one 64-lane wavefront

struct BoxDev {
  double cx, ch, k;
  int tree, level, parent, pos;
  int pt0, npt, child0, nchild;
};

struct FmmPlan {
  int p = 20, P = 41;
  int bc = 0;           // boundary condition (lm_bc): the targets see n . grad + i beta of the operator
  double beta = 0.0;    // impedance of the Robin condition
  std::vector<int> tree_side;  // side (coordinate h) of every tree
  int nlev = 0, lf = 0, lr = 0;
  double w_top = 0, x0 = 0;
  int n_boxes = 0;
  int64_t n_el = 0;               // boundary elements N
  std::vector<BoxDev> boxes;
  std::vector<int> level_ptr;     // boxes of level l: ids [level_ptr[l], level_ptr[l+1])
  std::vector<int> leaf_free, leaf_B, leaf_T;  // leaf boxes by tree class
  std::vector<int> pt_item;       // (leaf, first point, count) work items, by class
  int item_ptr[4] = {0, 0, 0, 0}; // items of class c: [item_ptr[c], item_ptr[c+1])
  std::vector<int> p2m_leaf, p2m_ptr;  // every leaf and the range of its items
  std::vector<int> p2m_dst;   // per item: its leaf when the leaf has one item (written directly), else -1
  std::vector<int> p2m_msel;  // positions (in p2m_leaf) of the leaves with several items
  std::vector<int> parents_by_level;           // boxes with children, grouped by level
  std::vector<int> parents_ptr;
  std::vector<int> children;
  std::vector<int> pt_elem;
  std::vector<double> pt_xh;      // (x, h) per point
  // M2L lists
  std::vector<int> m2l_tgt, m2l_ptr, m2l_src, m2l_tab;  // tab >= 0 reaction table, < 0: free table -(id+1)
  std::vector<double> free_geo;   // (k, dx, dh) per free table
  std::vector<int> free_lvl;      // (layer, level) per free table
  std::vector<int> reac_meta;     // (lt, ls, comp, level) per reaction table
  std::vector<double> reac_geo;   // (dx, ht, hs)
  // free near field
  std::vector<int> near_tgt, near_ptr, near_src;
  // reaction near field (pairs with their component masks)
  std::vector<int> rn_ptr, rn_src;
  std::vector<unsigned> rn_mask;
  std::vector<int> rn_rows;  // rows with reaction near pairs
  // near-field matrix (CSR by element, input numbering): free-space near
  // pairs, reaction near pairs and the self term, values precomputed
  std::vector<int> nm_ptr, nm_src;
  // M2L entries grouped by operator (reaction tables, then free classes)
  std::vector<int> tm_ptr, tm_slot, tm_src;
  std::vector<int> tm_item;  // (operator, first entry, end) work items
  // (target, first entry, end) items of the matrix-core M2L, longest first;
  // mf_slot: each item's partial slot (slots in target order, mf_ptr: slots per target)
  std::vector<int> mf_item, mf_slot, mf_ptr;
  std::vector<int> tr_item, tr_src, tr_op;  // matrix-core M2M (per parent) and L2L (per box) items
  // spectral rule: corrections of the same-scatterer pairs (CSR by node)
  std::vector<int> sc_ptr, sc_src;
  // free-space near field + self terms as leaf blocks: rows = the leaf's
  // elements, columns = the leaf's and its neighbours' elements
  std::vector<int> nb_jptr, nb_jidx, nb_rows, nb_item;
  std::vector<int64_t> nb_zoff;
  int64_t nb_nnz = 0;
  int l2l_item0 = 0;
  // level 0 by FFT along x: rows (tree, j) of level-0 boxes over top_nx
  // columns, transforms of length top_L (a power of two >= 2 top_nx - 1);
  // operator classes (one Toeplitz operator sequence per class) and the
  // frequency-domain M2L items (row * top_L + frequency, first entry, end)
  bool top_on = false;
  int top_rows = 0, top_nx = 0, top_L = 0, top_ncls = 0;
  int64_t top_direct = 0;  // level-0 list entries the transform replaces
  std::vector<int> top_grid;  // [row][top_nx] -> level-0 box or -1
  std::vector<int> top_item, top_ptr, top_src, top_op;
  int n_reac_tab = 0, n_free_tab = 0;
  // expansion scales sig[layer][level][0..p]; translation operators, P x P
  // each, column-major by input: [M2M: layer, level, pos][L2L: same][M2L]
  std::vector<double> sig;
  int n_tree_ops = 0, op_m2l = 0;
  std::vector<int> tree_layer;
  int n_layers = 0;
  int64_t stats[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};

  DevBuf d_boxes, d_children, d_pt_elem, d_pt_xh;
  DevBuf d_pt_item, d_p2m_leaf, d_p2m_ptr, d_p2m_part, d_parents;
  DevBuf d_m2l_tgt, d_m2l_ptr, d_m2l_src, d_m2l_tab;
  DevBuf d_sig, d_ops64, d_ops32, d_m2l_op;
  DevBuf d_near_tgt, d_near_ptr, d_near_src;
  DevBuf d_rn_ptr, d_rn_src, d_rn_val, d_rn_rows;
  DevBuf d_p2m_Z32, d_l2p_Z32;  // point matrices of the matrix-core P2M / L2P
  DevBuf d_self, d_me, d_le, d_tree_layer;
  DevBuf d_tr_item, d_tr_src, d_tr_op, d_box_id;
  DevBuf d_nb_jptr, d_nb_jidx, d_nb_rows, d_nb_item, d_nb_zoff, d_nb_Z32, d_rn_val32, d_xt;
  DevBuf d_nm_ptr, d_nm_src, d_nm_val, d_nm_val32, d_mf_item, d_mf_slot, d_mf_ptr, d_mf_part, d_tm_item, d_tm_ptr, d_tm_slot, d_tm_src, d_m2l_out;
  DevBuf d_top_grid, d_top_item, d_top_ptr, d_top_src, d_top_op, d_top_id, d_top_tw64, d_top_tw32;
  DevBuf d_top_T64, d_top_T32, d_top_mh, d_top_lh;
  DevBuf d_om_slot;  // per-entry M2L results of the few-right-hand-side (operator-major) launch
  DevBuf d_sc_ptr, d_sc_src, d_sc_val, d_sc_val32;
  DevBuf d_tree_side, d_l2p_Z64;  // sound-hard / impedance: per-tree side, FP64 L2P rows
  std::vector<int> le_zero;  // boxes no M2L or level-0 launch writes: their local expansions start at zero
  DevBuf d_le_zero;
  DevBuf d_p2m_dst, d_p2m_msel;
  int r_cap = 0;  // right-hand sides the expansion buffers hold
  // side stream of the near field (default priority) and its fork / join events
  hipStream_t s_near = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  FmmPlan() = default;
  FmmPlan(const FmmPlan&) = delete;
  FmmPlan& operator=(const FmmPlan&) = delete;
  ~FmmPlan() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (s_near) (void)hipStreamDestroy(s_near);
  }
  int64_t bytes() const {
    const DevBuf* all[] = {&d_boxes, &d_children, &d_pt_elem, &d_pt_xh, &d_pt_item, &d_p2m_leaf, &d_p2m_ptr,
                           &d_p2m_part, &d_parents, &d_m2l_tgt, &d_m2l_ptr, &d_m2l_src, &d_m2l_tab, &d_sig, &d_ops64,
                           &d_ops32, &d_m2l_op, &d_near_tgt, &d_near_ptr, &d_near_src, &d_rn_ptr, &d_rn_src,
                           &d_rn_val, &d_rn_rows, &d_p2m_Z32, &d_l2p_Z32, &d_self, &d_me, &d_le, &d_tree_layer,
                           &d_nm_ptr, &d_nm_src, &d_nm_val, &d_nm_val32, &d_nb_jptr, &d_nb_jidx, &d_nb_rows,
                           &d_nb_item, &d_nb_zoff, &d_nb_Z32, &d_rn_val32, &d_xt, &d_tr_item, &d_tr_src, &d_tr_op,
                           &d_box_id, &d_mf_item, &d_mf_slot, &d_mf_ptr, &d_mf_part, &d_tm_item, &d_tm_ptr, &d_tm_slot, &d_tm_src,
                           &d_m2l_out, &d_top_grid, &d_top_item, &d_top_ptr, &d_top_src, &d_top_op, &d_top_id,
                           &d_top_tw64, &d_top_tw32, &d_top_T64, &d_top_T32, &d_top_mh, &d_top_lh,
                           &d_om_slot, &d_p2m_dst, &d_p2m_msel, &d_sc_ptr, &d_sc_src, &d_sc_val,
                           &d_sc_val32, &d_tree_side, &d_l2p_Z64, &d_le_zero};
    int64_t b = 0;
    for (auto* d : all) b += d->bytes;
    return b;
  }
};

// Grow the expansion buffers to hold r right-hand sides per launch.
lm_status fmm_reserve(FmmPlan* F, int r);
