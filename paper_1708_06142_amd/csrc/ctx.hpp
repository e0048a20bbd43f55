// Host-side context of libocttree (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/octtree.h"
#include "common.hpp"

namespace ot {

enum { BC_ISO = 0, BC_3P = 1, BC_2P1I = 2, BC_1P2I = 3 };
// 1P2I: the analytic line-mass limit beyond this many Lx from the periodic axis
constexpr double RFAR_1P2I = 4.0;

// Device allocation owned by a context; counts bytes against the cap.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct Topology {
  int64_t nb = 0, na = 0;
  int lmax = 0;
  std::vector<int32_t> blev, bcoord;              // leaf blocks (input order)
  std::vector<int32_t> alev, acoord;              // amr nodes, (level, key) order
  std::vector<uint64_t> akey;
  std::vector<int64_t> aleaf, achild;             // leaf id / 8 children
  std::vector<int64_t> bamr;                      // leaf block -> amr index
  std::vector<int64_t> level_begin;               // first amr index per level, [lmax + 2]
  int64_t nroots = 0;
};

// Returns an empty string on success, else the reason the grid is invalid.
std::string build_topology(const int32_t nroot[3], int64_t nb, const int32_t *level,
                           const int32_t *coord, Topology &t);

}  // namespace ot

struct ot_ctx {
  ot_params p;
  int bctype = ot::BC_ISO;
  double box[3];
  std::string err;
  ot::Topology topo;
  bool have_blocks = false;
  bool dev_topo = false;
  bool built = false;
  size_t dev_bytes = 0;
  std::vector<ot::DevBuf *> bufs;
  // topology + moments
  ot::DevBuf alev, acoord, achild0, aleaf, blev, bcoord, bamr, amc, aS, btmc, cm, flag;
  // MPE moments: {B_2, B_3} of the amr and +1/+2 nodes, and the (amr node,
  // leaf block) pairs of their per-block partial sums, grouped by node
  ot::DevBuf mpe_a, mpe_b, mpe_pnode, mpe_pblock, mpe_poff, mpe_part;
  int64_t mpe_npairs = 0;
  ot::DevBuf abu_flag, abu_blist;  // adaptive block update: per-block flags, updated blocks
  // interaction lists
  ot::DevBuf lcount, lnodes, loff, lrec, lid, lscratch, llat;
  // lists of the last ot_solve_points call (per target point)
  ot::DevBuf pcount, pnodes, poff, prec, pid, pcheck;
  std::vector<int64_t> poff_host;
  int64_t npts = 0;
  int list_sub = 0;
  int64_t list_cap = 0;
  int64_t scratch_per_wg = 0;
  int list_grid = 0;
  bool lists_valid = false;
  std::vector<int64_t> off_host;  // list offsets of the last solve
  // APE limit from the BH pre-pass
  bool alim_valid = false;
  double alim = 0.0;
  // Ewald
  ot::DevBuf tab64, tab32;
  bool ewald_ready = false;
  int ew_n = 0, ew_rcut2 = 0, ew_fcut2 = 0;
  double ew_alpha = 0, ew_ext[3] = {0, 0, 0}, ew_step[3] = {0, 0, 0};
  double ms_build = 0.0;
  // columns
  ot::DevBuf rt_off, rt_pix, rt_w64, rt_rows, rt_ent, rt_rows8, rt_quad64, rt_lut, rt_thr, lh;
  bool rt_ready = false;
  int64_t rt_pairs = 0;
  // learned Ewald surrogate: FP32 parameters, packed FP16 operands, the
  // input / output scaling (ext[3], mu[10], sig[10]) and gradient scratch
  ot::DevBuf mlp_P, mlp_pk, mlp_part, mlp_lossp, mlp_loss;
  bool mlp_have = false, mlp_ok = false;
  double mlp_norm[OT_MLP_NNORM] = {0};
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};
