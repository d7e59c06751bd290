// Host-side plan: nested-dissection symbolic analysis of the 3^d stencil
// graph on the n^d grid, and the FFT factorisation of L = 2n.
#pragma once

#include <vector>
#include <cstdint>
#include "lsp_common.h"

namespace lsp {

// Blocked sweeps: rows of a super-block of pivots, and boundary columns per
// partial sum of the backward sweep's boundary product.
constexpr int kSweepRows = 256;
constexpr int kSweepCols = 512;

// One front (supernode) of the multifrontal factorisation.  Its index list
// is [I | B]: I = the variables it eliminates (a separator plane, or a whole
// leaf box), B = the halo of its box that lies on ancestor separators.
// Front matrices are dense, column-major, order p + q.
struct FrontDev {
  int p, q;               // fully-summed (pivot) and boundary counts
  int child0, child1;     // front ids of the children, -1 if absent
  long long idx_off;      // offset into the concatenated index lists (p+q ints)
  long long f_off;        // offset of the front matrix, in complex elements
  long long piv_off;      // offset of its p pivot / permutation entries
  long long dinv_off;     // offset of its inverted diagonal panel blocks
  int level, pad;
  // the children's idx_off, f_off and order (p + q), so kernels need no
  // dependent load of the child's descriptor; -1 / 0 if absent
  long long cidx[2];
  long long cfoff[2];
  int cm[2];
  long long g_off;        // offset of its formed sweep operators (dense
                          // levels, see Plan::level_dense; blocked levels,
                          // see Plan::level_blocked), -1 elsewhere
};

struct Plan {
  int n = 0, d = 0, N = 0, L = 0, max_nrhs = 1;
  lsp_options opts{};
  std::vector<FrontDev> fronts;   // sorted by level (leaves first)
  std::vector<int> idx;           // concatenated [I | B] lists, grid linear indices
  std::vector<unsigned> gpos;     // grid coordinates of each idx entry, packed
                                  // (gpos_shift(d) bits per axis, axis 0 lowest)
  std::vector<int> cpos;          // per front position: 2 ints, position of the
                                  // same grid point in child 0 / child 1 front, or -1
  std::vector<int> level_ptr;     // fronts of level l are [level_ptr[l], level_ptr[l+1])
  std::vector<int> level_maxp, level_maxpq;
  std::vector<int> level_tile;    // trailing-update tile (32, 64 or 128) per level
  // Levels whose sweeps apply formed dense operators instead of the panel
  // chain: per front the forward operator Gf (m x p, column-major) at g_off
  // and the backward operator Gb (p x m) stored by rows (Gb^T, m x p,
  // column-major) after it, 2 m p entries.
  std::vector<char> level_dense;
  long long dense_elems = 0;      // sum over dense fronts of 2 m p
  double dense_entries = 0.0;     // sum over dense fronts of m p (one sweep's reads)
  int dense_levels = 0;
  // Levels swept by the small-front kernels (not dense; at most two panels,
  // at most 160 rows, at most 128 rows below each front's first panel).
  std::vector<char> level_small_sweep;
  // Small-front levels swept by panel chains on the matrix cores (16
  // right-hand sides per wave, straight from the factor; nothing formed):
  // more than 16 fronts of at most 64 pivots and 256 rows, in plans for
  // blocks of right-hand sides (max_nrhs >= 4), or always with
  // dense_sweeps = 2.
  std::vector<char> level_mchain;
  int mchain_levels = 0;
  double mchain_entries = 0.0;     // factor entries one sweep of them reads
  // their fronts' vector rows: pivots (sum p), front rows (sum p + q), and
  // the children's update rows their forward sweeps add in (sum of q)
  double mchain_pivots = 0.0, mchain_rows = 0.0, mchain_child_rows = 0.0;
  // Levels swept by the blocked kernels (sweep.hip): not dense, not small,
  // and either fronts of more than 1024 rows or at most 32 fronts with more
  // than two panels.
  std::vector<char> level_blocked;
  int blocked_levels = 0;
  double blocked_entries = 0.0;   // formed super-block operator entries one
                                  // sweep reads (sum over fronts of nsb SB^2)
  long long bsweep_ystride = 0;   // per right-hand side: max over blocked
                                  // levels of fronts x max(SB, largest p)
  int bsweep_chunks = 0;          // max over blocked levels of boundary column chunks
  double assemble_entries = 0.0;  // front entries the assembly writes plus the
                                  // children's update-matrix entries it reads
  double chain_entries = 0.0;     // factor entries one sweep reads on the panel-chain
                                  // levels (neither dense nor blocked)
  double blocked_panel_entries = 0.0;  // factor entries one sweep's products read on the
                                       // blocked levels (outside the super-blocks' diagonal blocks)
  int nlevels = 0;
  long long front_elems = 0;      // sum (p+q)^2
  long long dinv_elems = 0;       // sum over panels of 2 nb^2
  int nb = 32;                    // frontal panel width
  long long sum_p = 0, sum_pq = 0;
  int max_front = 0, max_p = 0;
  double flops = 0.0, factor_entries = 0.0, sweep_entries = 0.0, update_flops = 0.0;
  double panel_blocks = 0.0;  // sum over fronts of ceil(p / nb)
  std::vector<int> radices;       // FFT radices for L, in pass order
  // General domain (Section 4): the support Omega of m as a mask over the
  // grid.  ptab per grid point: -1 interior (the whole 3^d block in Omega),
  // -2 outside Omega, else the point's row among the boundary points bpts
  // (increasing linear index), whose neighbours in Omega are the set bits q
  // = sum_a (s_a + 1) 3^a of bslots.  sketch_r: columns of the sketch R.
  // Points outside Omega keep their place in the dissection as identity rows.
  bool general = false;
  std::vector<int> ptab;
  std::vector<int> bpts;
  std::vector<unsigned> bslots;
  int sketch_r = 0;
  long long domain_points = 0;
};

// Bits per axis of a packed grid position: 16 in 2D (n <= 4096), 10 in 3D
// (N <= 2^28, so n <= 645).
inline int gpos_shift(int d) { return d == 2 ? 16 : 10; }

// Builds the plan; throws lsp::Error on invalid input.
void build_plan(Plan& plan, int n, int d, int max_nrhs, const lsp_options& opts);
// Classifies the points of a general domain (mask: n^d bytes, nonzero =
// in Omega) into plan.ptab / bpts / bslots; r = sketch columns.
void build_general(Plan& plan, const unsigned char* mask, int r);

}  // namespace lsp
