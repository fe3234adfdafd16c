// Host-side ordering and symbolic analysis for the supernodal factor.
//
// Nested dissection gives a fill-reducing symmetric permutation Pi (section
// 5.1 applies Pi to A once).  Every nested-dissection tree node (a leaf box of
// the grid or graph, or a separator) becomes one supernode whose columns are
// contiguous in the new order.  Its front has rows = its own columns followed
// by struct(s): the later nodes adjacent to its subtree.  Diagonal blocks and
// the rectangular blocks below them are held dense.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace lobpcg {

constexpr int kTile = 64;   // tile edge of the factor kernels
constexpr int kSolveItemInts = 12;   // ints per triangular-solve item
constexpr int kSolveWideK = 256;     // items with longer reduction ranges use four waves
// Tile items aimed at per level of the triangular-solve plan by default: levels with fewer output tiles
// split their reduction ranges until they have about this many (the autotuner may choose another).
// Items of an FP64 factor stream twice the bytes, so they are split further.
constexpr int default_split_target(int elem_bytes) { return elem_bytes == 4 ? 256 : 1024; }
// Leading dimension of a supernode panel with nr rows: nr rounded up to a multiple of 4, so that
// every panel column starts 16-byte aligned (FP32) and 4-row groups can be read as one vector.
constexpr int64_t panel_ld(int64_t nr) { return (nr + 3) & ~(int64_t)3; }

struct Symbolic {
  int64_t n = 0;
  std::vector<int32_t> perm;   // perm[new] = old
  std::vector<int32_t> iperm;  // iperm[old] = new
  int32_t nsuper = 0;
  std::vector<int32_t> begin, nc, nr, parent, level;  // per supernode
  std::vector<int64_t> row_off;                       // per supernode, into rows
  std::vector<int32_t> rows;                          // new indices; first nc are own columns
  std::vector<int32_t> relpos;                        // parallel to rows: for below rows, position in parent's rows
  int32_t nlevels = 0;
  std::vector<int32_t> level_ptr, level_sn;           // supernodes grouped by level (bottom-up)
  std::vector<int32_t> child_ptr, child_list;
  // inverse maps: for child c (indexed by c), inv_off[c] -> nr[parent(c)] entries:
  // -1 or the index j of the child's below row (0..nb_c-1) at that parent row.
  std::vector<int64_t> inv_off;
  std::vector<int32_t> invmap;
  // storage plans
  std::vector<int64_t> panel_off; int64_t panel_total = 0;   // panel_ld(nr)*nc each (col-major)
  std::vector<int64_t> upd_off;   int64_t upd_total = 0;     // nb*nb each (col-major, ld = nb)
  std::vector<int64_t> uvec_off;  int64_t uvec_total = 0;    // nb rows each (trisolve update vectors)
  std::vector<int64_t> dinv_off;  int64_t dinv_total = 0;    // 2*np*kTile*kTile each: inv(L_pp), then L_pp
  std::vector<int64_t> lcopy_off; int64_t lcopy_max = 0;     // 2*nc*nc + nb*nc within the level scratch
  double nnz_lower = 0;    // sum over supernodes of nc(nc+1)/2 + nb*nc
  double flops = 0;        // numeric factorization flops (Cholesky part)
  int32_t max_nr = 0, max_nc = 0;
  int nb(int s) const { return nr[s] - nc[s]; }
};

// Leaf volume of the nested dissection when the caller leaves it open (leaf_size < 1): 256 for a 3D
// grid (every dimension above 1), where a deeper tree costs more supernodal levels, and so more
// dependent launches per triangular solve, than the extra fill of larger leaves; 64 otherwise.
inline int default_leaf(const int32_t* grid) {
  return (grid && grid[0] > 1 && grid[1] > 1 && grid[2] > 1) ? 256 : 64;
}

// Build the ordering and supernode partition.  grid: structured-grid hint
// (all > 0) or zeros; dense = true gives one supernode with natural order; leaf_size < 1: default_leaf
// per component.  Returns an empty string on success, else a message.
std::string analyze(int64_t n, const int32_t* rowptr, const int32_t* colind, const int32_t grid[3],
                    bool dense, int leaf_size, Symbolic& out);

// Several independent problems stored as one block-diagonal matrix: component c owns
// the index range [off, off + n) and is ordered on its own (its own grid hint), so each
// component's new indices stay in its range and the supernodal tree is a forest.
struct Component { int64_t off; int64_t n; int32_t grid[3]; };
std::string analyze_multi(int64_t n, const int32_t* rowptr, const int32_t* colind, const std::vector<Component>& comps,
                          bool dense, int leaf_size, Symbolic& out);

// Permuted CSR pattern: for new row i, entries sorted by new column; map[e'] = old entry index.
void permute_pattern(const Symbolic& S, const int32_t* rowptr, const int32_t* colind,
                     std::vector<int32_t>& prow, std::vector<int32_t>& pcol, std::vector<int32_t>& map);

// For each entry e' of the permuted CSR (row j = column j by symmetry), the front row
// of column j's supernode holding A(i, j) when i >= j, else -1.
void assembly_positions(const Symbolic& S, const std::vector<int32_t>& prow,
                        const std::vector<int32_t>& pcol, std::vector<int32_t>& apos);

// Entries of the exact Cholesky factor (diagonal included) of the permuted pattern: what an
// elimination without the supernodes' explicit zeros would store.  O(nnz(L)) host work.
int64_t exact_fill(int64_t n, const std::vector<int32_t>& prow, const std::vector<int32_t>& pcol);

// Factorization task lists: tasks are int4 {s, I, J, p}; steps[] holds (offset, count, kind, level).
struct FactorPlan {
  std::vector<int32_t> tasks;        // 4 ints per task
  struct Step { int64_t off; int32_t count; int32_t kind; int32_t level; };
  std::vector<Step> steps;           // in execution order
  std::vector<int32_t> asm_items;    // 2 ints (s, t) per assembly work item, grouped per level
  std::vector<int64_t> asm_level_off;  // nlevels+1
  std::vector<int32_t> level_max_nr;   // per level: the largest front (rows) of the level
  int schur_wide_tiles = 8;            // fronts with at least this many tile rows below the panel use kSchur2
};
// kPotrf: update of column p by panel p - 1, then the Cholesky factor of diagonal tile p with the trsm
// of the tiles below it (kTrsm: the trsm alone); kUpdate: the move of L_pp into the panel and the
// trailing update of the panel columns after p + 1 (they may run while panel p + 1 is factored);
// kUpdateRest: no longer planned; kSchur: U_s -= L21 L21^T after the last panel step.
// kInvPrep / kInvT1 / kInvX21 / kInvP21: the inverse phase P_s = [inv(L11); L21 inv(L11)] (kInvScale and
// kInvUpdate: the column sweep it replaces, no longer planned).
enum StepKind { kAssemble = 0, kPotrf = 1, kTrsm = 2, kUpdate = 3, kInvPrep = 4, kInvScale = 5, kInvUpdate = 6,
                kSchur = 7, kInvT1 = 8, kInvX21 = 9, kInvP21 = 10, kUpdateRest = 11, kSchur2 = 12 };
// kSchur2: the Schur complement of fronts with at least schur_wide_tiles tile rows below the panel, on
// 128 x 128 blocks (task (s, I, J) with I - np and J - np even: tiles I, I + 1 by J, J + 1)
constexpr int kSchurWideTiles = 8;
void build_factor_plan(const Symbolic& S, FactorPlan& plan, int schur_wide_tiles = kSchurWideTiles);

// Trisolve work lists.  Each output tile (64 rows of P_s for the forward sweep, 64
// own columns for the backward sweep) is one item, or, on levels with fewer tiles
// than split_target, its reduction range is split into chunks (multiples of 16 rows)
// so that the level has about split_target items; a tile with one chunk is written
// directly, otherwise each chunk writes a partial tile to its own slot and a
// finalize item sums the slots in order.
struct SolvePlan {
  int rows_per_tile = 64;
  int split_target = 1024;   // tile items aimed at per level when splitting reduction ranges
  // forward gather, per level, one item per row of a supernode with children that receives
  // contributions (own rows) or passes them on (all below rows): gather_dst = right-hand-side
  // row (>= 0) or -(update-vector row) - 1; sources gather_src[gather_ptr[i] .. gather_ptr[i+1])
  // are update-vector rows of the children
  std::vector<int32_t> gather_dst, gather_ptr, gather_src; std::vector<int64_t> gather_level_off;
  // items: kSolveItemInts ints each: s, tile, k0, k1, slot, begin, nr, nc, panel offset (low,
  // high 32 bits), update-vector offset (forward) or source-row list offset (backward), flags
  // (bit 0: s has children)
  std::vector<int32_t> fwd_items;  std::vector<int64_t> fwd_level_off;
  std::vector<char> fwd_wide, bwd_wide;   // per level: items long enough to split over four waves
  std::vector<int32_t> fwd_fin;    std::vector<int64_t> fwd_fin_level_off; // 4 ints: s, tile, slot0, nchunks
  std::vector<int32_t> bwd_items;  std::vector<int64_t> bwd_level_off;
  std::vector<int32_t> bwd_fin;    std::vector<int64_t> bwd_fin_level_off;
  int64_t fwd_slots = 0, bwd_slots = 0;
  // backward operand source rows: supernode s owns panel_ld(nr) entries from bwd_src_off[s] (a
  // multiple of 4, the backward items' aux field); entry k < nc is begin + k (a row of y), entry
  // nc <= k < nr is n + rows[row_off + k] (a row of x, stored after y), the padding is 0
  std::vector<int32_t> bwd_src; std::vector<int64_t> bwd_src_off;
  // Bottom levels 0 .. sub_levels - 1 as whole subtrees: a subtree is a supernode of level <
  // sub_levels whose parent is above (or absent) together with all its descendants, and one
  // workgroup runs it level by level (no launch per level).  For subtree q and local level l,
  // entries [sub_*_off[q * sub_levels + l], sub_*_off[q * sub_levels + l + 1]) of the lists below
  // are its gather rows (same encoding as gather_*, sources in sub_gather_src) and its unsplit
  // tile items (kSolveItemInts ints each, slot -1).  The per-level lists of these levels are kept
  // but not launched.
  int sub_levels = 0;
  int64_t nsub = 0;
  std::vector<int32_t> sub_gather_dst, sub_gather_ptr, sub_gather_src; std::vector<int64_t> sub_gather_off;
  std::vector<int32_t> sub_fwd_items; std::vector<int64_t> sub_fwd_off;
  std::vector<int32_t> sub_bwd_items; std::vector<int64_t> sub_bwd_off;
};
// sub_levels < 0: chosen from the tree (the deepest bottom cut that still has enough subtrees to
// occupy the chip, or the whole tree when it is small); otherwise as given (0: no subtree pass).
void build_solve_plan(const Symbolic& S, int rows_per_tile, int split_target, SolvePlan& plan, int sub_levels = -1);

// Check every index the GPU kernels dereference against the buffer it indexes
// (rows, maps, offsets, task and item lists, assembly positions).  Returns an
// empty string when all are in range, else the first violation.
// The solve-plan part of verify().
std::string verify_solve_plan(const Symbolic& S, const SolvePlan& P);
std::string verify(const Symbolic& S, const FactorPlan& F, const SolvePlan& P, const std::vector<int32_t>& prow,
                   const std::vector<int32_t>& apos);

}  // namespace lobpcg
