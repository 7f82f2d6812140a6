// Internal host-side structures of the diffpd library (not part of the ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/diffpd.h"

namespace dpd {

// Dimensionless trilinear shape-function gradients dN_a/dxi_j at the 2x2x2
// Gauss points (xi = +-1/sqrt(3)); q = qx + 2qy + 4qz, a = ax + 2ay + 4az.
// Physical gradients are these times 2/dx.
void reference_gradients(double Bxi[8][3][8]);

// Mesh on the host (voxels or tetrahedra): public node numbering,
// connectivity, mass, the Dirichlet and contact sets.
struct HostMesh {
  int64_t n_nodes = 0, n_elems = 0, n_free = 0;
  std::vector<int32_t> node_ijk;     // [N][3]
  std::vector<int32_t> conn;         // [E][8] public node ids
  std::vector<double> mass;          // [N]
  std::vector<double> youngs;        // [E]
  std::vector<uint8_t> fixed;        // [N]
  std::vector<int32_t> free_index;   // [N] -> index among free nodes, or -1
  std::vector<int32_t> free_nodes;   // [n_free] public ids
  std::vector<int32_t> contact;      // public ids of contact candidates
  std::vector<uint8_t> is_contact;   // [N]
  std::vector<double> X;             // [3][N] rest positions
  // node -> incident (element, local corner) pairs, 8e + a, -1 padded: [8][N]
  std::vector<int32_t> node_inc;
  int32_t grid_min[3] = {0, 0, 0}, grid_max[3] = {0, 0, 0};
  // element kind: 8 (trilinear voxels, 8 Gauss points) or 4 (linear
  // tetrahedra, one constant deformation gradient); for tetrahedra conn is
  // [E][4], node_ijk is empty and these hold the element geometry and a
  // compressed node -> (element, corner) incidence
  int32_t corners = 8;
  std::vector<double> dminv;         // [E][9] D_m^{-1} row-major (tetrahedra)
  std::vector<double> vol;           // [E] element volumes (tetrahedra)
  std::vector<int32_t> inc_ptr, inc; // [N + 1], [4E]: entries 4e + a in (e, a) order
};

// Sparse symmetric matrix over free nodes in free-index order, full pattern
// (both triangles), CSR with sorted columns.
struct Csr {
  int32_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

std::string build_mesh(const int32_t* cells, int64_t n_cells, const double* youngs,
                       const int32_t* fixed_ijk, int64_t n_fixed, const dpd_options& o,
                       HostMesh& m);
void assemble_As(const HostMesh& m, const dpd_options& o, Csr& A);
// Linear tetrahedra: positions X [N][3] (host), corners tets [E][4], moduli
// [E], fixed node ids; the corotated term, gravity and the ground penalty only.
std::string build_tet_mesh(const double* X, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                           const double* youngs, const int32_t* fixed_nodes, int64_t n_fixed, const dpd_options& o,
                           HostMesh& m);

// Supernode of the nested-dissection factor.  Its panel is an ld x ncols
// column-major block, ld = ncols + nrows: rows [0, ncols) hold the inverse of
// the diagonal Cholesky block (lower triangular), rows [ncols, ld) hold
// W = L_{R,s} L_ss^{-1} for the rows R_s below the block.
struct Supernode {
  int32_t col0 = 0, ncols = 0, nrows = 0, parent = -1, level = 0;
  int64_t rows_off = 0;   // into Symbolic::rows
  int64_t panel_off = 0;  // into the panel array (elements)
  int64_t u_off = 0;      // into the forward-update buffer (positions)
};

struct Symbolic {
  int32_t n = 0;                       // free nodes
  std::vector<int32_t> perm;           // internal -> free index
  std::vector<int32_t> iperm;          // free index -> internal
  std::vector<Supernode> sn;
  std::vector<int32_t> rows;           // concatenated R_s (internal indices, ascending)
  std::vector<int32_t> snode_of;       // internal column -> supernode
  std::vector<std::vector<int32_t>> children;
  int32_t n_levels = 0;
  std::vector<int32_t> cptr, cidx;     // forward-update contributions per internal row
  int64_t panel_size = 0, u_size = 0, packed_nnz = 0;
};

// Task of a triangular-sweep level: supernode s, first row/column, count, and
// a copy of the supernode's fields so a kernel reads them in one load.
struct SweepTask {
  int32_t sn, first, count, col0;
  int32_t ncols, nrows, pad0, pad1;
  int64_t panel_off, rows_off, u_off, pad2;
};

constexpr int kBlock = 256;          // threads per workgroup of every kernel
constexpr int kColsPerTask = 64;     // most backward-sweep columns per workgroup

// Lanes that share one panel row (wide forward sweep) or column (backward
// sweep), from the level's widest row or longest column: every lane then
// reads at least about eight panel entries.
inline int sweep_lanes(int extent) { return extent >= 512 ? 64 : (extent >= 256 ? 32 : 16); }
// Lanes of a wide forward task and of a backward column task: one pass of
// their 16 waves covers the task's rows (columns).
constexpr int kWideTaskThreads = 1024;

// Level schedule of the sweeps: supernodes of equal tree level are
// independent.  Levels whose blocks have more than 64 columns use the
// wave-per-row forward kernel; task sizes shrink on levels with little work
// so that every level offers many workgroups.
struct LevelPlan {
  std::vector<int32_t> fwd_off, bwd_off;   // task ranges per level (size L + 1)
  std::vector<int32_t> fwd_cols, bwd_rows; // dynamic LDS extents per level
  std::vector<uint8_t> fwd_wide;           // 1: wave-per-row forward kernel (row-major panel)
  std::vector<uint8_t> bwd_narrow;         // 1: one task per supernode, lanes over columns
  // levels whose supernodes span many tasks gather their right-hand sides once
  // in a separate pass: the internal columns of those supernodes per level
  std::vector<int32_t> gather_off;         // size L + 1 (empty range: gather inside the tasks)
  std::vector<int32_t> gather_cols;
  std::vector<SweepTask> fwd, bwd;
  // algorithmic traffic of one launch per level: panel entries read (packed
  // lower triangle of the diagonal block plus the off-diagonal block) and the
  // right-hand-side, update and solution vectors read and written once
  std::vector<double> fwd_bytes, bwd_bytes, fwd_flops, bwd_flops;
};

// Single-launch solve: both sweeps as one queue of entries that persistent
// workgroups of 1024 lanes claim in queue order.  An entry runs one level
// task above with the level kernel's arithmetic (on the whole workgroup), or
// up to sixteen pre-gathered columns of one supernode (a wave each).  Queue
// order is forward levels ascending (a level's gathers before its row
// tasks), then backward levels descending, so every entry depends only on
// entries before it.  An entry waits, for the supernode s it serves, for
//   forward row task:  every child of s finished its forward rows, and s's
//                      gathers done;
//   forward gather:    every child of s finished its forward rows;
//   backward task:     every backward task of s's parent done (s a root: every
//                      forward row task of s done).
// A supernode's forward rows are finished when all of its forward row tasks
// are (they only start once its children's have), which the last of them
// reports to the parent's child counter.
enum DagKind : int32_t { kDagFwdNarrow = 0, kDagFwdWide = 1, kDagGather = 2, kDagBwdCols = 3, kDagBwdNarrow = 4 };
constexpr int kDagSub = 4;          // supernode slots of an entry (one is used)
constexpr int kDagNarrowCols = 64;  // widest block of a narrow forward level
constexpr int kDagGatherCols = 16;  // gathered columns per entry
constexpr int kDagThreads = 1024;
struct DagEntry {
  int32_t kind;     // DagKind
  int32_t n;        // 1 level task, or gathered columns (<= kDagGatherCols)
  int32_t first;    // first level task (forward or backward task array) or first gather_cols index
  int32_t lpr;      // lanes per panel row (wide forward) or column (backward columns)
  int32_t flags;    // bit 0: right-hand sides pre-gathered; bit 1: backward vector staged in LDS
  int32_t sn[kDagSub];   // supernode of each level task (gather: sn[0])
  int32_t pad[7];
};
static_assert(sizeof(DagEntry) == 64, "one entry per 64-byte line");
struct DagSn {
  int32_t parent;   // -1: a root
  int32_t nch;      // children
  int32_t ntf;      // forward row tasks
  int32_t ngt;      // gather entries
  int32_t ntb;      // backward tasks
  int32_t pad[3];
};
// Counter words of the single-launch solve: queue ticket, exited workgroups,
// abort flag, launches that aborted (kept across launches), then per
// supernode: children finished, forward row tasks done, gather entries done,
// backward tasks done.  The last workgroup to leave a launch zeroes all but
// the abort count.
constexpr int kDagTicket = 0, kDagExit = 1, kDagAbort = 2, kDagAborts = 3, kDagHeader = 64;
struct DagPlan {
  std::vector<DagEntry> q;
  std::vector<DagSn> sn;
  int32_t n_fwd = 0;        // entries of the forward sweep (they come first)
  int64_t lds_bytes = 0;    // dynamic LDS of the launch: the largest entry's need
  int32_t bwd_region = 0;   // doubles of LDS of a narrow backward entry
  bool usable = false;      // every entry's LDS fits the budget (else the level launches are used)
  int64_t counter_words() const { return kDagHeader + 4 * (int64_t)sn.size(); }
};
// LDS extents (doubles) of the level task kinds, shared by the level kernels'
// launchers and the single-launch plan.
constexpr int64_t lds_fwd_narrow(int cols) { return 3 * (int64_t)cols + 4 * 64 * 3; }
constexpr int64_t lds_bwd_narrow(int rows) { return 3 * (int64_t)rows + 1024 * 3; }
void build_dag(const Symbolic& S, const LevelPlan& P, int64_t lds_budget_bytes, DagPlan& D);

// Geometric nested dissection of the free nodes on the voxel grid, then the
// supernodal symbolic analysis (row structures, tree, levels, contributions).
void analyse(const HostMesh& m, const Csr& A, int32_t leaf_max, int32_t sep_max, Symbolic& S);

// Multifrontal numeric Cholesky of A (permuted to internal order) and the
// panel construction.  Returns false (with message) on a non-positive pivot.
bool factor_panels(const Symbolic& S, const Csr& A, std::vector<double>& panels, std::string& err);

void build_plan(const Symbolic& S, LevelPlan& P);

// Multifrontal factorization on the device.  Every supernode s owns a dense
// front F_s (ld x ld, column-major, lower triangle used; ld = ncols + nrows)
// in one workspace: the entries of A in its columns, plus the Schur
// complements of its children (extend-add).  Levels run in ascending order
// (children first); within a level all fronts advance together, one block
// column of kFactorNB at a time, right-looking:
//   panel op:  Cholesky of the diagonal block, the rows below it solved
//              against it (L_{below,k}), and block row k of the panel
//              X = M^{-1}[I; 0] solved (M = [L11 0; L21 I]);
//   update op: trailing lower triangle F_{>k,>k} -= L_{>k,k} L_{>k,k}^T and
//              X_{>k,<=k} -= L_{>k,k} X_{k,<=k} (FP64 MFMA tiles of 64 x 64).
// After the last block column X holds [inv(L11); -L21 inv(L11)], the panel
// of the sweeps, and F_s's trailing block the update for the parent.
constexpr int kFactorNB = 32;     // block-column width
constexpr int kFactorTile = 64;   // output tile of the update op
constexpr int kFactorTransposeChunk = 1024;
struct FrontDesc {
  int64_t front_off;   // into the front workspace (doubles)
  int64_t panel_off;   // into the panel array
  int64_t rows_off;    // into Symbolic::rows (and the parent-position map)
  int32_t ld, nc, nrows, parent, col0, pad;
};
static_assert(sizeof(FrontDesc) == 48, "device layout");
enum FactorOpKind : int32_t { kFactorExtend = 0, kFactorPanel = 1, kFactorUpdate = 2, kFactorTranspose = 3 };
// One launch: n items (supernodes; for extend-add the children of the level's
// fronts with a given sibling rank) at ints[list_off ...], then their
// workgroup prefix sums (n + 1 entries, the last = blocks), then each
// workgroup's item index (blocks entries).
struct FactorOp {
  int32_t kind, k0, n, list_off, blocks, level;
};
struct FactorPlan {
  std::vector<FrontDesc> fronts;       // per supernode
  int64_t front_size = 0;              // doubles of the workspace
  std::vector<int64_t> a_dst;          // lower entries of A: position in the fronts
  std::vector<int32_t> a_src;          //   and index into Csr::val
  std::vector<int32_t> relmap;         // per Symbolic::rows entry: its position in the parent's front
  std::vector<int32_t> ints;           // item lists and prefix sums of the ops
  std::vector<FactorOp> ops;           // in launch order
  FactorOp transpose{};                // the row-major panel copy: every supernode,
                                       // kFactorTransposeChunk panel entries per workgroup
  double flops = 0.0;                  // of the dense work (Cholesky, updates, panel)
};
// Builds the plan and checks every index it holds against its buffer; returns
// an error message if one is out of range (nothing is launched then).
std::string build_factor_plan(const Symbolic& S, const Csr& A, FactorPlan& P);

// Row-major copy of every panel (same offsets): element (r, c) of supernode s
// at panel_off + r * ncols + c.
template <typename T>
std::vector<T> transpose_panels(const Symbolic& S, const std::vector<double>& panels) {
  std::vector<T> out(panels.size());
  for (const Supernode& sn : S.sn) {
    const int64_t ld = sn.ncols + sn.nrows;
    for (int64_t c = 0; c < sn.ncols; ++c)
      for (int64_t r = 0; r < ld; ++r)
        out[sn.panel_off + r * sn.ncols + c] = (T)panels[sn.panel_off + c * ld + r];
  }
  return out;
}

// Two-stage mesh creation (api.hip), used by dpd_create_mesh and the server.
dpd_status create_host(const int32_t* cells_ijk, int64_t n_cells, const double* youngs,
                       const int32_t* fixed_ijk, int64_t n_fixed, const dpd_options* opt,
                       dpd_mesh** out);
dpd_status create_tet_host(const double* X, int64_t n_nodes, const int32_t* tets, int64_t n_tets,
                           const double* youngs, const int32_t* fixed_nodes, int64_t n_fixed, const dpd_options* opt,
                           dpd_mesh** out);
void plan_host(dpd_mesh* m);
int64_t footprint_bytes(const dpd_mesh* m);
dpd_status upload_device(dpd_mesh* m);
void destroy_synced(dpd_mesh* m);

}  // namespace dpd
