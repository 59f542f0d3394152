// Internal data structures shared by the host planner and the gfx950 kernels
// of the Chebyshev-moment library.  Not part of the public ABI (include/kpm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace kpm {

constexpr int kThreads = 256;     // threads per workgroup (4 wave64)
constexpr int kMaxBonds = 512;    // bonds per problem
constexpr int kMaxLd = 64;        // real columns per recursion block (padded)
constexpr int kBinomN = 33;       // binomial table C(n, j), n, j < 33
constexpr int kKoffLen = 34;      // popcount-class offsets of the low-word table (0..32, end)
constexpr uint32_t kNoRun = 0xFFFFFFFFu;   // per-block table entry: no target block

// One (cluster, S^z sector) problem as the kernels see it.
struct ProbDev {
  int64_t dim;        // C(n_sites, n_up)
  int32_t n_sites, n_up, n_bonds, bond_off;   // bonds at [bond_off, bond_off + n_bonds)
  int32_t B0, B1, B2, tab_off;                // rank-table split and offset (u32 entries)
  int32_t tab_len, cluster;                   // table entries; RNG cluster id
  double shift;       // -b / a   (diagonal shift of H' = (H - b)/a)
  double inv_a;       // 1 / a
  int64_t state_off;  // offset of this sector's basis words in the state table
  // Block geometry (block kernel): the low blk_L bits of a state index it
  // inside its block; bonds in class order (low-low, high-high, mixed) are
  // listed by bperm[bond_off + q].
  int32_t blk_L, n_ll, n_hh, n_mx;
  // Block-table kernel: this problem's blocks are [blk_off, blk_off + n_blk)
  // of the plan's block list (ascending h, i.e. rank order).
  int32_t blk_off, n_blk;
  // Spin-s sites (spin kernel): 2s; the rank table at tab_off is
  // P[i][r][d] = number of digit strings of sites 0..i with sum r and digit
  // < d at site i, [n_sites][2s n_sites + 1][2s + 1]; bond masks hold i | j << 8.
  int32_t two_s;
  // Block kernels: the sites are relabelled (site i of the problem is bit
  // perm[i] of the words the kernels see) so that few bonds join the low
  // bits to the high bits.  Rows are then in the rank order of the
  // relabelled words; the start vectors and exported rows use the rank of
  // the original word.
  int32_t relabel;
  uint8_t perm[32];
};

// One recursion block: a problem and a contiguous range of its real columns.
// Vector storage is slot-major: slot k of this block is [dim][ld] at
// base + k * slot_stride + vec_off (slot_stride is the same for all blocks).
struct UnitDev {
  int64_t vec_off;    // element offset of this block inside every slot
  int64_t part_off;   // offset of this unit's partial dots: [2 * ld][ntiles]
  int64_t bd_off;     // offset of this unit's bond-dot partials: [ntiles][n_bonds]
  int32_t prob, ld, ncols, col0;              // columns [col0, col0 + ncols) of the problem
  int32_t tile0, ntiles, col_off, pad;        // first tile; column offset in dot rows
};

// Arguments of the fused recursion step (one launch per step).
// Slice kernel: what a workgroup needs first, one scalar load each.
struct SliceWg {
  int32_t tile;      // plan tile (< 0: the workgroup has no tile)
  int32_t unit;      // its column block
  int32_t prob;      // the block's problem
  int32_t g0, ng;    // its low-bit blocks [g0, g0 + ng) (global block index)
  int32_t pad[3];
};
struct SliceBlk {    // written once per call with the per-block tables
  uint32_t h;        // high word
  uint32_t start;    // rank of the first member
  uint32_t size;     // members C(L, k), k = n_up - popcount(h) (0 if k is out of range)
  uint32_t kofs;     // position of popcount class k in the low-word tables
  uint32_t nh;       // acting high-high bonds
  uint32_t pad;
  double dhh;        // -b/a + high-high part of the diagonal
};

struct StepArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* tile_unit;    // [n_tiles]: unit of each tile
  const int64_t* tile_row0;    // [n_tiles]: first state of each tile
  const int32_t* tile_nrows;   // [n_tiles]: states in each tile
  const int32_t* job_unit;     // [2 * total_cols]: unit of each reduction job
  const uint32_t* tables;      // rank tables of all problems
  const uint32_t* bmask;       // per bond: (1 << i) | (1 << j)
  const double* boff;          // per bond: J_b / (2a)   (off-diagonal element of H')
  const double* bzz;           // per bond: J_b / (4a)   (diagonal contribution)
  const uint32_t* binom;       // C(n, j) [33][33]
  const uint32_t* states;      // basis words of every sector, rank order (row kernel);
                               // spin kernel: digit strings (u64) then neighbour ranks
  int64_t spin_rows;           // spin kernel: rows of all problems (u64 digit strings)
  void* vec;                   // vector storage base (float or double)
  int64_t slot_stride;         // elements between consecutive slots
  double* part_out;            // partial dots written by this step
  const double* part_in;       // partial dots of the previous step (reduced here)
  double* alpha;               // [steps + 1][total_cols]: <v_n, v_n>
  double* beta;                // [steps][total_cols]:     <v_n+1, v_n>
  const int64_t* step_base;    // device step counter base (NULL => 0)
  int32_t step_add;            // step index s = *step_base + step_add
  int32_t n_tiles;             // real tiles
  int32_t grid_tiles;          // launched tiles (multiple of 8)
  int32_t x_slot;              // slot of x = v_n (slot k of a block: + k * dim * ld)
  int32_t yin_slot;            // slot of v_{n-1} (read)
  int32_t yout_slot;           // slot receiving v_{n+1} (may equal yin_slot)
  int32_t first;               // 1: y = H' x; 0: y = 2 H' x - y
  int32_t n_jobs;              // reduction jobs of the previous step (0 = none)
  int32_t total_cols;          // row length of alpha / beta
  int32_t sub_rows;            // rows per LDS sub-tile (power of two <= 256)
  int32_t sub_per_tile;        // sub-tiles per workgroup tile
  int32_t lds_nb;              // neighbour-list capacity per row in LDS
  int32_t lds_tab;             // table capacity (u32 entries) in LDS
  int32_t lds_bonds;           // bond capacity in LDS
  int* err;                    // bit 1 set if a neighbour rank fell outside its sector
  int32_t xcd_remap;           // 1: contiguous tile ranges per XCD
  int32_t dense;               // 1: one neighbour slot per bond (bond-major gathers)
  // block kernel
  const uint16_t* bperm;       // per problem: bond indices in class order
  int32_t blk_max;             // blocks per tile (capacity)
  int32_t blk_rows;            // rows per tile (capacity, <= kThreads)
  int32_t lds_lr;              // entries of the low-word rank table (1 << max blk_L)
  int32_t lds_hh;              // high-high bond capacity
  int32_t lds_mx;              // mixed bond capacity
  int32_t ld_max;              // widest block (LDS copy of v_n)
  const int32_t* tile_sub0;    // [n_tiles + 1]: sub-tiles of tile t are [tile_sub0[t], tile_sub0[t+1])
  const int32_t* sub_nrows;    // states of each sub-tile (consecutive from tile_row0)
  const uint16_t* lrank;       // colex rank of every low word (1 << max blk_L entries)
  // block-table kernel
  const uint32_t* blk_h;       // [n_blk] high word h of each block
  const uint32_t* blk_start;   // [n_blk] rank of the block's first state in its sector
  const int32_t* sub_blk0;     // per sub-tile: first block (global block index)
  const int32_t* sub_nblk;     // per sub-tile: blocks
  const uint16_t* lunr;        // low words by (popcount, colex rank): lunr[koff[k] + i]
  const int32_t* koff;         // [kKoffLen] start of popcount class k in lunr
  const uint32_t* meta_hcnt;   // [n_blk] acting high-high bonds of the block
  const uint32_t* meta_hstart; // [n_blk][meta_hh] first rank of each target block (acting first)
  const uint16_t* meta_hq;     // [n_blk][meta_hh] its bond index inside the high-high class
  const uint32_t* meta_mstart; // [n_blk][meta_mx] per mixed bond: target block's first rank
  int32_t meta_hh, meta_mx;    // row lengths of the per-block tables (>= 1)
  int32_t lds_ll;              // low-low bond capacity per row (block-table kernel)
  // slice kernel
  const uint32_t* cmask;       // per bond in class order (bond_off + q): mask
  const double* coff;          // ... J_b / (2a)
  const double* czz;           // ... J_b / (4a)
  const double* meta_hcoef;    // [n_blk][meta_hh] J_b/(2a) of each acting high-high bond
  const double* meta_dhh;      // [n_blk] -b/a + high-high part of the diagonal
  const uint8_t* wtab;         // [n_probs][slice_words][slice_wb] word tables
  int32_t slice_wb;            // bytes per word-table row (32 or 64)
  int32_t slice_words;         // rows per problem (1 << largest blk_L)
  int32_t blk_lds_rows;        // slice kernel: LDS rows per buffer (largest block, or tile when shared)
  const SliceWg* wg_rec;       // slice kernel: per workgroup, its tile (tile < 0: idle)
  const SliceBlk* blk_rec;     // slice kernel: per block (global index), its record
  int16_t* vec_lo;             // float32 + residual storage: the residual q of every
                               // element, same element index as the float32 part
                               // (NULL for plain float32 / float64 storage)
  const double* yscale;        // slice kernel, float64 storage: per column (col_off + c) the
                               // factor of v_{n-1} in 2 H' v_n - y (NULL: 1; the FTLM's beta_j)
};

// Device-side plan of one run (pointers into the workspace) + launch shape.
struct DevicePlan {
  ProbDev* probs = nullptr;
  UnitDev* units = nullptr;
  int32_t* tile_unit = nullptr;
  int64_t* tile_row0 = nullptr;
  int32_t* tile_nrows = nullptr;
  int32_t* job_unit = nullptr;
  int32_t* prob_unit0 = nullptr;
  uint32_t* tables = nullptr;
  uint32_t* bmask = nullptr;
  double* boff = nullptr;
  double* bzz = nullptr;
  uint32_t* binom = nullptr;
  uint32_t* states = nullptr;  // basis words (row and block kernels), filled by fill_states
  uint16_t* bperm = nullptr;   // bond class order (block kernel)
  int32_t* tile_sub0 = nullptr;  // block kernel: sub-tile range of each tile
  int32_t* sub_nrows = nullptr;  // block kernel: states of each sub-tile
  uint16_t* lrank = nullptr;     // block kernel: low-word colex ranks
  uint32_t* blk_h = nullptr;     // block-table kernel: blocks (see StepArgs)
  uint32_t* blk_start = nullptr;
  int32_t* sub_blk0 = nullptr;
  int32_t* sub_nblk = nullptr;
  uint16_t* lunr = nullptr;
  int32_t* koff = nullptr;
  int* err = nullptr;          // device error word (see StepArgs::err)
  int32_t n_probs = 0, n_units = 0, n_tiles = 0, grid_tiles = 0, total_cols = 0;
  int32_t sub_rows = 256, sub_per_tile = 1, lds_nb = 0, lds_tab = 0, lds_bonds = 0;
  int32_t cpl = 1;
  int32_t fp32 = 0;
  int32_t resid = 0;           // 1: float32 + 16-bit residual storage (fp32 is set too);
                               // the residuals follow the float32 part, vec_elems int16
  int32_t xcd_remap = 1;
  int32_t dense = 0;
  int32_t row_ld = 0;          // > 0: one lane per state with all row_ld columns
  int32_t gather_batch = 4;    // neighbour rows in flight per lane (2, 4 or 8)
  int32_t block = 0;           // 1: block kernel (tiles of whole low-bit blocks),
                               // 2: block-table kernel (same tiles, per-block tables),
                               // 3: slice kernel (block-table tiles and tables, each
                               //    wave on rows of one block at a time),
  int32_t n_blk = 0;           // block-table kernel: blocks of all problems
  int32_t meta_hh = 1, meta_mx = 1;   // per-block table widths (StepArgs)
  int32_t tab_xl = 0;          // block-table kernel: sub-tile rows of v_n staged in LDS
  int32_t spin = 0;            // 1: spin-s plan (spin kernel for every step)
  int64_t spin_rows = 0;       // spin plan: rows of all problems; the state table holds
                               // the u64 digit string of every row, then per problem
                               // [lds_nb][dim] u32 neighbour ranks (slot 2b + w: bond b,
                               // w = 0 S^+_i S^-_j, w = 1 S^-_i S^+_j; written when acting)
  int32_t lds_ll = 1;          // block-table kernel: low-low bond capacity per row (<= 255)
  uint32_t* cmask = nullptr;   // bonds of every problem in class order (slice kernel)
  double* coff = nullptr;
  double* czz = nullptr;
  int32_t slice_wb = 0;        // slice kernel: word-table row bytes (0 = no slice plan)
  int32_t slice_words = 0;     // slice kernel: word-table rows per problem
  int32_t blk_lds_rows = 0;    // slice kernel: members of the largest block
  SliceWg* wg_rec = nullptr;   // slice kernel: record of each of slice_grid workgroups
  int32_t slice_grid = 0;      // slice kernel: workgroups launched (0 = grid_tiles)
  int32_t slice_nw = 1;        // slice kernel: waves per workgroup (1; 2 or 4 share a tile)
  int32_t slice_tile_rows = 0; // slice kernel: rows of the largest tile
  int32_t blk_max = 16, blk_rows = kThreads, lds_lr = 1, lds_hh = 1, lds_mx = 1, ld_max = 1;
  int64_t n_states = 0;        // entries of the state table
  int64_t part_len = 0;        // doubles per partial buffer
  int64_t slot_stride = 0;     // elements of one slot (all blocks)
  int64_t vec_elems = 0;       // elements of the two-slot storage of the recursion
  int64_t bd_len = 0;          // doubles of bond-dot partials (adjoint)
};

struct ReduceArgs {
  const UnitDev* units;
  const int32_t* job_unit;
  const double* part;
  double* dst_a;   // per column: sum of alpha-part partials (NULL: skip)
  double* dst_b;   // per column: sum of beta-part partials (NULL: skip)
  int n_jobs;
};

struct InitArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* tile_unit;
  const int64_t* tile_row0;
  const int32_t* tile_nrows;
  void* vec;                 // slot 0 is written
  int16_t* lo;               // float32 + residual storage: residual part (NULL otherwise)
  const double* norms;   // per column: Gaussian sums of squares (modes 1, 2)
  double* part_out;
  uint64_t seed;
  const uint32_t* binom;     // C(n, j) [33][33] (rank of the original word of a relabelled row)
  int32_t n_tiles, grid_tiles, mode, vec_kind;   // mode 0 sums of squares, 1 write, 2 unit-norm
};

struct FinalArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* prob_unit0;  // [n_probs + 1]: units of problem p are [u0[p], u0[p+1])
  const double* alpha;
  const double* beta;
  double* mu;
  int* flag;
  int32_t n_probs, M, total_cols, cols_per_vec, R;   // R = 0: complete basis (R_eff = dim)
};

struct MatrixArgs {
  const ProbDev* probs;
  const uint32_t* tables;
  const uint32_t* bmask;
  const double* boff;
  const double* bzz;
  const uint32_t* binom;
  int64_t row0, nrows;
  int32_t max_nb, lds_tab, lds_bonds, sub_rows, lds_nb;
  uint32_t* cols;
  int32_t* bond;
  int32_t* cnt;
  double* diag;
};

struct LzArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* tile_unit;
  const int64_t* tile_row0;
  const int32_t* tile_nrows;
  double* w;
  const double* q;
  const double* coef;      // per column (col_off + c): alpha_j
  double* part_out;
  int64_t slot_stride;
  int32_t n_tiles, grid_tiles;
  int32_t w_hi, q_hi;      // select slot 1 instead of slot 0
  double* ybeta;           // non-NULL => q_j stays in its slot and ybeta[col] gets the
                           // beta_{j+1} by which the next step scales it (0: term dropped)
};

// Per-problem metadata of the thermodynamic sums.
struct ThermoProb {
  int32_t cluster;
  int32_t weight;   // 1 for S^z = 0, 2 otherwise
  double sz;        // S^z = n_up - N/2
};

struct ThermoArgs {
  const ThermoProb* tp;
  const int32_t* cl_start;   // [n_clusters + 1] into cl_list
  const int32_t* cl_list;    // problems grouped by cluster
  const double* gamma;       // [n_probs][n_nodes]
  const double* ab;          // [n_probs][2]
  const double* T;           // [n_T]
  double* lnZ;
  double* E;
  double* C;
  double* chi;
  uint8_t* znonpos;
  double* stats;             // [n_clusters][n_T][6]: S0, Ebar, Var, <m^2>, Eref, beta
  int32_t n_nodes, n_T, n_clusters;
  const double* h;           // [n_T] Zeeman energies g mu_B B (field kernel only)
  double* mag;               // [n_clusters][n_T] <S^z> (field kernel, may be NULL)
  // hybrid kernel: problem p with ed_count[p] > 0 contributes the eigenvalues
  // evals[p * evals_ld + i], i < ed_count[p], instead of its nodes
  const int32_t* ed_count;
  const double* evals;
  int32_t evals_ld;
};

// Exact spectrum of one small sector (dense diagonalisation).
struct EigProb {
  int32_t n_sites, n_up, dim, n_bonds;
  int32_t bond_off, out_row;   // bonds in the packed arrays; row of the output
  int64_t mat_off;             // doubles from the matrix workspace base
  int32_t two_s, tab_off;      // spin s > 1/2: 2s and its rank table (EigArgs::tables)
  int64_t vec_off;             // doubles from the work-vector bases (hv, hp, hd, he)
};

constexpr int kEdRows = 4;     // rows of the trailing block per workgroup (Householder steps)

struct EigArgs {
  const EigProb* probs;        // one per workgroup
  const uint32_t* bmask;       // per bond: (1 << i) | (1 << j); spin s > 1/2: i | j << 8
  const double* J;             // per bond: J_b (unscaled H)
  const uint32_t* binom;       // C(n, j) [33][33]
  const uint32_t* tables;      // spin-s rank tables P[i][r][d] (as ProbDev)
  double* mat;                 // dense sector matrices
  double* hv;                  // per sector [max(dim, 4)]: Householder vector of the current
                               // step, then the bisection interval, pivot floor and radius
  double* hp;                  // per sector [dim]: 2 A' v
  double* hd;                  // per sector [dim]: diagonal of the tridiagonal matrix
  double* he;                  // per sector [dim]: its off-diagonal
  double* evals;               // [rows][ld] ascending eigenvalues
  int* err;                    // bit 1: rank out of range
  int32_t ld, max_dim;
  int32_t o_bonds;             // LDS byte offset of the bond J values (build kernel)
};
// probs sorted by descending dim; dims[i] = probs[i].dim on the host.
hipError_t launch_sector_eig(const EigArgs& a, const int* dims, int n_sectors, size_t lds_build,
                             size_t lds_finish, hipStream_t st);
hipError_t launch_thermo_hybrid(const ThermoArgs& a, hipStream_t st);

// Finite-temperature Lanczos: Ritz values/weights per column and the sums.
struct FtlmArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* job_unit;
  const int32_t* prob_unit0;
  const double* dots;        // [steps][total_cols] alpha_j
  const double* b2;          // [steps][total_cols] beta_j^2
  const double* norms;       // [total_cols] |start column|^2
  double* ritz;              // [total_cols][steps]
  double* escr;              // [total_cols][steps] scratch
  double* weight;            // [total_cols][steps]
  int32_t* len;              // [total_cols] Ritz values per column
  int* err;                  // bit 3: QL did not converge
  int32_t total_cols, steps, vec_kind, R;
  const ThermoProb* tp;
  const int32_t* cl_start;
  const int32_t* cl_list;
  const double* T;           // [n_pts]
  const double* h;           // [n_pts] Zeeman energies or NULL
  double* lnZ;
  double* E;
  double* C;
  double* chi;
  double* mag;               // may be NULL
  int32_t n_pts, n_clusters;
};
hipError_t launch_ftlm_ritz(const FtlmArgs& a, hipStream_t st);
hipError_t launch_ftlm_thermo(const FtlmArgs& a, hipStream_t st);

struct ThermoVjpArgs {
  const ThermoProb* tp;
  const double* ab;
  const double* stats;
  const double* wC;          // [n_clusters][n_T]
  const double* wchi;
  const double* g;           // kernel coefficients [M]
  double* node_adj;          // [n_probs][n_nodes]
  double* lambda;            // [n_probs][M]
  int32_t n_probs, M, n_nodes, n_T;
};

struct DoublingVjpArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* job_unit;
  const double* lambda;      // [n_probs][M] = dL/dmu
  const double* alpha0;      // [total_cols] = <v_0, v_0> per column
  double* abar;              // [K + 1][total_cols]
  double* bbar;              // [K + 1][total_cols] (row K stays zero)
  int32_t total_cols, M, K, cols_per_vec, R;   // R = 0: complete basis
};

// Threads per basis state in adjoint_kernel for a block of ld columns (each
// takes min(ld, kAdjCpt) of them).
constexpr int kAdjCpt = 4;
__host__ __device__ inline int adjoint_lanes(int ld) { return ld / (ld < kAdjCpt ? ld : kAdjCpt); }

struct AdjArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* tile_unit;
  const int64_t* tile_row0;
  const int32_t* tile_nrows;
  const uint32_t* tables;
  const uint32_t* bmask;
  const double* boff;
  const double* bzz;
  const uint32_t* binom;
  const void* vseg;          // slots of v (slot-major)
  void* wbuf;                // two slots of w
  int64_t slot_stride;
  int32_t vm1_slot, v0_slot, vp1_slot;   // v_{n-1}, v_n, v_{n+1} (-1: absent)
  int32_t wx_slot, wy_slot;              // w_{n+1} (gathered); w_{n+2} in, w_n out
  const double* abar_n;      // [total_cols] row n
  const double* bbar_n;      // row n
  const double* bbar_nm1;    // row n-1
  double* part_bd;           // per-tile bond dots, accumulated across launches
  double coef;               // weight of this launch's bond dots
  int32_t accumulate, dots_only;
  int32_t n_tiles, grid_tiles, sub_rows, sub_per_tile, lds_tab, lds_bonds, xcd_remap;
  int* err;
};

struct BondReduceArgs {
  const ProbDev* probs;
  const UnitDev* units;
  const int32_t* prob_unit0;
  const double* part_bd;
  double* dJ;
  int32_t n_probs;
};

size_t step_lds_bytes(const DevicePlan& p);
size_t adjoint_lds_bytes(const DevicePlan& p);
hipError_t launch_doubling_vjp(const DoublingVjpArgs& a, hipStream_t st);
hipError_t launch_adjoint(const DevicePlan& p, AdjArgs a, int ld, hipStream_t st);
hipError_t launch_bond_reduce(const BondReduceArgs& a, int total_bonds, hipStream_t st);
hipError_t launch_cluster_grad(const int32_t* info, int n, const int32_t* cinfo, int n_clusters,
                               int max_bonds, const double* dJ, double* out, hipStream_t st);
hipError_t launch_loss(const double* C, const double* chi, const double* wC, const double* wchi,
                       int n, double* L, hipStream_t st);

hipError_t launch_step(const DevicePlan& p, void* vec, double* part_out, const double* part_in,
                       int n_jobs, double* alpha, double* beta, const int64_t* step_base,
                       int step_add, int x_parity, int first, hipStream_t st);
// Same step with explicit buffer slots (x, v_{n-1} in, v_{n+1} out).
hipError_t launch_step_slots(const DevicePlan& p, void* vec, double* part_out, int x_slot,
                             int yin_slot, int yout_slot, int first, hipStream_t st);
// A step with explicit slots that also reduces the previous step's dots
// (as launch_step does in the two-slot ring).
hipError_t launch_step_slots_dots(const DevicePlan& p, void* vec, double* part_out, const double* part_in,
                                  int n_jobs, double* alpha, double* beta, int step_add, int x_slot,
                                  int yin_slot, int yout_slot, hipStream_t st);
// The two-slot step 2 H' x - s y with v_{n-1} scaled per column by yscale
// (slice plans in float64 storage only; the FTLM's beta_j q_{j-1}).
hipError_t launch_step_scaled(const DevicePlan& p, void* vec, double* part_out, int x_parity,
                              const double* yscale, hipStream_t st);
hipError_t launch_reduce(const DevicePlan& p, const double* part, double* dst_a, double* dst_b,
                         hipStream_t st);
hipError_t launch_init(const DevicePlan& p, void* vec, int mode, int vec_kind, uint64_t seed,
                       const double* norms, double* part_out, hipStream_t st);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t st);
hipError_t launch_set_i64(int64_t* dst, int64_t v, hipStream_t st);

struct ExportArgs {
  const UnitDev* units;
  const void* vec;       // vector storage base
  int64_t slot_stride;
  int32_t slot, unit0, rb, n_cols;
  int64_t dim;
  void* out;             // [dim][n_cols], storage type
  const ProbDev* prob;   // the problem (rows of relabelled sites are mapped back)
  const uint32_t* binom; // C(n, j) [33][33]
};
hipError_t launch_export(const ExportArgs& a, int fp32, hipStream_t st);
hipError_t launch_states(int N, int k, const uint32_t* binom, uint32_t* out, int64_t dim,
                         hipStream_t st);
// Basis words of every sector of the plan into p.states.
hipError_t fill_states(const DevicePlan& p, hipStream_t st);
size_t row_lds_bytes(const DevicePlan& p);
size_t block_lds_bytes(const DevicePlan& p);
size_t spin_lds_bytes(const DevicePlan& p);
size_t tab_lds_bytes(const DevicePlan& p);
size_t slice_lds_bytes(const DevicePlan& p);
int slice_word_bytes(int n_mx, int n_ll);   // 32, 64, or 0 when a word row cannot hold the bonds
hipError_t build_slice_words(const DevicePlan& p, uint8_t* wtab, hipStream_t st);
hipError_t launch_slice(const DevicePlan& p, const StepArgs& a, hipStream_t st);
// Bytes of the per-block tables of the block-table kernel (kept in the state
// table region; built by fill_states).
size_t tab_meta_bytes(const DevicePlan& p);
hipError_t launch_matrix(const MatrixArgs& a, size_t lds, int grid, hipStream_t st);
// Lanczos turn (bounds and FTLM): fused w -= alpha q_j and turn for well-conditioned columns (ww = <w, w>),
// then the exact finish of the others (fixed = their |w - alpha q_j|^2) and
// beta_{j+1}^2 of every column.  ybeta NULL: slot x receives beta_{j+1} q_j;
// else q_j stays and ybeta[col] receives beta_{j+1} for launch_step_scaled.
hipError_t launch_lz_fused(const DevicePlan& p, double* vec, int y_hi, const double* alpha, const double* ww,
                           double* part_out, double* ybeta, hipStream_t st);
hipError_t launch_lz_fix(const DevicePlan& p, double* vec, int y_hi, const double* alpha, const double* ww,
                         const double* fixed, double* beta2, double* ybeta, hipStream_t st);
hipError_t launch_kernel_coef(int M, int kernel, double* g, hipStream_t st);
hipError_t launch_gamma(int n_probs, int M, int n_nodes, const double* g, const double* mu,
                        double* gamma, hipStream_t st);
hipError_t launch_thermo(const ThermoArgs& a, hipStream_t st);
hipError_t launch_thermo_field(const ThermoArgs& a, hipStream_t st);
hipError_t launch_thermo_vjp(const ThermoVjpArgs& a, hipStream_t st);

}  // namespace kpm
