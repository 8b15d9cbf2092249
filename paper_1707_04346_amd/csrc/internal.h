// internal.h -- shared declarations of the cisigma library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cisigma.h"

namespace cis {

constexpr int kMaxGas = 16;

// GAS description passed by value to table kernels.
struct GasDesc {
    int n;                        // orbitals
    int ngas;
    uint32_t mask[kMaxGas];       // orbital mask of each space
    int first[kMaxGas];           // first orbital of each space
    uint64_t keymul[kMaxGas];     // type key = sum_g occ_g * keymul[g]
};

// Per-spin string tables.  Strings are grouped by occupation type (types in
// lexicographic order of their per-space counts), ascending bitmask inside a
// type.
struct SpinTables {
    int nel = 0;
    int ntype = 0;
    std::vector<int> tocc;        // ntype x ngas
    std::vector<int> tcount;      // strings per type
    std::vector<int> tstart;      // ntype + 1
    std::vector<int> tirrep;      // irrep of each type (0 without spatial symmetry)
    // GAS-level types (occupation tuples) and the raw numbering of their strings:
    // the strings of GAS type g, in ascending bitmask order, are raw indices
    // graw[g] .. graw[g+1]-1.  Without spatial symmetry the types are the GAS
    // types and the raw index is the string index; with it a type is (GAS type,
    // irrep) and remap[raw] is the string index (-1: the string is in no type).
    int ngtype = 0;
    std::vector<int> gtocc;       // ngtype x ngas
    std::vector<uint64_t> gkey;   // sorted GAS type keys
    std::vector<int> graw;        // ngtype + 1
    std::vector<int> remap;       // [graw[ngtype]] (spatial symmetry only)
    int nstr = 0;
    int nexc = 0;                 // single excitations per string: nel*(n-nel)
    // pair (two-electron same-spin) lists over (nel-2)-electron strings K
    int nK = 0;                   // number of K strings
    int npv = 0;                  // pairs disjoint from K: C(n-nel+2, 2)
    // device
    uint32_t *d_str = nullptr;    // [nstr] bitmasks
    int *d_stype = nullptr;       // [nstr] type of each string
    uint32_t *d_exc = nullptr;    // [nstr][nexc] packed single excitations
    uint32_t *d_pairs = nullptr;  // [nK][npv] packed pair entries
    int *d_pair_inv = nullptr;    // [nstr][nel(nel-1)/2] rows K*npv+e producing each string
    // materialised same-spin rows of spaces with several types: the row of pair
    // entry (K, e), which produces string J, is J's padded sigma row (the blocks
    // allowed with J's type, concatenated); ny = 0: no such rows
    int64_t ny = 0;               // elements of all rows
    int64_t *d_yoff = nullptr;    // [nK][npv] first element of each entry's row (-1: no string)
    int *d_ycol = nullptr;        // [ntype][ntype_other] offset of each block in a row (-1: not allowed)
    // spaces with several types: the entries of each K whose string is in the space
    // come first in its pair list, and the K are grouped by that count into
    // buckets of one compiled pair-kernel shape each (K without entries in none)
    std::vector<int> bk_ks, bk_mbl, bk_start;   // per bucket: shape, first position in d_klist (+ end)
    int *d_klist = nullptr;                     // K indices, bucket by bucket
    uint64_t *d_gkey = nullptr;   // [ngtype]
    int *d_graw = nullptr;        // [ngtype+1]
    uint32_t *d_radix = nullptr;  // [ngtype][ngas] mixed-radix digit weights of the raw rank
    int *d_remap = nullptr;       // raw index -> string index (spatial symmetry only)
    // per-string diagonal pieces (FP64): sum_{p in I} h_pp + 1/2 sum_{p,q in I} ((pp|qq) - (pq|qp))
    double *d_adiag = nullptr;    // [nstr]
};

// packed single-excitation entry:  J << 11 | k << 6 | l << 1 | negative
__host__ __device__ inline uint32_t exc_pack(uint32_t J, int k, int l, bool neg) {
    return (J << 11) | (uint32_t(k) << 6) | (uint32_t(l) << 1) | (neg ? 1u : 0u);
}
constexpr uint32_t kExcNone = 0xFFFFFFFFu;
// packed pair entry:  J << 11 | pairindex << 1 | negative
constexpr uint32_t kPairNone = 0xFFFFFFFFu;

// index of the unordered pair {p, q} with p >= q among pairs including the
// diagonal: p(p+1)/2 + q
__host__ __device__ inline int pair_ge(int p, int q) {
    return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p;
}
// index of the strict pair {p, q}, p > q: p(p-1)/2 + q
__host__ __device__ inline int pair_gt(int p, int q) {
    return p > q ? p * (p - 1) / 2 + q : q * (q - 1) / 2 + p;
}

// Blocks of the vector: (alpha type, beta type) in alpha-type-major order.
struct Layout {
    int nblk = 0;
    std::vector<int> blk_a, blk_b;
    std::vector<int64_t> blk_off;   // nblk + 1
    std::vector<int64_t> boff;      // [ntype_a][ntype_b], -1 = absent
    int64_t ndet = 0;
};

// Padded block layout of the CI vector with rows = strings of spin `rs` and
// columns = strings of the other spin.  Block (row type t, column type u)
// starts at seg[t][u] (-1 when the block is not in the space) and has row
// stride ld[u] = width of column type u rounded up to a multiple of 64, so
// every row segment is 256-byte aligned and 64-column tiles never straddle a
// row end.  The padding columns hold zeros.
constexpr int kTileCols = 64;
struct PadLayout {
    int rs = 0;
    std::vector<int> ld;          // [ntype_other]
    std::vector<int64_t> seg;     // [ntype_rs][ntype_other]
    int64_t size = 0;             // elements
    int ntiles = 0;               // 64-column tiles over all column types
    std::vector<int> tile_u, tile_c0;
    // device copies
    int64_t *d_seg = nullptr;
    int *d_ld = nullptr;
    int *d_tile_u = nullptr;
    int *d_tile_c0 = nullptr;
};

// One (alpha type, beta type) block as the conversion kernels see it.
struct BlockDev {
    int ta, tb, na, nb;         // types and string counts of the block
    int64_t off;                // offset in the caller's vector
    int64_t sega, segb;         // offsets in the alpha-major / beta-major padded layouts
    int lda, ldb;               // padded row strides there
};

struct BlockTilesDev {
    BlockDev *blk;
    int *tb, *tr, *tc;          // 64x64 tiles: block, first row, first column
    int ntiles;
};

// Conflict-free schedule of the beta-side scatter of the owner-computes
// sigma_3 kernel (32-column tiles): per tile, every contribution (target beta
// string, W row kl, column, sign) sorted by target and cut into 256
// per-thread ranges of whole target groups, each padded to a multiple of 4
// entries, so no two threads write the same sigma element within a tile.
// entry = first-of-group << 29 | negative << 28 | target << 13 | (kl*33 + column)
// no-op entry = 1 << 29 | ld << 13 | npair*33 (zero row of W, spare sigma slot).
struct ScatterPlan {
    uint32_t *d_entries[2] = {nullptr, nullptr};  // [FP64, FP32] entry encodings, [ntile][4][ew][64]
    int ntile = 0;
    int ew = 0;                                    // entries per lane and tile (0: no plan)
};

// Owner-computes sigma_3 for GAS spaces: W rows are the orbital pairs grouped
// by the GAS spaces of their two orbitals, the gathered rows of an alpha string
// are its single excitations grouped by source type, and every alpha type has
// the list of 32-column source tiles (of one beta type each) that can change
// its sigma, with the k steps and row blocks that can.
// Owner-computes sigma_3 on GAS spaces.  The sigma row of an alpha string
// holds only the beta strings of the blocks allowed with its type (the types
// concatenated: compact columns); a "unit" is one alpha type and a range of
// its compact columns short enough for the LDS of the precision (units differ
// per precision), with its own list of source tiles and its own scatter plan.
struct GasUnit {
    int ta = 0;                          // alpha type
    int lo = 0, hi = 0;                  // compact column range owned
    int act0 = 0, nact = 0;              // its source tiles in the act array
};
struct GasOwner {
    int ks = 0, rb = 0;                  // k steps (4 gathered rows each), 16-row blocks of W
    int *d_slot = nullptr;               // [ntype_a][4*ks] excitation index of each gathered row,
                                         //   -2: the string itself, -1: none
    int *d_coff = nullptr;               // [ntype_a][ntype_b] first compact column of each allowed block, -1
    float *d_g32 = nullptr;              // [n*n][16*rb] (ij|kl), kl in the grouped row order
    double *d_g64 = nullptr;
    // per precision ([0] FP64, [1] FP32)
    std::vector<GasUnit> units[2];
    std::vector<std::pair<int, int>> launch[2];   // per unit in device-table order: first workgroup, rows
    uint32_t *d_act[2] = {nullptr, nullptr};   // [.][4]: {plan tile, k-step mask, row-block mask,
                                               //   beta type | first column << 8}
    int *d_units[2] = {nullptr, nullptr};      // [.][8]: ta, lo, hi, act0, nact, first alpha string, first block
    int nblocks[2] = {0, 0};                   // workgroups of one launch over all units
    int maxcols[2] = {0, 0};                   // longest unit row
    ScatterPlan plan[2];                 // plan[d].d_entries[d]: tiles of all units (slots: elements)
};

struct Workspace {
    void *cp = nullptr;    // C in the alpha-major padded layout
    void *sp = nullptr;    // sigma accumulator, alpha-major padded layout
    void *ct = nullptr;    // C in the beta-major padded layout
    void *st = nullptr;    // beta same-spin sigma, beta-major padded layout
    void *ys = nullptr;    // materialised same-spin rows (one-type spins), ys_chunk columns each
    int ys_chunk = 0;
    bool ready = false;
};

}  // namespace cis

struct cisigma_ctx {
    int n = 0, na = 0, nb = 0;
    int sym = 0;                   // spatial symmetry (cisigma_init_sym)
    int orbsym[32] = {0};          // irrep of each orbital (0..7, products as XOR)
    int target = 0;                // irrep of the space
    cis::GasDesc gas{};
    std::vector<int> gas_norb, gas_min, gas_max;
    cis::SpinTables sp[2];
    cis::Layout lay;
    cis::PadLayout pl[2];          // [0] alpha-major, [1] beta-major
    int *d_tstart[2] = {nullptr, nullptr};   // device copies of SpinTables::tstart
    bool cas = true;               // one type per spin (single block)
    // the alpha and beta tables, layouts and allowed blocks are mirror images
    // (n_alpha = n_beta): the M_S = 0 sector is available; d_pblk[b] is the block
    // (tb, ta) of block b = (ta, tb), d_blkoff the caller-layout block offsets
    bool spin_sym = false;
    int *d_pblk = nullptr;
    int64_t *d_blkoff = nullptr;
    std::vector<double> h, g;      // host copies of the integrals
    // device integral tables
    int npair = 0;                 // n(n+1)/2 (pairs with diagonal)
    int kp = 0;                    // npair rounded up to a multiple of 4
    int nps = 0;                   // n(n-1)/2 strict pairs
    double *d_gp64 = nullptr;      // [n*n][kp]: (ij|kl) with kl = pair_ge(k, l)
    float *d_gp32 = nullptr;
    double *d_v64[2] = {nullptr, nullptr};  // [nps][nps] same-spin pair matrix per spin
    float *d_v32[2] = {nullptr, nullptr};
    double *d_h64 = nullptr;       // [n][n]
    float *d_h32 = nullptr;
    double *d_jpq = nullptr;       // [n][n] (pp|qq)
    cis::Workspace ws[2];          // per dtype (0 FP64, 1 FP32)
    cis::BlockTilesDev bt{};       // tiles of the caller-layout blocks
    cis::ScatterPlan plan;         // beta-side scatter plan of the owner-computes sigma_3 kernel
    // general sigma_3 kernel: per alpha type, the 64-column beta tiles that can
    // change sigma (CSR over alpha types; all tiles for one-block spaces)
    int *d_act_start = nullptr;    // [ntype_a + 1]
    int *d_act_tiles = nullptr;
    int act_max = 0;
    cis::GasOwner go;              // owner-computes sigma_3 tables for GAS spaces (go.ks = 0: none)
    hipStream_t stream = nullptr;  // own stream for synchronous calls
    int dev = 0;                   // HIP device the context's tables live on
    void *scratch = nullptr;       // device address of that device's no-allocation scratch (api.hip)
    // beta-beta pass of apply on a second stream, overlapping the alpha-beta pass
    // (CISIGMA_OPT_OVERLAP); created with the workspace, default priority
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int overlap = 0;
    // options
    int precision = CISIGMA_FP64;
    int max_space = 0;
    int max_iter = 100;
    int ss_split = 0;              // same-spin atomic kernels: column split of the grid (0: heuristic; autotuned)
    int unit_order[2] = {0, 0};    // GAS owner units' launch order per precision ([0] FP64, [1] FP32; autotuned)
    int low_memory = 0;            // swap the sigma workspaces around refinements (CISIGMA_OPT_LOW_MEMORY)
    int pspace = 256;              // Davidson P-space size (CISIGMA_OPT_PSPACE)
    int thick_restart = 1;         // collapses keep the previous Ritz vectors too (CISIGMA_OPT_THICK_RESTART)
    int refine_every = 0;          // mixed mode: 0 = refine only when the FP32 iteration converges
    double resid_tol = -1.0;
    int verbose = 0;
    std::string log_path;          // Davidson JSON-lines log (cisigma_set_log; empty: none)
    int log_calls = 0;             // Davidson calls logged so far
    int last_path[2] = {0, 0};     // CISIGMA_PATH_* flags of the last apply, [FP64, FP32]
    int last_shape[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};   // owner-computes sigma_3 shape of the last apply
    int abx_shared[2] = {0, 0};    // the one-block owner kernel last ran two workgroups per CU, [FP64, FP32]
    // kernel choice: 0 automatic, 1 the general scatter-atomic kernels only (CISIGMA_OPT_SIGMA_PATH)
    int ab_mode = 0;               // CISIGMA_OPT_SIGMA_PATH
    int deterministic = 0;         // CISIGMA_OPT_DETERMINISTIC
    int unit_cols = 0;             // CISIGMA_OPT_UNIT_COLS (0: what the LDS holds)
    int unit_launch = 0;           // CISIGMA_OPT_UNIT_LAUNCH (0: one launch over all units, 1: one per unit)
    int ss_chunk = 0;      // cap on the materialised same-spin column chunk (0: none)
    int spin_parity = 0;   // M_S = 0 sector: C(Ib, Ia) = p C(Ia, Ib) assumed (0: none)
    // captured apply graphs (CISIGMA_OPT_GRAPH)
    struct ApplyGraph {
        const void *C;
        void *sigma;
        int dtype;
        hipStream_t stream;
        hipGraphExec_t exec;
        int path;
    };
    int graph_mode = 0;
    std::vector<ApplyGraph> graphs;
    double *d_rdm = nullptr;   // density-matrix partial sums (allocated on first use)
    size_t rdm_elems = 0;
    // per-pass event timing of apply (CISIGMA_OPT_PROFILE)
    bool profile = false;
    std::vector<hipEvent_t> prof_events;   // pending pairs, (CISIGMA_NPASS + 1) events per call
    std::vector<int> prof_pending;         // calls recorded but not yet summed
    double prof_ms[CISIGMA_NPASS] = {0};
    int prof_calls = 0;
    std::string err;
};

// ---- launchers (defined in the .hip files) -------------------------------
namespace cis {

hipError_t build_string_tables(cisigma_ctx *ctx, int spin);
hipError_t build_diag_tables(cisigma_ctx *ctx);

// sigma pieces; dtype 0 = double, 1 = float
// padded K extent of the (ij|kl) table used by the alpha-beta kernel
int sigma_ab_kp(int npair);
hipError_t launch_fill(void *x, int64_t n, int dtype, hipStream_t s);
hipError_t launch_sigma_ab(const cisigma_ctx *ctx, const void *C, void *sigma, int dtype, hipStream_t s);
// owner-computes sigma_3 (one-block spaces with a scatter plan): false when the
// shape has no compiled kernel (nothing launched), else *err is the launch status
bool launch_sigma_ab_owner(const cisigma_ctx *ctx, const void *C, void *sigma, int dtype, hipStream_t s,
                           hipError_t *err);
// plan width (entries per lane and tile) the owner-computes kernel uses for a
// shape that needs `need`; 0 when no compiled kernel covers it
int sigma_ab_owner_width(int anexc, int npair, int need);
// the same for the GAS owner-computes kernel with ks k steps and rb row blocks
int sigma_ab_gas_width(int ks, int rb, int need);
// owner-computes sigma_3 on a GAS space: false when no compiled kernel covers it
bool launch_sigma_ab_gas(const cisigma_ctx *ctx, const void *C, void *sigma, int dtype, hipStream_t s,
                         hipError_t *err);
// Ys == nullptr: scatter with atomics into Y (Y holds what to add to).
// Ys != nullptr (one-type spins): materialise into Ys chunk by chunk (chunk
// columns, a multiple of 64) and gather into Y, overwriting Y.
hipError_t launch_sigma_same_spin(const cisigma_ctx *ctx, int spin, const void *X, void *Y, int dtype,
                                  hipStream_t s, void *Ys = nullptr, int chunk = 0);
// whether the same-spin pair count npv has compiled MFMA kernels (else a plain
// atomic kernel serves it and the materialised form is not used)
bool same_spin_materialisable(int npv);
// smallest compiled same-spin pair-kernel shape (k steps, 16-row blocks) for
// lists of `count` pairs; false when none is compiled
bool same_spin_shape_for(int count, int *ks, int *mbl);
// caller vector -> alpha-major and beta-major padded copies
hipError_t launch_scatter_in(const cisigma_ctx *ctx, const void *C, void *cp, void *ct, int dtype, hipStream_t s);
// sigma = alpha-major accumulator + transpose of the beta-major accumulator
hipError_t launch_gather_out(const cisigma_ctx *ctx, const void *sp, const void *st, void *sigma, int dtype,
                             hipStream_t s);
hipError_t launch_hdiag(const cisigma_ctx *ctx, double *out, hipStream_t s);
// sigma = sp + st + p st^T on the one-block layout (st: the alpha-alpha part, alpha-major)
hipError_t launch_gather_parity(const cisigma_ctx *ctx, const void *sp, const void *st, void *sigma, int parity,
                                int dtype, hipStream_t s);
// x <- (x + p x^T) / 2 for the caller's one-block vector x[n][n]
hipError_t launch_symmetrize(void *x, int n, int parity, int dtype, hipStream_t s);
// (x + p x^T) / 2 in place on a caller-layout vector of a space with several
// blocks (the transpose maps block (ta, tb) onto block (tb, ta))
hipError_t launch_symmetrize_blocks(const cisigma_ctx *ctx, void *x, int parity, int dtype, hipStream_t s);
inline BlockTilesDev block_tiles(const cisigma_ctx *ctx) { return ctx->bt; }

// density matrices (rdm.hip): one-block spaces, n <= 16
int rdm_blocks(int n);
size_t rdm_lds_bytes(const cisigma_ctx *ctx, int dtype);
size_t rdm_part_elems(const cisigma_ctx *ctx);
hipError_t launch_rdm(const cisigma_ctx *ctx, const void *cp, int dtype, double *part, double *rdm1, double *rdm2,
                      hipStream_t s);

// Hamiltonian elements between single determinants (hmat.hip): the strings of
// vector element idx (from host copies of both string tables), and H_IJ by the
// Slater-Condon rules
bool det_strings(const cisigma_ctx *c, int64_t idx, const std::vector<uint32_t> &astr,
                 const std::vector<uint32_t> &bstr, uint32_t *a, uint32_t *b);
double hmat_element(const cisigma_ctx *c, uint32_t a1, uint32_t b1, uint32_t a2, uint32_t b2);

// Davidson driver (davidson.hip)
int davidson(cisigma_ctx *ctx, int nroots, double tol, double *energies, void *vecs, cisigma_stats *stats);
// sigma of one device vector on the given stream (api.hip)
int apply_sigma(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, hipStream_t s);
// the same with the workspace carved from the static scratch array (no allocation)
int apply_sigma_noalloc(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, hipStream_t s);
// the same through a captured graph (CISIGMA_OPT_GRAPH; non-NULL stream)
int apply_sigma_graph(cisigma_ctx *ctx, const void *C, void *sigma, int dtype, hipStream_t s);
void drop_graphs(cisigma_ctx *ctx);
// whether one dtype's sigma workspace is allocated or its layout copies fit in
// free memory; freeing it (synchronises the device; the next apply of that
// dtype allocates it again)
bool workspace_fits(cisigma_ctx *ctx, int dtype);
// launch order of the GAS owner units of one precision: 0 most source tiles per
// row first (as built), 1 alpha type order, 2 most total work first, 3 heavy
// and light alternating; rewrites the device unit table
int gas_set_unit_order(cisigma_ctx *ctx, int d, int order);
int rebuild_gas_owner(cisigma_ctx *ctx);
int release_workspace(cisigma_ctx *ctx, int dtype);

}  // namespace cis

int cis_set_error(cisigma_ctx *ctx, int code, const std::string &msg);
