// mtpt_kernels.h -- device data layout and kernel entry points of the MTPT
// step on gfx950.  Shared by the single-sim runtime and the serving pool.
//
// Layout in HBM (per simulation, n particles, S species, T = double in FP64
// mode and float otherwise, M = float in Kahan mode and double otherwise):
//   X[k][n]     T    positions, structure of arrays, sorted by cell (cells
//                    numbered x fastest) and inside a cell by (x, pid), so
//                    every row of cells is one x-sorted run of the arrays
//   XT[k][n]    T    walked positions in the order before re-binning
//   J[k][n]     T    the next step's jumps, sorted order (drawn by place)
//   M[2][S][n]  M    masses, two buffers (Jacobi update)
//   P[2][n]     u32  pid of each sorted slot, two buffers
//   Srow[n]     T    row sums s_i = sum_j K_ij
//   cmask[pl][n] u64 neighbour bits of the candidate rows, per plane
//   cwin[pl][n]  u64 trimmed x-windows of the candidate rows, per plane (trimmed sims only)
//   cell, rank, perm [n] u32   binning scratch (rank bit 31: left its tile)
//   counts[], tcounts[], starts[] u32   cell histograms (global atomics;
//                    per-tile stores) and offsets, tile-padded
//   bsum[]      u32  per-tile partial sums of the scan
//   partials[]  f64  per-workgroup mass partial sums [parts][S]
//   pair_part[] u32  per-workgroup pair counts
//   DevStats         counters and totals
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtpt {

constexpr int kBlock = 256;          // threads per workgroup, 4 wave64s
#ifndef MTPT_SCAN_ITEMS
#define MTPT_SCAN_ITEMS 8
#endif
constexpr int kScanItems = MTPT_SCAN_ITEMS;   // counts per thread in the scan (a multiple of 4)
constexpr int kScanTile = kBlock * kScanItems;
// rows of three cells holding at least this many particles on average are
// trimmed to each particle's x-window before its candidate loop (measured:
// it pays at ~20 per row in 3-d, and costs 20-30 % at 4-6 per row)
#ifndef MTPT_TRIM_MIN_ROW
#define MTPT_TRIM_MIN_ROW 12.0
#endif
constexpr int kFinalBlock = 1024;    // threads of the finalize kernel
// neighbour bits of a particle whose row-sum tile did not record them (a
// recorded mask covers at most 63 candidates, so bit 63 is free)
constexpr uint64_t kMaskInvalid = 1ull << 63;
constexpr uint32_t kScanFold = 2048;  // scans of at most this many tiles skip the top pass
// LDS staging budget (bytes) of a tile of the mass-transfer passes, per
// dimension, precision and species count (3-d halos hold three planes of
// cell rows).  Chosen by measurement: the FP32 one-species kernels trade
// workgroups per CU (LDS-limited) against halo overhead per tile; the FP64
// and three-species kernels are limited by registers and take larger tiles.
#ifndef MTPT_LDS_BUDGET_2D
#define MTPT_LDS_BUDGET_2D 20480
#endif
#ifndef MTPT_LDS_BUDGET_2D_F64
#define MTPT_LDS_BUDGET_2D_F64 24576
#endif
#ifndef MTPT_LDS_BUDGET_3D
#define MTPT_LDS_BUDGET_3D 35000
#endif
#ifndef MTPT_LDS_BUDGET_3D_WIDE
#define MTPT_LDS_BUDGET_3D_WIDE 46080
#endif
// 3-d three-species FP32-position transfer pass: with 32 KiB and its candidate
// loop unrolled by 2 (114 VGPRs) it holds four workgroups per CU (measured
// 2.13 ms per launch on the 3.2e7-particle reacting workload, against 2.24 ms
// with 45 KiB tiles at three workgroups per CU; 32 KiB unrolled by 4 at
// three workgroups: 2.54 ms)
#ifndef MTPT_LDS_BUDGET_3D_S3
#define MTPT_LDS_BUDGET_3D_S3 32768
#endif
template <int D, int PREC, int NS> struct LdsBudget {
    static constexpr int value =
        D == 3 ? (PREC != 0 ? (NS == 1 ? MTPT_LDS_BUDGET_3D : MTPT_LDS_BUDGET_3D_S3) : MTPT_LDS_BUDGET_3D_WIDE)
               : (PREC == 0 ? MTPT_LDS_BUDGET_2D_F64 : MTPT_LDS_BUDGET_2D);
};
// 3-d tiled passes keep a table of each own particle's row (else a search)
#ifndef MTPT_ROW_TABLE_3D
#define MTPT_ROW_TABLE_3D 0
#endif
// the 2-d FP64 row-sum pass hands its own cells to lanes in order of their
// candidate count
#ifndef MTPT_CELL_ORDER_2D
#define MTPT_CELL_ORDER_2D 1
#endif
#ifndef MTPT_CELL_ORDER_2D_F32
#define MTPT_CELL_ORDER_2D_F32 0
#endif
// unroll factor of the candidate loop of the tiled passes (the FP64 2-d
// loops run at lower occupancy and gain from two candidates in flight)
#ifndef MTPT_CAND_UNROLL_2D
#define MTPT_CAND_UNROLL_2D 1
#endif
#ifndef MTPT_CAND_UNROLL_2D_F64
#define MTPT_CAND_UNROLL_2D_F64 2
#endif
#ifndef MTPT_CAND_UNROLL_3D
#define MTPT_CAND_UNROLL_3D 4
#endif
// the 3-d three-species transfer pass (registers: its occupancy level)
#ifndef MTPT_CAND_UNROLL_3D_S3
#define MTPT_CAND_UNROLL_3D_S3 2
#endif

// Largest tile (cells in x, y and z) of the mass-transfer passes, the halo
// cell rows it spans and the cell boundaries kept per halo row.  Halo rows
// (segments) are numbered with a fixed pitch per plane, seg_y (a power of two
// in 3-d), and the tile's own rows with the same pitch, so that a row's plane
// and the halo row of an own row follow from shifts and adds; col_p is the
// power of two >= cols used to hand boundaries to threads.
template <int D> struct TileLimits {
    static constexpr int max_x = D == 2 ? 24 : 12;
    static constexpr int max_y = D == 2 ? 24 : 6;
    static constexpr int max_z = D == 2 ? 1 : 6;
    static constexpr int seg_y = max_y + 2;
    static constexpr int segs = (D == 3 ? max_z + 2 : 1) * seg_y;
    static constexpr int own_rows = (D == 3 ? max_z : 1) * seg_y;
    static constexpr int cols = max_x + 3;
    static constexpr int col_p = D == 2 ? 32 : 16;
    static_assert(D == 2 || (seg_y & (seg_y - 1)) == 0, "3-d halo rows need a power-of-two pitch");
    static_assert(cols <= col_p, "column pitch too small");
};
inline int tile_max(int dim, int axis)
{
    if (dim == 2)
        return axis == 0 ? TileLimits<2>::max_x : axis == 1 ? TileLimits<2>::max_y : 1;
    return axis == 0 ? TileLimits<3>::max_x : axis == 1 ? TileLimits<3>::max_y : TileLimits<3>::max_z;
}

struct DevStats {
    unsigned long long pairs_last;   // pairs of the last step
    unsigned long long pairs_total;  // over all steps
    int nonfinite;                   // sticky: a total was NaN or infinite
    int pad0;
    double totals[3];                // mass totals after the last step
    long long steps;                 // steps completed on the device
    double initial[3];               // totals after the set-up binning (copied on the
                                     // device, read when the statistics are asked for)
};

// Everything one launch of one phase needs about one simulation.  Pointers
// are resolved by the host for the step being enqueued.
struct SimArgs {
    int64_t n;
    int32_t ns;              // species (1 or 3)
    int32_t moving;          // particles move (D_RW > 0 or a drift)
    // cell grid: cell side >= the cutoff's reach along every axis (psi, or
    // psi sqrt(T_kk) with a dispersion tensor)
    double glo[3];
    double inv_side[3];
    int32_t nc[3];
    uint32_t ncells;
    // tiles of the mass-transfer passes: tx * ty * tz cells (tz = 1 in 2-d),
    // numbered x fastest; the row-sum pass (tile...) and the transfer pass
    // (ttile...) each have their own plan (they differ when the transfer
    // stages more species than the row-sum pass's positions)
    int32_t tile[3];
    uint32_t tiles_x, tiles_y, ntiles;
    int32_t ttile[3];
    uint32_t ttiles_x, ttiles_y, nttiles;
    // box and walk
    double lo[3], hi[3];
    float lof[3], hif[3];
    double sdev;             // sqrt(2 D_RW dt)
    double drift[3];         // v dt, the advective displacement per step
    uint64_t seed;
    int64_t step;
    // weights: K = exp(-kc r^2), kc = beta / (4 D_MT dt)
    double psi;
    double psi2;             // psi * psi (FP64, the canonical cutoff)
    double win;              // x-window half width, psi (1 + 1e-6)
    double side[3];          // cell side per dimension
    double win2d;            // win * win
    float win2f;
    float wmarginf;          // rounding margin of row windows (FP32 positions)
    double wmargind;         // the same for FP64 positions
    float psi2_in;           // FP32 r^2 below this: inside for sure
    float psi2_out;          // FP32 r^2 above this: outside for sure
    double kc;
    float kcf;
    float kcf2;              // -kc log2(e): K = 2^(kcf2 r^2) in FP32
    float betaf;
    float pad2;
    double beta;
    double k_react, to_c, to_m, dt;
    // buffers
    void* x[3];
    void* xt[3];
    void* jmp[3];            // next step's jumps (type of the positions), sorted order
    void* m_src[3];          // masses in the order before re-binning (place source)
    void* m_mid[3];          // masses in the current sorted order
    void* m_dst[3];          // transfer output
    uint32_t* pid_src;
    uint32_t* pid_dst;       // place output = current sorted pids
    void* srow;
    uint32_t* cell;
    uint32_t* rank;
    uint32_t* perm;          // slot -> particle of the order before re-binning
    uint32_t* src_slot;      // null, or: the place pass records each sorted slot's
                             // particle of the order before re-binning here (the
                             // cell buffer, free by then) and leaves the masses to
                             // the row-sum pass, which gathers them from m_src
    uint32_t* counts;        // per-cell histogram filled with global atomics
    uint32_t* tcounts;       // per-cell counts of particles that stayed in their tile
    uint64_t* cmask;         // [plane][n] neighbour bits of the candidate rows (row-sum pass;
                             // kMaskInvalid where the pass recorded none)
    uint64_t* cwin;          // [plane][n] x-windows of the trimmed rows (row-sum pass), or null
    uint32_t* starts;
    uint32_t* bsum;
    double* partials;
    uint32_t* pair_part;
    DevStats* st;
    uint32_t scan_blocks;    // ceil((ncells + 1) / kScanTile)
    int32_t scan_fold;       // scan_blocks <= kScanFold: the down pass sums the block totals itself
    uint32_t part_blocks;    // ceil(n / kBlock)
    int32_t recompute_s;     // the row-sum pass ran this step
    int32_t walk;            // apply the jump in the bin pass (0 at create)
    int32_t fuse_bin;        // the transfer pass also bins for the next step
    int32_t tcounts_valid;   // this step's binning came from the transfer pass:
                             // cell count = counts + tcounts
    int32_t trim_rows;       // trim candidate rows to the per-row x-window
    // dispersion tensor T = L L^T (shape of D_RW and D_MT): jumps L z, distance
    // q = |M dx|^2 with M = L^-1 (tensor == 0: isotropic, L = M = I unused)
    int32_t tensor;
    int32_t pad4;
    double lch[6];           // L00, L10, L11, L20, L21, L22
    double minv[6];          // M00, M10, M11, M20, M21, M22
    float minvf[6];          // M rounded to FP32
    // export of the pairs a tiled pass uses (mtpt_step_neighbors; null otherwise)
    uint32_t* nb_cnt;        // count pass: pairs + 1 per pid
    const int64_t* nb_row;   // fill pass: CSR row offsets by pid
    int64_t* nb_col;         // fill pass: CSR columns (pids)
};

// Batched launches: a device array of SimArgs and a device prefix of blocks
// per sim; block b of the launch belongs to the sim whose prefix range holds b.
struct Batch {
    const SimArgs* args;
    const uint32_t* blk_off;   // [nsims + 1]
    int32_t nsims;
    uint32_t total_blocks;
};

enum Phase {
    PH_BIN = 0,       // walk + reflect + cell id + histogram
    PH_SCAN_REDUCE,   // per-tile sums of the histogram
    PH_SCAN_TOP,      // scan of the tile sums
    PH_SCAN_DOWN,     // cell offsets, histogram cleared
    PH_SCATTER,       // slot of every particle inside its cell
    PH_PLACE,         // rank inside the cell by (x, pid); gather into place
    PH_ROWSUM,        // s_i
    PH_TRANSFER,      // exchange (+ reaction), per-workgroup mass sums
    PH_FINALIZE,      // totals, pair counters
    PH_COUNT
};

const char* phase_name(int ph);

// particles staged per workgroup by the transfer pass (the tighter of the
// two tiled passes)
int tile_capacity(int dim, int prec, int ns);

// blocks a phase needs for one sim
uint32_t phase_blocks(int ph, const SimArgs& a);

// single-sim launch of a phase
hipError_t launch_phase(int ph, int dim, int prec, const SimArgs& a, hipStream_t s);
// PH_PLACE of a, with the PH_FINALIZE of the previous step prev run by one
// more workgroup of the same launch
hipError_t launch_place_fin(int dim, int prec, const SimArgs& a, const SimArgs& prev, hipStream_t s);
// batched launch of a phase over sims that share (dim, prec, ns, tensor)
hipError_t launch_phase_batched(int ph, int dim, int prec, int ns, int tn, const Batch& b, hipStream_t s);
// the two tiled passes (PH_ROWSUM, PH_TRANSFER) of dimension D, isotropic or
// tensor metric TN: one sim (a) or a batch (b, with a == nullptr)
template <int D, bool TN>
hipError_t launch_tiles(int ph, int prec, int ns, const SimArgs* a, const Batch* b, hipStream_t s);
// the same passes recording the pairs they use (a.nb_* set), storing nothing
template <int D, bool TN>
hipError_t launch_tiles_export(int ph, int prec, int ns, const SimArgs& a, hipStream_t s);
// rows of a CSR sorted ascending, in place
hipError_t launch_nb_sort(int64_t n, const int64_t* row_ptr, int64_t* col, hipStream_t s);

// exports and set-up
hipError_t launch_unpermute_mass(int prec, const SimArgs& a, const void* const* m_cur,
                                 const uint32_t* pid_cur, double* out, hipStream_t s);
hipError_t launch_unpermute_pos(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                                double* out, hipStream_t s);
hipError_t launch_totals(int prec, const SimArgs& a, const void* const* m_cur, hipStream_t s);
hipError_t launch_nb_count(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                           uint32_t* rowcnt, hipStream_t s);
hipError_t launch_nb_fill(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                          const int64_t* row_ptr, int64_t* col, hipStream_t s);
// out[i] = i for i < n (the pids of the input order)
hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_scan_u32_to_i64(const uint32_t* in, int64_t* out, int64_t len, uint32_t* tmp,
                                  uint32_t* bsum, hipStream_t s);

}  // namespace mtpt
