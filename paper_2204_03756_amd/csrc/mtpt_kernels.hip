// mtpt_kernels.hip -- HIP kernels of the MTPT step for gfx950 (wave64) other
// than the two tiled passes: binning (walk, histogram, scan, scatter,
// place), totals, exports, and the host-side launchers of every phase (the
// tiled passes are instantiated in mtpt_tiles_*.hip).
#include "mtpt_device.h"

namespace mtpt {

// the tiled passes, compiled in their own translation units
extern template hipError_t launch_tiles<2, false>(int, int, int, const SimArgs*, const Batch*, hipStream_t);
extern template hipError_t launch_tiles<2, true>(int, int, int, const SimArgs*, const Batch*, hipStream_t);
extern template hipError_t launch_tiles<3, false>(int, int, int, const SimArgs*, const Batch*, hipStream_t);
extern template hipError_t launch_tiles<3, true>(int, int, int, const SimArgs*, const Batch*, hipStream_t);
extern template hipError_t launch_tiles_export<2, false>(int, int, int, const SimArgs&, hipStream_t);
extern template hipError_t launch_tiles_export<2, true>(int, int, int, const SimArgs&, hipStream_t);
extern template hipError_t launch_tiles_export<3, false>(int, int, int, const SimArgs&, hipStream_t);
extern template hipError_t launch_tiles_export<3, true>(int, int, int, const SimArgs&, hipStream_t);


template <int D, typename T>
__global__ __launch_bounds__(kBlock) void bin_k(SimArgs a) { bin_body<D, T>(a, xcd_block(blockIdx.x, gridDim.x)); }
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void bin_kb(Batch b) { MTPT_BATCH_PROLOGUE; bin_body<D, T>(a, l); }

__global__ __launch_bounds__(kBlock) void scan_reduce_k(SimArgs a) { scan_reduce_body(a.counts, a.tcounts_valid ? a.tcounts : nullptr, a.bsum, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void scan_reduce_kb(Batch b) { MTPT_BATCH_PROLOGUE; scan_reduce_body(a.counts, a.tcounts_valid ? a.tcounts : nullptr, a.bsum, l); }
__global__ __launch_bounds__(kBlock) void scan_top_k(SimArgs a) { if (!a.scan_fold) scan_top_body(a.bsum, a.scan_blocks); }
__global__ __launch_bounds__(kBlock) void scan_top_kb(Batch b) { MTPT_BATCH_PROLOGUE; (void)l; if (!a.scan_fold) scan_top_body(a.bsum, a.scan_blocks); }
__global__ __launch_bounds__(kBlock) void scan_down_k(SimArgs a) { scan_down_body(a.counts, a.tcounts_valid ? a.tcounts : nullptr, a.starts, a.bsum, blockIdx.x, true, a.scan_fold != 0); }
__global__ __launch_bounds__(kBlock) void scan_down_kb(Batch b) { MTPT_BATCH_PROLOGUE; scan_down_body(a.counts, a.tcounts_valid ? a.tcounts : nullptr, a.starts, a.bsum, l, true, a.scan_fold != 0); }
__global__ __launch_bounds__(kBlock) void scatter_k(SimArgs a) { scatter_body(a, xcd_block(blockIdx.x, gridDim.x)); }
__global__ __launch_bounds__(kBlock) void scatter_kb(Batch b) { MTPT_BATCH_PROLOGUE; scatter_body(a, l); }

template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void place_k(SimArgs a)
{
    place_body<D, typename Types<PREC>::T, typename Types<PREC>::M>(a, xcd_block(blockIdx.x, gridDim.x));
}
template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void place_kb(Batch b)
{
    MTPT_BATCH_PROLOGUE;
    place_body<D, typename Types<PREC>::T, typename Types<PREC>::M>(a, l);
}

// place_k with one more workgroup, the first, that finalizes the previous
// step (its totals and pair counters) while the gathers run
template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void place_fin_k(SimArgs a, SimArgs prev)
{
    if (blockIdx.x == 0) {
        finalize_body<kBlock>(prev, prev.nttiles, 0);
        return;
    }
    place_body<D, typename Types<PREC>::T, typename Types<PREC>::M>(a, xcd_block(blockIdx.x - 1, gridDim.x - 1));
}
__global__ __launch_bounds__(kFinalBlock) void finalize_k(SimArgs a, uint32_t nparts, int mode)
{
    finalize_body<kFinalBlock>(a, nparts, mode);
}
__global__ __launch_bounds__(kFinalBlock) void finalize_kb(Batch b)
{
    MTPT_BATCH_PROLOGUE;
    (void)l;
    finalize_body<kFinalBlock>(a, a.nttiles, 0);
}

#undef MTPT_BATCH_PROLOGUE
// ----------------------------------------------------------------- exports
template <typename M>
__global__ __launch_bounds__(kBlock) void unpermute_mass_k(int64_t n, int ns, const M* m0, const M* m1,
                                                           const M* m2, const uint32_t* pid, double* out)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= n)
        return;
    const int64_t p = pid[k];
    out[p] = static_cast<double>(m0[k]);
    if (ns == 3) {
        out[n + p] = static_cast<double>(m1[k]);
        out[2 * n + p] = static_cast<double>(m2[k]);
    }
}

__global__ __launch_bounds__(kBlock) void iota_k(uint32_t* out, int64_t n)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n)
        out[i] = static_cast<uint32_t>(i);
}

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void unpermute_pos_k(int64_t n, const T* x0, const T* x1, const T* x2,
                                                          const uint32_t* pid, double* out)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= n)
        return;
    const int64_t p = pid[k];
    out[p * D + 0] = static_cast<double>(x0[k]);
    out[p * D + 1] = static_cast<double>(x1[k]);
    if (D == 3)
        out[p * D + 2] = static_cast<double>(x2[k]);
}

// per-block sums of the current masses (then finalize in totals-only mode)
template <typename M>
__global__ __launch_bounds__(kBlock) void totals_k(SimArgs a, const M* m0, const M* m1, const M* m2)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const M* ms[3] = {m0, m1, m2};
    for (int c = 0; c < a.ns; ++c) {
        const double v = i < a.n ? static_cast<double>(ms[c][i]) : 0.0;
        const double t = block_sum<kBlock, double>(v);
        if (threadIdx.x == 0)
            a.partials[static_cast<size_t>(blockIdx.x) * a.ns + c] = t;
    }
}

// The neighbour export walks the full 3^d cells around each particle
// (independent of the tiles and windows of the hot passes).
template <int D, typename T, typename F>
__device__ __forceinline__ void for_candidates(const SimArgs& a, const T* xi, F&& f)
{
    int cc[3];
#pragma unroll
    for (int k = 0; k < D; ++k)
        cc[k] = cell_coord(static_cast<double>(xi[k]), a.glo[k], a.inv_side[k], a.nc[k]);
    const int x0 = cc[0] > 0 ? cc[0] - 1 : 0;
    const int x1 = cc[0] < a.nc[0] - 1 ? cc[0] + 1 : a.nc[0] - 1;
    const int zlo = (D == 3) ? (cc[2] > 0 ? cc[2] - 1 : 0) : 0;
    const int zhi = (D == 3) ? (cc[2] < a.nc[2] - 1 ? cc[2] + 1 : a.nc[2] - 1) : 0;
    const int ylo = cc[1] > 0 ? cc[1] - 1 : 0;
    const int yhi = cc[1] < a.nc[1] - 1 ? cc[1] + 1 : a.nc[1] - 1;
    for (int z = zlo; z <= zhi; ++z) {
        for (int y = ylo; y <= yhi; ++y) {
            const uint32_t row = (static_cast<uint32_t>(z) * a.nc[1] + y) * a.nc[0];
            const uint32_t j0 = a.starts[row + x0];
            const uint32_t j1 = a.starts[row + x1 + 1];
            for (uint32_t j = j0; j < j1; ++j)
                f(j);
        }
    }
}

template <int D, int PREC, bool TN>
__global__ __launch_bounds__(kBlock) void nb_count_k(SimArgs a, const uint32_t* pid, uint32_t* rowcnt)
{
    using T = typename Types<PREC>::T;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= a.n)
        return;
    T xi[3];
#pragma unroll
    for (int k = 0; k < D; ++k)
        xi[k] = static_cast<const T*>(a.x[k])[i];
    uint32_t cnt = 0;
    for_candidates<D, T>(a, xi, [&](uint32_t j) {
        T xj[3];
#pragma unroll
        for (int k = 0; k < D; ++k)
            xj[k] = static_cast<const T*>(a.x[k])[j];
        T r2;
        if (Metric<D, T, TN>::inside(a, xi, xj, &r2))
            ++cnt;
    });
    rowcnt[pid[i]] = cnt;
}

template <int D, int PREC, bool TN>
__global__ __launch_bounds__(kBlock) void nb_fill_k(SimArgs a, const uint32_t* pid, const int64_t* row_ptr,
                                                    int64_t* col)
{
    using T = typename Types<PREC>::T;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= a.n)
        return;
    T xi[3];
#pragma unroll
    for (int k = 0; k < D; ++k)
        xi[k] = static_cast<const T*>(a.x[k])[i];
    const int64_t base = row_ptr[pid[i]];
    int64_t cnt = 0;
    for_candidates<D, T>(a, xi, [&](uint32_t j) {
        T xj[3];
#pragma unroll
        for (int k = 0; k < D; ++k)
            xj[k] = static_cast<const T*>(a.x[k])[j];
        T r2;
        if (Metric<D, T, TN>::inside(a, xi, xj, &r2))
            col[base + cnt++] = static_cast<int64_t>(pid[j]);
    });
    for (int64_t k = 1; k < cnt; ++k) {
        const int64_t v = col[base + k];
        int64_t j = k;
        while (j > 0 && col[base + j - 1] > v) {
            col[base + j] = col[base + j - 1];
            --j;
        }
        col[base + j] = v;
    }
}

// each CSR row sorted ascending (insertion sort: rows are short)
__global__ __launch_bounds__(kBlock) void nb_sort_k(int64_t n, const int64_t* row_ptr, int64_t* col)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const int64_t b = row_ptr[i], e = row_ptr[i + 1];
    for (int64_t k = b + 1; k < e; ++k) {
        const int64_t v = col[k];
        int64_t j = k;
        while (j > b && col[j - 1] > v) {
            col[j] = col[j - 1];
            --j;
        }
        col[j] = v;
    }
}

// exclusive scan of n u32 counts into int64 offsets (n+1 values): copy into a
// tile-padded buffer, scan like the histogram, widen
__global__ __launch_bounds__(kBlock) void widen_k(const uint32_t* in, int64_t* out, int64_t len)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k <= len)
        out[k] = static_cast<int64_t>(in[k]);
}
__global__ __launch_bounds__(kBlock) void copy_pad_k(const uint32_t* in, uint32_t* out, int64_t len, int64_t padded)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k < padded)
        out[k] = k < len ? in[k] : 0u;
}
__global__ __launch_bounds__(kBlock) void scan_reduce_raw_k(const uint32_t* in, uint32_t* bsum) { scan_reduce_body(in, nullptr, bsum, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void scan_top_raw_k(uint32_t* bsum, uint32_t nb) { scan_top_body(bsum, nb); }
__global__ __launch_bounds__(kBlock) void scan_down_raw_k(uint32_t* in, uint32_t* out, const uint32_t* bsum)
{
    scan_down_body(in, nullptr, out, bsum, blockIdx.x, false);
}

// ------------------------------------------------------------- host side
const char* phase_name(int ph)
{
    static const char* names[PH_COUNT] = {"bin", "scan_reduce", "scan_top", "scan_down", "scatter",
                                          "place", "rowsum", "transfer", "finalize"};
    return (ph >= 0 && ph < PH_COUNT) ? names[ph] : "?";
}

int tile_capacity(int dim, int prec, int ns)
{
#define MTPT_CAP(D, P) (ns == 3 ? TileCap<D, P, 3, true>::value : TileCap<D, P, 1, true>::value)
    if (dim == 2)
        return prec == 0 ? MTPT_CAP(2, 0) : prec == 1 ? MTPT_CAP(2, 1) : MTPT_CAP(2, 2);
    return prec == 0 ? MTPT_CAP(3, 0) : prec == 1 ? MTPT_CAP(3, 1) : MTPT_CAP(3, 2);
#undef MTPT_CAP
}

static uint32_t ceil_div(int64_t a, int64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

uint32_t phase_blocks(int ph, const SimArgs& a)
{
    if (a.n <= 0)
        return 0;
    switch (ph) {
    case PH_SCAN_REDUCE:
    case PH_SCAN_DOWN: return a.scan_blocks;
    case PH_SCAN_TOP:
    case PH_FINALIZE: return 1;
    case PH_ROWSUM: return a.ntiles;
    case PH_TRANSFER: return a.nttiles;
    default: return ceil_div(a.n, kBlock);
    }
}

#define MTPT_DISPATCH_D_PREC(KERNEL, GRID, NT, ARG)                                              \
    do {                                                                                         \
        if (dim == 2) {                                                                          \
            if (prec == 0) KERNEL<2, 0><<<GRID, NT, 0, s>>>(ARG);                                \
            else if (prec == 1) KERNEL<2, 1><<<GRID, NT, 0, s>>>(ARG);                           \
            else KERNEL<2, 2><<<GRID, NT, 0, s>>>(ARG);                                          \
        } else {                                                                                 \
            if (prec == 0) KERNEL<3, 0><<<GRID, NT, 0, s>>>(ARG);                                \
            else if (prec == 1) KERNEL<3, 1><<<GRID, NT, 0, s>>>(ARG);                           \
            else KERNEL<3, 2><<<GRID, NT, 0, s>>>(ARG);                                          \
        }                                                                                        \
    } while (0)

hipError_t launch_phase(int ph, int dim, int prec, const SimArgs& a, hipStream_t s)
{
    const uint32_t grid = phase_blocks(ph, a);
    if (grid == 0)
        return hipSuccess;
    const int ns = a.ns;
    switch (ph) {
    case PH_BIN:
        if (dim == 2) {
            if (prec == 0) bin_k<2, double><<<grid, kBlock, 0, s>>>(a);
            else bin_k<2, float><<<grid, kBlock, 0, s>>>(a);
        } else {
            if (prec == 0) bin_k<3, double><<<grid, kBlock, 0, s>>>(a);
            else bin_k<3, float><<<grid, kBlock, 0, s>>>(a);
        }
        break;
    case PH_SCAN_REDUCE: scan_reduce_k<<<grid, kBlock, 0, s>>>(a); break;
    case PH_SCAN_TOP: scan_top_k<<<1, kBlock, 0, s>>>(a); break;
    case PH_SCAN_DOWN: scan_down_k<<<grid, kBlock, 0, s>>>(a); break;
    case PH_SCATTER: scatter_k<<<grid, kBlock, 0, s>>>(a); break;
    case PH_PLACE: MTPT_DISPATCH_D_PREC(place_k, grid, kBlock, a); break;
    case PH_ROWSUM:
    case PH_TRANSFER:
        if (dim == 2)
            return a.tensor ? launch_tiles<2, true>(ph, prec, ns, &a, nullptr, s)
                            : launch_tiles<2, false>(ph, prec, ns, &a, nullptr, s);
        return a.tensor ? launch_tiles<3, true>(ph, prec, ns, &a, nullptr, s)
                        : launch_tiles<3, false>(ph, prec, ns, &a, nullptr, s);
    case PH_FINALIZE: finalize_k<<<1, kFinalBlock, 0, s>>>(a, a.nttiles, 0); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_place_fin(int dim, int prec, const SimArgs& a, const SimArgs& prev, hipStream_t s)
{
    const uint32_t grid = phase_blocks(PH_PLACE, a) + 1;
    if (dim == 2) {
        if (prec == 0) place_fin_k<2, 0><<<grid, kBlock, 0, s>>>(a, prev);
        else if (prec == 1) place_fin_k<2, 1><<<grid, kBlock, 0, s>>>(a, prev);
        else place_fin_k<2, 2><<<grid, kBlock, 0, s>>>(a, prev);
    } else {
        if (prec == 0) place_fin_k<3, 0><<<grid, kBlock, 0, s>>>(a, prev);
        else if (prec == 1) place_fin_k<3, 1><<<grid, kBlock, 0, s>>>(a, prev);
        else place_fin_k<3, 2><<<grid, kBlock, 0, s>>>(a, prev);
    }
    return hipGetLastError();
}

hipError_t launch_phase_batched(int ph, int dim, int prec, int ns, int tn, const Batch& b, hipStream_t s)
{
    const uint32_t grid = b.total_blocks;
    if (grid == 0 || b.nsims == 0)
        return hipSuccess;
    switch (ph) {
    case PH_BIN:
        if (dim == 2) {
            if (prec == 0) bin_kb<2, double><<<grid, kBlock, 0, s>>>(b);
            else bin_kb<2, float><<<grid, kBlock, 0, s>>>(b);
        } else {
            if (prec == 0) bin_kb<3, double><<<grid, kBlock, 0, s>>>(b);
            else bin_kb<3, float><<<grid, kBlock, 0, s>>>(b);
        }
        break;
    case PH_SCAN_REDUCE: scan_reduce_kb<<<grid, kBlock, 0, s>>>(b); break;
    case PH_SCAN_TOP: scan_top_kb<<<grid, kBlock, 0, s>>>(b); break;
    case PH_SCAN_DOWN: scan_down_kb<<<grid, kBlock, 0, s>>>(b); break;
    case PH_SCATTER: scatter_kb<<<grid, kBlock, 0, s>>>(b); break;
    case PH_PLACE: MTPT_DISPATCH_D_PREC(place_kb, grid, kBlock, b); break;
    case PH_ROWSUM:
    case PH_TRANSFER:
        if (dim == 2)
            return tn ? launch_tiles<2, true>(ph, prec, ns, nullptr, &b, s)
                      : launch_tiles<2, false>(ph, prec, ns, nullptr, &b, s);
        return tn ? launch_tiles<3, true>(ph, prec, ns, nullptr, &b, s)
                  : launch_tiles<3, false>(ph, prec, ns, nullptr, &b, s);
    case PH_FINALIZE: finalize_kb<<<grid, kFinalBlock, 0, s>>>(b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_unpermute_mass(int prec, const SimArgs& a, const void* const* m_cur,
                                 const uint32_t* pid_cur, double* out, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = ceil_div(a.n, kBlock);
    if (prec == 2)
        unpermute_mass_k<float><<<grid, kBlock, 0, s>>>(a.n, a.ns, static_cast<const float*>(m_cur[0]),
                                                        static_cast<const float*>(m_cur[1]),
                                                        static_cast<const float*>(m_cur[2]), pid_cur, out);
    else
        unpermute_mass_k<double><<<grid, kBlock, 0, s>>>(a.n, a.ns, static_cast<const double*>(m_cur[0]),
                                                         static_cast<const double*>(m_cur[1]),
                                                         static_cast<const double*>(m_cur[2]), pid_cur, out);
    return hipGetLastError();
}

hipError_t launch_unpermute_pos(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                                double* out, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = ceil_div(a.n, kBlock);
    if (prec == 0) {
        const double* x[3] = {static_cast<const double*>(a.x[0]), static_cast<const double*>(a.x[1]),
                              static_cast<const double*>(a.x[2])};
        if (dim == 2) unpermute_pos_k<2, double><<<grid, kBlock, 0, s>>>(a.n, x[0], x[1], x[2], pid_cur, out);
        else unpermute_pos_k<3, double><<<grid, kBlock, 0, s>>>(a.n, x[0], x[1], x[2], pid_cur, out);
    } else {
        const float* x[3] = {static_cast<const float*>(a.x[0]), static_cast<const float*>(a.x[1]),
                             static_cast<const float*>(a.x[2])};
        if (dim == 2) unpermute_pos_k<2, float><<<grid, kBlock, 0, s>>>(a.n, x[0], x[1], x[2], pid_cur, out);
        else unpermute_pos_k<3, float><<<grid, kBlock, 0, s>>>(a.n, x[0], x[1], x[2], pid_cur, out);
    }
    return hipGetLastError();
}

hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s)
{
    if (n > 0)
        iota_k<<<ceil_div(n, kBlock), kBlock, 0, s>>>(out, n);
    return hipGetLastError();
}

hipError_t launch_totals(int prec, const SimArgs& a, const void* const* m_cur, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = a.part_blocks;
    if (prec == 2)
        totals_k<float><<<grid, kBlock, 0, s>>>(a, static_cast<const float*>(m_cur[0]),
                                                static_cast<const float*>(m_cur[1]),
                                                static_cast<const float*>(m_cur[2]));
    else
        totals_k<double><<<grid, kBlock, 0, s>>>(a, static_cast<const double*>(m_cur[0]),
                                                 static_cast<const double*>(m_cur[1]),
                                                 static_cast<const double*>(m_cur[2]));
    finalize_k<<<1, kFinalBlock, 0, s>>>(a, grid, 1);
    return hipGetLastError();
}

#define MTPT_DISPATCH_NB(KERNEL, ...)                                                            \
    do {                                                                                         \
        const bool tn = a.tensor != 0;                                                           \
        if (dim == 2) {                                                                          \
            if (prec == 0) { if (tn) KERNEL<2, 0, true><<<grid, kBlock, 0, s>>>(__VA_ARGS__);     \
                             else KERNEL<2, 0, false><<<grid, kBlock, 0, s>>>(__VA_ARGS__); }     \
            else if (prec == 1) { if (tn) KERNEL<2, 1, true><<<grid, kBlock, 0, s>>>(__VA_ARGS__);\
                                  else KERNEL<2, 1, false><<<grid, kBlock, 0, s>>>(__VA_ARGS__); }\
            else { if (tn) KERNEL<2, 2, true><<<grid, kBlock, 0, s>>>(__VA_ARGS__);               \
                   else KERNEL<2, 2, false><<<grid, kBlock, 0, s>>>(__VA_ARGS__); }               \
        } else {                                                                                 \
            if (prec == 0) { if (tn) KERNEL<3, 0, true><<<grid, kBlock, 0, s>>>(__VA_ARGS__);     \
                             else KERNEL<3, 0, false><<<grid, kBlock, 0, s>>>(__VA_ARGS__); }     \
            else if (prec == 1) { if (tn) KERNEL<3, 1, true><<<grid, kBlock, 0, s>>>(__VA_ARGS__);\
                                  else KERNEL<3, 1, false><<<grid, kBlock, 0, s>>>(__VA_ARGS__); }\
            else { if (tn) KERNEL<3, 2, true><<<grid, kBlock, 0, s>>>(__VA_ARGS__);               \
                   else KERNEL<3, 2, false><<<grid, kBlock, 0, s>>>(__VA_ARGS__); }               \
        }                                                                                        \
    } while (0)

hipError_t launch_nb_count(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                           uint32_t* rowcnt, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = ceil_div(a.n, kBlock);
    MTPT_DISPATCH_NB(nb_count_k, a, pid_cur, rowcnt);
    return hipGetLastError();
}

hipError_t launch_nb_fill(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                          const int64_t* row_ptr, int64_t* col, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = ceil_div(a.n, kBlock);
    MTPT_DISPATCH_NB(nb_fill_k, a, pid_cur, row_ptr, col);
    return hipGetLastError();
}
#undef MTPT_DISPATCH_NB

hipError_t launch_nb_sort(int64_t n, const int64_t* row_ptr, int64_t* col, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    nb_sort_k<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, row_ptr, col);
    return hipGetLastError();
}

// tmp must hold ceil((len+1)/kScanTile)*kScanTile u32 values, bsum
// ceil((len+1)/kScanTile) values.  The result out[0..len] is exclusive.
hipError_t launch_scan_u32_to_i64(const uint32_t* in, int64_t* out, int64_t len, uint32_t* tmp,
                                  uint32_t* bsum, hipStream_t s)
{
    const int64_t tiles = (len + 1 + kScanTile - 1) / kScanTile;
    const int64_t padded = tiles * kScanTile;
    copy_pad_k<<<ceil_div(padded, kBlock), kBlock, 0, s>>>(in, tmp, len, padded);
    scan_reduce_raw_k<<<static_cast<uint32_t>(tiles), kBlock, 0, s>>>(tmp, bsum);
    scan_top_raw_k<<<1, kBlock, 0, s>>>(bsum, static_cast<uint32_t>(tiles));
    scan_down_raw_k<<<static_cast<uint32_t>(tiles), kBlock, 0, s>>>(tmp, tmp, bsum);
    widen_k<<<ceil_div(len + 1, kBlock), kBlock, 0, s>>>(tmp, out, len);
    return hipGetLastError();
}

}  // namespace mtpt
