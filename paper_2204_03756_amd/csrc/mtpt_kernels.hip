// mtpt_kernels.hip -- HIP kernels of the MTPT step for gfx950 (wave64).
//
// One step of the method (Schauer et al., arXiv 2204.03756, Sec. 3) runs as:
//   bin        random walk + reflection (Sec. 3 random-walk update, zero-flux
//              walls), cell id of the walked position, cell histogram
//   scan       exclusive scan of the histogram -> cell offsets
//   scatter    slot of every particle inside its cell
//   cellsort   order inside every cell by pid (makes the layout, and with it
//              every floating-point sum, independent of atomic order)
//   gather     positions, masses and pids into the new sorted order
//   rowsum     s_i = sum_j K_ij over the 3^d neighbouring cells, K_ii = 1 included
//              (Eq. (2)-(3) without the prefactor, which cancels in W)
//   transfer   W_ij = 2 K_ij / (s_i + s_j), M_i' = M_i + beta sum_j W_ij (M_j - M_i)
//              (Eq. (4)-(5)), optional A+B->C epilogue, per-block mass sums and
//              the final FP64 totals in the last block to finish
// The K-D tree of the paper is replaced by the cell list: with cell side >=
// psi every neighbour within psi lies in the 3^d cells around a particle, and
// since cells are numbered x-fastest, the three cells of one (y, z) row are
// one contiguous range of the sorted arrays.
#include "mtpt_kernels.h"
#include "mtpt_rng.h"

#include <math.h>

namespace mtpt {

// ------------------------------------------------------------------ basics
template <int PREC> struct Types;
template <> struct Types<0> { using T = double; using M = double; using A = double; };
template <> struct Types<1> { using T = float;  using M = double; using A = double; };
template <> struct Types<2> { using T = float;  using M = float;  using A = float;  };

__device__ __forceinline__ int cell_coord(double x, double glo, double inv, int nc)
{
#pragma clang fp contract(off)
    int c = static_cast<int>((x - glo) * inv);
    c = c < 0 ? 0 : c;
    return c > nc - 1 ? nc - 1 : c;
}

template <int D>
__device__ __forceinline__ double r2_canonical(const double* xi, const double* xj)
{
#pragma clang fp contract(off)
    const double d0 = xj[0] - xi[0];
    const double d1 = xj[1] - xi[1];
    double r2 = d0 * d0 + d1 * d1;
    if (D == 3) {
        const double d2 = xj[2] - xi[2];
        r2 = r2 + d2 * d2;
    }
    return r2;
}

// Inside test and squared distance for the arithmetic of the path.  FP64:
// the canonical r^2 against psi^2.  FP32: the FP32 r^2 decides outside a
// 1e-5 relative band around psi^2; inside it the canonical FP64 r^2 of the
// same FP32 positions decides (FP32 r^2 error is below 1e-6 relative).
template <int D, typename T> struct Pair;

template <int D> struct Pair<D, double> {
    __device__ __forceinline__ static bool inside(const SimArgs& a, const double* xi,
                                                  const double* xj, double* r2o)
    {
        const double r2 = r2_canonical<D>(xi, xj);
        *r2o = r2;
        return r2 <= a.psi2;
    }
    __device__ __forceinline__ static double kernel(const SimArgs& a, double r2)
    {
        return exp(-a.kc * r2);
    }
};

template <int D> struct Pair<D, float> {
    __device__ __forceinline__ static bool inside(const SimArgs& a, const float* xi,
                                                  const float* xj, float* r2o)
    {
        const float d0 = xj[0] - xi[0];
        const float d1 = xj[1] - xi[1];
        float r2 = d0 * d0 + d1 * d1;
        if (D == 3) {
            const float d2 = xj[2] - xi[2];
            r2 = r2 + d2 * d2;
        }
        *r2o = r2;
        if (r2 < a.psi2_in)
            return true;
        if (r2 > a.psi2_out)
            return false;
        double pi[3], pj[3];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            pi[k] = static_cast<double>(xi[k]);
            pj[k] = static_cast<double>(xj[k]);
        }
        return r2_canonical<D>(pi, pj) <= a.psi2;
    }
    __device__ __forceinline__ static float kernel(const SimArgs& a, float r2)
    {
        return __expf(-a.kcf * r2);
    }
};

template <typename T>
__device__ __forceinline__ T walk_reflect(T x, double z, double sdev, double lo, double hi,
                                          float lof, float hif);

template <>
__device__ __forceinline__ double walk_reflect<double>(double x, double z, double sdev, double lo,
                                                       double hi, float, float)
{
#pragma clang fp contract(off)
    const double jump = z * sdev;
    double v = x + jump;
    while (v < lo || v > hi)
        v = (v < lo) ? 2.0 * lo - v : 2.0 * hi - v;
    return v;
}

template <>
__device__ __forceinline__ float walk_reflect<float>(float x, double z, double sdev, double, double,
                                                     float lof, float hif)
{
#pragma clang fp contract(off)
    const double jump = z * sdev;
    const float jf = static_cast<float>(jump);
    float v = x + jf;
    while (v < lof || v > hif)
        v = (v < lof) ? 2.0f * lof - v : 2.0f * hif - v;
    return v;
}

// wave64 inclusive scan and block (4 waves) exclusive scan
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off)
            v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63)
        wsum[wid] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        base += (w < wid) ? wsum[w] : 0u;
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

template <typename V>
__device__ __forceinline__ V block_sum(V v)
{
    __shared__ V red[kBlock / 64];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_down(v, off, 64);
    if (lane == 0)
        red[wid] = v;
    __syncthreads();
    V t = V(0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w)
            t += red[w];
    }
    __syncthreads();
    return t;  // valid in thread 0
}

// -------------------------------------------------------------- phase bodies
template <int D, typename T>
__device__ __forceinline__ void bin_body(const SimArgs& a, uint32_t blk)
{
    const int64_t i = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    if (i >= a.n)
        return;
    T v[3];
#pragma unroll
    for (int k = 0; k < D; ++k)
        v[k] = static_cast<const T*>(a.x[k])[i];
    if (a.walk) {
        const uint32_t pid = a.pid_src[i];
        double z[3], spare;
        normal_pair(a.seed, a.step, pid, 0u, &z[0], &z[1]);
        if (D == 3)
            normal_pair(a.seed, a.step, pid, 1u, &z[2], &spare);
#pragma unroll
        for (int k = 0; k < D; ++k)
            v[k] = walk_reflect<T>(v[k], z[k], a.sdev, a.lo[k], a.hi[k], a.lof[k], a.hif[k]);
    }
    uint32_t c = 0;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        static_cast<T*>(a.xt[k])[i] = v[k];
        c = c * static_cast<uint32_t>(a.nc[k]) +
            static_cast<uint32_t>(cell_coord(static_cast<double>(v[k]), a.glo[k], a.inv_side[k], a.nc[k]));
    }
    a.cell[i] = c;
    a.rank[i] = atomicAdd(&a.counts[c], 1u);
}

__device__ __forceinline__ void scan_reduce_body(const uint32_t* in, uint32_t* bsum, uint32_t blk)
{
    const uint4* p = reinterpret_cast<const uint4*>(in + static_cast<size_t>(blk) * kScanTile +
                                                    threadIdx.x * kScanItems);
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
        const uint4 w = p[q];
        s += w.x + w.y + w.z + w.w;
    }
    const uint32_t t = block_sum<uint32_t>(s);
    if (threadIdx.x == 0)
        bsum[blk] = t;
}

__device__ __forceinline__ void scan_top_body(uint32_t* bsum, uint32_t nb)
{
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kBlock) {
        const uint32_t idx = base + threadIdx.x;
        const uint32_t v = idx < nb ? bsum[idx] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot);
        if (idx < nb)
            bsum[idx] = carry + ex;
        carry += tot;
    }
}

__device__ __forceinline__ void scan_down_body(uint32_t* in, uint32_t* out, const uint32_t* bsum,
                                               uint32_t blk, bool zero_in)
{
    const size_t base = static_cast<size_t>(blk) * kScanTile + threadIdx.x * kScanItems;
    uint4* p = reinterpret_cast<uint4*>(in + base);
    uint32_t v[kScanItems];
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
        const uint4 w = p[q];
        v[4 * q + 0] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t t = v[k];
        v[k] = s;
        s += t;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(s, &tot) + bsum[blk];
    uint4* o = reinterpret_cast<uint4*>(out + base);
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q)
        o[q] = make_uint4(ex + v[4 * q], ex + v[4 * q + 1], ex + v[4 * q + 2], ex + v[4 * q + 3]);
    if (zero_in) {
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q)
            p[q] = make_uint4(0u, 0u, 0u, 0u);
    }
}

__device__ __forceinline__ void scatter_body(const SimArgs& a, uint32_t blk)
{
    const int64_t i = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    if (i >= a.n)
        return;
    a.perm[a.starts[a.cell[i]] + a.rank[i]] = static_cast<uint32_t>(i);
}

__device__ __forceinline__ void cellsort_body(const SimArgs& a, uint32_t blk)
{
    const int64_t c = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    if (c >= a.ncells)
        return;
    const uint32_t b = a.starts[c], e = a.starts[c + 1];
    for (uint32_t k = b + 1; k < e; ++k) {
        const uint32_t v = a.perm[k];
        const uint32_t key = a.pid_src[v];
        uint32_t j = k;
        while (j > b) {
            const uint32_t u = a.perm[j - 1];
            if (a.pid_src[u] <= key)
                break;
            a.perm[j] = u;
            --j;
        }
        a.perm[j] = v;
    }
}

template <int D, typename T, typename M>
__device__ __forceinline__ void gather_body(const SimArgs& a, uint32_t blk)
{
    const int64_t k = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    if (k >= a.n)
        return;
    const uint32_t src = a.perm[k];
#pragma unroll
    for (int d = 0; d < D; ++d)
        static_cast<T*>(a.x[d])[k] = static_cast<const T*>(a.xt[d])[src];
    for (int c = 0; c < a.ns; ++c)
        static_cast<M*>(a.m_mid[c])[k] = static_cast<const M*>(a.m_src[c])[src];
    a.pid_dst[k] = a.pid_src[src];
}

// The neighbour rows of particle i: for each (dy, dz), the contiguous slot
// range of cells cx-1 .. cx+1 of that row.  f(j) is called for every
// candidate slot in a fixed order (z, then y, then slot).
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

template <int D, int PREC>
__device__ __forceinline__ void rowsum_body(const SimArgs& a, uint32_t blk)
{
    using T = typename Types<PREC>::T;
    const int64_t i = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    uint32_t pairs = 0;
    if (i < a.n) {
        T xi[3];
#pragma unroll
        for (int k = 0; k < D; ++k)
            xi[k] = static_cast<const T*>(a.x[k])[i];
        T acc = T(0);
        uint32_t cnt = 0;
        for_candidates<D, T>(a, xi, [&](uint32_t j) {
            T xj[3];
#pragma unroll
            for (int k = 0; k < D; ++k)
                xj[k] = static_cast<const T*>(a.x[k])[j];
            T r2;
            if (Pair<D, T>::inside(a, xi, xj, &r2)) {
                acc += Pair<D, T>::kernel(a, r2);
                ++cnt;
            }
        });
        static_cast<T*>(a.srow)[i] = acc;
        pairs = cnt - 1u;
    }
    const unsigned long long tot = block_sum<unsigned long long>(pairs);
    if (threadIdx.x == 0 && tot)
        atomicAdd(&a.st->pairs_acc, tot);
}

// A+B->C inside one particle over dt, exact solution of da/dt = db/dt = -k a b
// on concentrations (c = N M / V): with D = a - b >= 0,
// a' = a D / (D - b expm1(-k D dt)), or a/(1 + k a dt) when D = 0; b' = a' - D.
__device__ __forceinline__ void react3(double* m, const SimArgs& a)
{
    double ca = m[0] * a.to_c, cb = m[1] * a.to_c;
    const bool sw = cb > ca;
    if (sw) {
        const double t = ca;
        ca = cb;
        cb = t;
    }
    const double d = ca - cb;
    const double an = d > 0.0 ? ca * d / (d - cb * expm1(-a.k_react * d * a.dt))
                              : ca / (1.0 + a.k_react * ca * a.dt);
    const double bn = an - d;
    const double reacted = ca - an;
    m[0] = (sw ? bn : an) * a.to_m;
    m[1] = (sw ? an : bn) * a.to_m;
    m[2] = m[2] + reacted * a.to_m;
}

template <int D, int PREC, int NS>
__device__ __forceinline__ void transfer_body(const SimArgs& a, uint32_t blk)
{
    using T = typename Types<PREC>::T;
    using M = typename Types<PREC>::M;
    using A = typename Types<PREC>::A;
    const int64_t i = static_cast<int64_t>(blk) * kBlock + threadIdx.x;
    double outv[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c)
        outv[c] = 0.0;
    if (i < a.n) {
        T xi[3];
#pragma unroll
        for (int k = 0; k < D; ++k)
            xi[k] = static_cast<const T*>(a.x[k])[i];
        const T si = static_cast<const T*>(a.srow)[i];
        M mi[NS];
        A dl[NS], comp[NS];
#pragma unroll
        for (int c = 0; c < NS; ++c) {
            mi[c] = static_cast<const M*>(a.m_mid[c])[i];
            dl[c] = A(0);
            comp[c] = A(0);
        }
        const uint32_t self = static_cast<uint32_t>(i);
        for_candidates<D, T>(a, xi, [&](uint32_t j) {
            if (j == self)
                return;
            T xj[3];
#pragma unroll
            for (int k = 0; k < D; ++k)
                xj[k] = static_cast<const T*>(a.x[k])[j];
            T r2;
            if (!Pair<D, T>::inside(a, xi, xj, &r2))
                return;
            const T kv = Pair<D, T>::kernel(a, r2);
            const T sj = static_cast<const T*>(a.srow)[j];
            const T w = (kv + kv) / (si + sj);
#pragma unroll
            for (int c = 0; c < NS; ++c) {
                const M mj = static_cast<const M*>(a.m_mid[c])[j];
                if (PREC == 2) {
                    // Kahan-compensated FP32 accumulation
                    const A y = static_cast<A>(w) * static_cast<A>(mj - mi[c]) - comp[c];
                    const A t = dl[c] + y;
                    comp[c] = (t - dl[c]) - y;
                    dl[c] = t;
                } else {
                    dl[c] += static_cast<A>(w) * static_cast<A>(mj - mi[c]);
                }
            }
        });
        double mo[3];
#pragma unroll
        for (int c = 0; c < NS; ++c) {
            if (PREC == 2) {
                const float nv = mi[c] + a.betaf * dl[c];
                mo[c] = static_cast<double>(nv);
            } else {
                mo[c] = static_cast<double>(mi[c]) + a.beta * static_cast<double>(dl[c]);
            }
        }
        if (NS == 3 && a.k_react > 0.0)
            react3(mo, a);
#pragma unroll
        for (int c = 0; c < NS; ++c) {
            const M st = static_cast<M>(mo[c]);
            static_cast<M*>(a.m_dst[c])[i] = st;
            outv[c] = static_cast<double>(st);
        }
    }
    // per-block mass sums, fixed order
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        const double t = block_sum<double>(outv[c]);
        if (threadIdx.x == 0)
            a.partials[static_cast<size_t>(blk) * NS + c] = t;
    }
    __shared__ int last;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(&a.st->blocks_done, 1u);
        last = (prev == a.part_blocks - 1u);
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    const volatile double* part = a.partials;
#pragma unroll
    for (int c = 0; c < NS; ++c) {
        double s = 0.0;
        for (uint32_t b = threadIdx.x; b < a.part_blocks; b += kBlock)
            s += part[static_cast<size_t>(b) * NS + c];
        const double t = block_sum<double>(s);
        if (threadIdx.x == 0) {
            a.st->totals[c] = t;
            if (!isfinite(t))
                a.st->nonfinite = 1;
        }
    }
    if (threadIdx.x == 0) {
        DevStats* st = a.st;
        if (a.recompute_s) {
            st->pairs_last = st->pairs_acc;
            st->pairs_acc = 0ull;
        }
        st->pairs_total += st->pairs_last;
        st->steps += 1;
        st->blocks_done = 0u;
        __threadfence();
    }
}

// ---------------------------------------------------------------- kernels
__device__ __forceinline__ int find_sim(const Batch& b, uint32_t blk, uint32_t* local)
{
    int lo = 0, hi = b.nsims - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.blk_off[mid] <= blk)
            lo = mid;
        else
            hi = mid - 1;
    }
    *local = blk - b.blk_off[lo];
    return lo;
}

template <int D, typename T>
__global__ __launch_bounds__(kBlock) void bin_k(SimArgs a) { bin_body<D, T>(a, blockIdx.x); }
template <int D, typename T>
__global__ __launch_bounds__(kBlock) void bin_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    bin_body<D, T>(a, l);
}

__global__ __launch_bounds__(kBlock) void scan_reduce_k(SimArgs a) { scan_reduce_body(a.counts, a.bsum, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void scan_reduce_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    scan_reduce_body(a.counts, a.bsum, l);
}
__global__ __launch_bounds__(kBlock) void scan_top_k(SimArgs a) { scan_top_body(a.bsum, a.scan_blocks); }
__global__ __launch_bounds__(kBlock) void scan_top_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    scan_top_body(a.bsum, a.scan_blocks);
}
__global__ __launch_bounds__(kBlock) void scan_down_k(SimArgs a) { scan_down_body(a.counts, a.starts, a.bsum, blockIdx.x, true); }
__global__ __launch_bounds__(kBlock) void scan_down_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    scan_down_body(a.counts, a.starts, a.bsum, l, true);
}

__global__ __launch_bounds__(kBlock) void scatter_k(SimArgs a) { scatter_body(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void scatter_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    scatter_body(a, l);
}
__global__ __launch_bounds__(kBlock) void cellsort_k(SimArgs a) { cellsort_body(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void cellsort_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    cellsort_body(a, l);
}

template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void gather_k(SimArgs a)
{
    gather_body<D, typename Types<PREC>::T, typename Types<PREC>::M>(a, blockIdx.x);
}
template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void gather_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    gather_body<D, typename Types<PREC>::T, typename Types<PREC>::M>(a, l);
}

template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void rowsum_k(SimArgs a) { rowsum_body<D, PREC>(a, blockIdx.x); }
template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void rowsum_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    rowsum_body<D, PREC>(a, l);
}

template <int D, int PREC, int NS>
__global__ __launch_bounds__(kBlock) void transfer_k(SimArgs a) { transfer_body<D, PREC, NS>(a, blockIdx.x); }
template <int D, int PREC, int NS>
__global__ __launch_bounds__(kBlock) void transfer_kb(Batch b)
{
    uint32_t l;
    const SimArgs& a = b.args[find_sim(b, blockIdx.x, &l)];
    transfer_body<D, PREC, NS>(a, l);
}

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

// totals of the current masses: per-block sums, then the last block sums
// them in block order (same scheme as the transfer pass)
template <typename M>
__global__ __launch_bounds__(kBlock) void totals_k(SimArgs a, const M* m0, const M* m1, const M* m2)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const M* ms[3] = {m0, m1, m2};
    for (int c = 0; c < a.ns; ++c) {
        const double v = i < a.n ? static_cast<double>(ms[c][i]) : 0.0;
        const double t = block_sum<double>(v);
        if (threadIdx.x == 0)
            a.partials[static_cast<size_t>(blockIdx.x) * a.ns + c] = t;
    }
    __shared__ int last;
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(&a.st->blocks_done, 1u);
        last = (prev == a.part_blocks - 1u);
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    const volatile double* part = a.partials;
    for (int c = 0; c < a.ns; ++c) {
        double s = 0.0;
        for (uint32_t b = threadIdx.x; b < a.part_blocks; b += kBlock)
            s += part[static_cast<size_t>(b) * a.ns + c];
        const double t = block_sum<double>(s);
        if (threadIdx.x == 0) {
            a.st->totals[c] = t;
            if (!isfinite(t))
                a.st->nonfinite = 1;
        }
    }
    if (threadIdx.x == 0)
        a.st->blocks_done = 0u;
}

template <int D, int PREC>
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
        if (Pair<D, T>::inside(a, xi, xj, &r2))
            ++cnt;
    });
    rowcnt[pid[i]] = cnt;
}

template <int D, int PREC>
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
        if (Pair<D, T>::inside(a, xi, xj, &r2))
            col[base + cnt++] = static_cast<int64_t>(pid[j]);
    });
    // ascending pid inside the row
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

// exclusive scan of n u32 counts into int64 offsets (n+1 values): the
// counts are copied into a tile-padded buffer, scanned like the histogram,
// and widened
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
__global__ __launch_bounds__(kBlock) void scan_reduce_raw_k(const uint32_t* in, uint32_t* bsum) { scan_reduce_body(in, bsum, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void scan_top_raw_k(uint32_t* bsum, uint32_t nb) { scan_top_body(bsum, nb); }
__global__ __launch_bounds__(kBlock) void scan_down_raw_k(uint32_t* in, uint32_t* out, const uint32_t* bsum)
{
    scan_down_body(in, out, bsum, blockIdx.x, false);
}

// ------------------------------------------------------------- host side
const char* phase_name(int ph)
{
    static const char* names[PH_COUNT] = {"bin", "scan_reduce", "scan_top", "scan_down", "scatter",
                                          "cellsort", "gather", "rowsum", "transfer"};
    return (ph >= 0 && ph < PH_COUNT) ? names[ph] : "?";
}

static uint32_t ceil_div(int64_t a, int64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

uint32_t phase_blocks(int ph, const SimArgs& a)
{
    switch (ph) {
    case PH_SCAN_REDUCE:
    case PH_SCAN_DOWN: return a.scan_blocks;
    case PH_SCAN_TOP: return 1;
    case PH_CELLSORT: return ceil_div(a.ncells, kBlock);
    default: return a.n > 0 ? ceil_div(a.n, kBlock) : 0;
    }
}

#define MTPT_DISPATCH_D_PREC(KERNEL, GRID, ARG)                                                  \
    do {                                                                                         \
        if (dim == 2) {                                                                          \
            if (prec == 0) KERNEL<2, 0><<<GRID, kBlock, 0, s>>>(ARG);                            \
            else if (prec == 1) KERNEL<2, 1><<<GRID, kBlock, 0, s>>>(ARG);                       \
            else KERNEL<2, 2><<<GRID, kBlock, 0, s>>>(ARG);                                      \
        } else {                                                                                 \
            if (prec == 0) KERNEL<3, 0><<<GRID, kBlock, 0, s>>>(ARG);                            \
            else if (prec == 1) KERNEL<3, 1><<<GRID, kBlock, 0, s>>>(ARG);                       \
            else KERNEL<3, 2><<<GRID, kBlock, 0, s>>>(ARG);                                      \
        }                                                                                        \
    } while (0)

#define MTPT_DISPATCH_D_PREC_NS(KERNEL, GRID, ARG)                                               \
    do {                                                                                         \
        if (ns == 1) {                                                                           \
            if (dim == 2) {                                                                      \
                if (prec == 0) KERNEL<2, 0, 1><<<GRID, kBlock, 0, s>>>(ARG);                     \
                else if (prec == 1) KERNEL<2, 1, 1><<<GRID, kBlock, 0, s>>>(ARG);                \
                else KERNEL<2, 2, 1><<<GRID, kBlock, 0, s>>>(ARG);                               \
            } else {                                                                             \
                if (prec == 0) KERNEL<3, 0, 1><<<GRID, kBlock, 0, s>>>(ARG);                     \
                else if (prec == 1) KERNEL<3, 1, 1><<<GRID, kBlock, 0, s>>>(ARG);                \
                else KERNEL<3, 2, 1><<<GRID, kBlock, 0, s>>>(ARG);                               \
            }                                                                                    \
        } else {                                                                                 \
            if (dim == 2) {                                                                      \
                if (prec == 0) KERNEL<2, 0, 3><<<GRID, kBlock, 0, s>>>(ARG);                     \
                else if (prec == 1) KERNEL<2, 1, 3><<<GRID, kBlock, 0, s>>>(ARG);                \
                else KERNEL<2, 2, 3><<<GRID, kBlock, 0, s>>>(ARG);                               \
            } else {                                                                             \
                if (prec == 0) KERNEL<3, 0, 3><<<GRID, kBlock, 0, s>>>(ARG);                     \
                else if (prec == 1) KERNEL<3, 1, 3><<<GRID, kBlock, 0, s>>>(ARG);                \
                else KERNEL<3, 2, 3><<<GRID, kBlock, 0, s>>>(ARG);                               \
            }                                                                                    \
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
    case PH_CELLSORT: cellsort_k<<<grid, kBlock, 0, s>>>(a); break;
    case PH_GATHER: MTPT_DISPATCH_D_PREC(gather_k, grid, a); break;
    case PH_ROWSUM: MTPT_DISPATCH_D_PREC(rowsum_k, grid, a); break;
    case PH_TRANSFER: MTPT_DISPATCH_D_PREC_NS(transfer_k, grid, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_phase_batched(int ph, int dim, int prec, int ns, const Batch& b, hipStream_t s)
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
    case PH_CELLSORT: cellsort_kb<<<grid, kBlock, 0, s>>>(b); break;
    case PH_GATHER: MTPT_DISPATCH_D_PREC(gather_kb, grid, b); break;
    case PH_ROWSUM: MTPT_DISPATCH_D_PREC(rowsum_kb, grid, b); break;
    case PH_TRANSFER: MTPT_DISPATCH_D_PREC_NS(transfer_kb, grid, b); break;
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
    return hipGetLastError();
}

hipError_t launch_nb_count(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                           uint32_t* rowcnt, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = ceil_div(a.n, kBlock);
    if (dim == 2) {
        if (prec == 0) nb_count_k<2, 0><<<grid, kBlock, 0, s>>>(a, pid_cur, rowcnt);
        else if (prec == 1) nb_count_k<2, 1><<<grid, kBlock, 0, s>>>(a, pid_cur, rowcnt);
        else nb_count_k<2, 2><<<grid, kBlock, 0, s>>>(a, pid_cur, rowcnt);
    } else {
        if (prec == 0) nb_count_k<3, 0><<<grid, kBlock, 0, s>>>(a, pid_cur, rowcnt);
        else if (prec == 1) nb_count_k<3, 1><<<grid, kBlock, 0, s>>>(a, pid_cur, rowcnt);
        else nb_count_k<3, 2><<<grid, kBlock, 0, s>>>(a, pid_cur, rowcnt);
    }
    return hipGetLastError();
}

hipError_t launch_nb_fill(int dim, int prec, const SimArgs& a, const uint32_t* pid_cur,
                          const int64_t* row_ptr, int64_t* col, hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    const uint32_t grid = ceil_div(a.n, kBlock);
    if (dim == 2) {
        if (prec == 0) nb_fill_k<2, 0><<<grid, kBlock, 0, s>>>(a, pid_cur, row_ptr, col);
        else if (prec == 1) nb_fill_k<2, 1><<<grid, kBlock, 0, s>>>(a, pid_cur, row_ptr, col);
        else nb_fill_k<2, 2><<<grid, kBlock, 0, s>>>(a, pid_cur, row_ptr, col);
    } else {
        if (prec == 0) nb_fill_k<3, 0><<<grid, kBlock, 0, s>>>(a, pid_cur, row_ptr, col);
        else if (prec == 1) nb_fill_k<3, 1><<<grid, kBlock, 0, s>>>(a, pid_cur, row_ptr, col);
        else nb_fill_k<3, 2><<<grid, kBlock, 0, s>>>(a, pid_cur, row_ptr, col);
    }
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
