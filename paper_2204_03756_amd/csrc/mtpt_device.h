// mtpt_device.h -- device code of the MTPT step for gfx950 (wave64): the
// helpers, the phase bodies and the tiled mass-transfer kernels, shared by
// the translation units that instantiate them (mtpt_kernels.hip: binning,
// exports and the host launchers; mtpt_tiles_*.hip: the two tiled passes per
// dimension and metric, compiled in parallel).
//
// One step of the method (Schauer et al., arXiv 2204.03756, Sec. 3) runs as:
//   bin        random walk + reflection (Sec. 3 random-walk update, zero-flux
//              walls), cell id of the walked position, cell histogram
//   scan       exclusive scan of the histogram -> cell offsets
//   scatter    slot of every particle inside its cell
//   place      rank inside the cell by (x, pid), gather positions, masses and
//              pids into that slot: the layout, and with it every
//              floating-point sum, does not depend on the order of atomics
//   rowsum     s_i = sum_j K_ij, K_ii = 1 included (Eq. (2)-(3) without the
//              prefactor, which cancels in W)
//   transfer   W_ij = 2 K_ij / (s_i + s_j), M_i' = M_i + beta sum_j W_ij (M_j - M_i)
//              (Eq. (4)-(5)), optional A+B->C epilogue, per-workgroup mass sums
//   finalize   FP64 totals and pair counters, summed in a fixed order
// The K-D tree search of the paper is replaced by the cell list (cell side
// >= the cutoff's reach along each axis).  The two mass-transfer passes run
// per tile of cells: the workgroup stages the positions (and row sums) of
// every cell row of the tile and its one-cell halo in LDS -- each such row is
// one contiguous, x-sorted run of the sorted arrays -- and every particle
// scans its 3^(d-1) neighbouring rows (trimmed to its x-window where rows are
// long).  With a dispersion tensor the distance is the Mahalanobis form
// q = |M dx|^2 (M = L^-1, T = L L^T), the cutoff an ellipsoid.
#pragma once
#include "mtpt_kernels.h"
#include "mtpt_rng.h"

#include <math.h>

namespace mtpt {

// ------------------------------------------------------------------ basics
template <int PREC> struct Types;
template <> struct Types<0> { using T = double; using M = double; using A = double; };
template <> struct Types<1> { using T = float;  using M = double; using A = double; };
template <> struct Types<2> { using T = float;  using M = float;  using A = float;  };

// Particles a tile (cells plus halo) can stage in LDS: positions, and for the
// transfer pass also row sums and masses.  The row-sum pass (one
// instantiation for every species count) takes the capacity of the
// one-species transfer pass, so that it needs no more LDS than its tiles use
// (it stages positions only); each pass has its own tile plan.
template <int D, int PREC, int NS, bool TRANSFER> struct TileCap {
    using T = typename Types<PREC>::T;
    using M = typename Types<PREC>::M;
    static constexpr int bytes = D * static_cast<int>(sizeof(T)) + static_cast<int>(sizeof(T) + NS * sizeof(M));
    static constexpr int value = LdsBudget<D, PREC, NS>::value / bytes;
};

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

// Inside test and kernel value in the arithmetic of the path.  FP64: the
// canonical r^2 against psi^2.  FP32: the FP32 r^2 decides outside a 1e-5
// relative band around psi^2 (its error is below 1e-6 relative); inside the
// band the canonical FP64 r^2 of the same FP32 positions decides.
template <int D, typename T> struct Pair;

template <int D> struct Pair<D, double> {
    __device__ __forceinline__ static double r2(const double* xi, const double* xj)
    {
        return r2_canonical<D>(xi, xj);
    }
    __device__ __forceinline__ static bool inside(const SimArgs& a, const double* xi,
                                                  const double* xj, double* r2o)
    {
        const double r2 = r2_canonical<D>(xi, xj);
        *r2o = r2;
        return r2 <= a.psi2;
    }
    __device__ __forceinline__ static double kernel(const SimArgs& a, double r2) { return exp(-a.kc * r2); }
    __device__ __forceinline__ static double weight(double k, double si, double sj)
    {
        return (k + k) / (si + sj);
    }
};

template <int D> struct Pair<D, float> {
    // FP32 r^2 with a fixed contraction: fma(d0, d0, d1 d1) (+ fma(d2, d2, .))
    __device__ __forceinline__ static float r2(const float* xi, const float* xj)
    {
        const float d0 = xj[0] - xi[0];
        const float d1 = xj[1] - xi[1];
        float r = __builtin_fmaf(d0, d0, d1 * d1);
        if (D == 3) {
            const float d2 = xj[2] - xi[2];
            r = __builtin_fmaf(d2, d2, r);
        }
        return r;
    }
    __device__ __forceinline__ static bool inside(const SimArgs& a, const float* xi,
                                                  const float* xj, float* r2o)
    {
        const float r2 = Pair::r2(xi, xj);
        *r2o = r2;
        // below psi2_in inside for sure, above psi2_out outside; between the
        // two the FP64 test decides
        bool in = r2 <= a.psi2_out;
        if (__builtin_expect(in && r2 >= a.psi2_in, 0)) {
            double pi[3], pj[3];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                pi[k] = static_cast<double>(xi[k]);
                pj[k] = static_cast<double>(xj[k]);
            }
            in = r2_canonical<D>(pi, pj) <= a.psi2;
        }
        return in;
    }
    __device__ __forceinline__ static float kernel(const SimArgs& a, float r2)
    {
        return __builtin_amdgcn_exp2f(a.kcf2 * r2);
    }
    __device__ __forceinline__ static float weight(float k, float si, float sj)
    {
        return (k + k) * __builtin_amdgcn_rcpf(si + sj);
    }
};

// Distance in the cutoff's metric.  Isotropic (TN = false): the squared
// distance of Pair.  Tensor (TN = true): the Mahalanobis form q = |M dx|^2,
// M = L^-1 lower triangular, in FP64 in the canonical order
//   y0 = M00 d0, y1 = M10 d0 + M11 d1, y2 = (M20 d0 + M21 d1) + M22 d2,
//   q = (y0 y0 + y1 y1) + y2 y2   (no contraction),
// or in FP32 with fused multiply-adds; the FP32 q decides outside a relative
// band around psi^2 sized on the host from the tensor's conditioning, the
// canonical FP64 q of the same FP32 positions inside it.
template <int D>
__device__ __forceinline__ double q_canonical(const double* m, const double* xi, const double* xj)
{
#pragma clang fp contract(off)
    const double d0 = xj[0] - xi[0];
    const double d1 = xj[1] - xi[1];
    const double y0 = m[0] * d0;
    const double y1 = m[1] * d0 + m[2] * d1;
    double q = y0 * y0 + y1 * y1;
    if (D == 3) {
        const double d2 = xj[2] - xi[2];
        const double y2 = (m[3] * d0 + m[4] * d1) + m[5] * d2;
        q = q + y2 * y2;
    }
    return q;
}

template <int D, typename T, bool TN> struct Metric;

template <int D, typename T> struct Metric<D, T, false> {
    __device__ __forceinline__ static T r2(const SimArgs&, const T* xi, const T* xj)
    {
        return Pair<D, T>::r2(xi, xj);
    }
    __device__ __forceinline__ static bool inside(const SimArgs& a, const T* xi, const T* xj, T* r2o)
    {
        return Pair<D, T>::inside(a, xi, xj, r2o);
    }
};

template <int D> struct Metric<D, double, true> {
    __device__ __forceinline__ static double r2(const SimArgs& a, const double* xi, const double* xj)
    {
        return q_canonical<D>(a.minv, xi, xj);
    }
    __device__ __forceinline__ static bool inside(const SimArgs& a, const double* xi, const double* xj,
                                                  double* r2o)
    {
        const double q = q_canonical<D>(a.minv, xi, xj);
        *r2o = q;
        return q <= a.psi2;
    }
};

template <int D> struct Metric<D, float, true> {
    __device__ __forceinline__ static float r2(const SimArgs& a, const float* xi, const float* xj)
    {
        const float* m = a.minvf;
        const float d0 = xj[0] - xi[0];
        const float d1 = xj[1] - xi[1];
        const float y0 = m[0] * d0;
        const float y1 = __builtin_fmaf(m[2], d1, m[1] * d0);
        float q = __builtin_fmaf(y1, y1, y0 * y0);
        if (D == 3) {
            const float d2 = xj[2] - xi[2];
            const float y2 = __builtin_fmaf(m[5], d2, __builtin_fmaf(m[4], d1, m[3] * d0));
            q = __builtin_fmaf(y2, y2, q);
        }
        return q;
    }
    __device__ __forceinline__ static bool inside(const SimArgs& a, const float* xi, const float* xj, float* r2o)
    {
        const float q = r2(a, xi, xj);
        *r2o = q;
        bool in = q <= a.psi2_out;
        if (__builtin_expect(in && q >= a.psi2_in, 0)) {
            double pi[3], pj[3];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                pi[k] = static_cast<double>(xi[k]);
                pj[k] = static_cast<double>(xj[k]);
            }
            in = q_canonical<D>(a.minv, pi, pj) <= a.psi2;
        }
        return in;
    }
};

// The displacement of one coordinate in the type of the positions: the FP64
// z sdev + v dt (each operation rounded), rounded once more for FP32
// positions; then the position after the jump, reflected at the walls.
template <typename T>
__device__ __forceinline__ T jump_of(double z, double sdev, double drift)
{
#pragma clang fp contract(off)
    const double j = z * sdev + drift;
    return static_cast<T>(j);
}
template <typename T>
__device__ __forceinline__ T reflect_jump(T x, T jump, double lo, double hi, float lof, float hif);
template <>
__device__ __forceinline__ double reflect_jump<double>(double x, double jump, double lo, double hi, float, float)
{
#pragma clang fp contract(off)
    double v = x + jump;
    while (v < lo || v > hi)
        v = (v < lo) ? 2.0 * lo - v : 2.0 * hi - v;
    return v;
}
template <>
__device__ __forceinline__ float reflect_jump<float>(float x, float jump, double, double, float lof, float hif)
{
#pragma clang fp contract(off)
    float v = x + jump;
    while (v < lof || v > hif)
        v = (v < lof) ? 2.0f * lof - v : 2.0f * hif - v;
    return v;
}

// The D displacements of one particle from its standard normals z: with a
// dispersion tensor z is first replaced by u = L z (FP64, ascending column
// order, no contraction: u0 = L00 z0, u1 = L10 z0 + L11 z1,
// u2 = (L20 z0 + L21 z1) + L22 z2).
template <int D, typename T>
__device__ __forceinline__ void make_jumps(const SimArgs& a, const double* z, T* jv)
{
#pragma clang fp contract(off)
    double u[3] = {z[0], z[1], D == 3 ? z[2] : 0.0};
    if (a.tensor) {
        const double* l = a.lch;
        u[0] = l[0] * z[0];
        u[1] = l[1] * z[0] + l[2] * z[1];
        if (D == 3)
            u[2] = (l[3] * z[0] + l[4] * z[1]) + l[5] * z[2];
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
        jv[k] = jump_of<T>(u[k], a.sdev, a.drift[k]);
}

// x-window [x_i - win, x_i + win] in the type of the positions, rounded
// outward so that no x within the exact window falls outside it
template <typename T> struct Window;
template <> struct Window<double> {
    __device__ __forceinline__ static void make(double xi, double win, double* lo, double* hi)
    {
        *lo = xi - win;
        *hi = xi + win;
    }
};
// next float below / above a finite v
__device__ __forceinline__ float float_down(float v)
{
    const uint32_t b = __float_as_uint(v);
    if (v == 0.0f)
        return __uint_as_float(0x80000001u);
    return __uint_as_float(v > 0.0f ? b - 1u : b + 1u);
}
__device__ __forceinline__ float float_up(float v)
{
    const uint32_t b = __float_as_uint(v);
    if (v == 0.0f)
        return __uint_as_float(0x00000001u);
    return __uint_as_float(v > 0.0f ? b + 1u : b - 1u);
}

template <> struct Window<float> {
    __device__ __forceinline__ static void make(float xi, double win, float* lo, float* hi)
    {
        const double l = static_cast<double>(xi) - win;
        const double h = static_cast<double>(xi) + win;
        float lf = static_cast<float>(l);
        float hf = static_cast<float>(h);
        if (static_cast<double>(lf) > l)
            lf = float_down(lf);
        if (static_cast<double>(hf) < h)
            hf = float_up(hf);
        *lo = lf;
        *hi = hf;
    }
};

// v / d for 0 <= v < 4096 and 1 <= d <= 256, with inv = 1.0f / d: the exact
// quotient plus (v mod d + 0.5) / d lies at least 0.5 / d >= 2^-9 from an
// integer, and the FP32 product is off by less than 4096 * 2^-22 = 2^-10, so
// the truncation is exact (no integer divide sequence)
__device__ __forceinline__ int small_div(int v, float inv)
{
    return static_cast<int>((static_cast<float>(v) + 0.5f) * inv);
}

// Wave64 primitives on DPP lane moves (no LDS round trip).  Every lane of
// the wave must be active.
// one DPP move: lane value from the lane that dpp_ctrl selects, 0 where that
// lane is outside the row or the row is masked off
template <int Ctrl, int RowMask = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), Ctrl, RowMask, 0xF, true));
}

// inclusive scan over the 64 lanes: shifts by 1, 2, 4 and 8 inside each row
// of 16 lanes, then the last lane of row 0 (2) added to row 1 (3) and the
// last lane of row 1 added to rows 2 and 3
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += dpp_u32<0x111>(v);          // row_shr:1
    v += dpp_u32<0x112>(v);          // row_shr:2
    v += dpp_u32<0x114>(v);          // row_shr:4
    v += dpp_u32<0x118>(v);          // row_shr:8
    v += dpp_u32<0x142, 0xA>(v);     // row_bcast:15 into rows 1 and 3
    v += dpp_u32<0x143, 0xC>(v);     // row_bcast:31 into rows 2 and 3
    return v;
}

// maximum over the 64 lanes, wave-uniform: the maximum of every quad, then of
// every row (rotations by 4 and 8), then of the four rows' lanes 0
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, dpp_u32<0xB1>(v));    // quad_perm [1,0,3,2]
    v = max(v, dpp_u32<0x4E>(v));    // quad_perm [2,3,0,1]
    v = max(v, dpp_u32<0x124>(v));   // row_ror:4
    v = max(v, dpp_u32<0x128>(v));   // row_ror:8
    const uint32_t r0 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 0));
    const uint32_t r1 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 16));
    const uint32_t r2 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 32));
    const uint32_t r3 = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 48));
    return max(max(r0, r1), max(r2, r3));
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

// workgroup sum in a fixed order; result valid in thread 0
template <int NT, typename V>
__device__ __forceinline__ V block_sum(V v)
{
    __shared__ V red[NT / 64];
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
        for (int w = 0; w < NT / 64; ++w)
            t += red[w];
    }
    __syncthreads();
    return t;
}

// N workgroup sums at once, each in the order of block_sum (wave shuffle
// tree, then the waves in order); results valid in thread 0.  One barrier
// for all N (the caller's last use of the workgroup, so none after it).
template <int NT, int N, typename V>
__device__ __forceinline__ void block_sum_n_final(V* v)
{
    __shared__ V red[N][NT / 64];
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        V x = v[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1)
            x += __shfl_down(x, off, 64);
        if (lane == 0)
            red[q][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            V t = V(0);
#pragma unroll
            for (int w = 0; w < NT / 64; ++w)
                t += red[q][w];
            v[q] = t;
        }
    }
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b on XCD
// b mod 8), each XCD with its own L2.  Remapping b so that every XCD runs one
// contiguous chunk of logical blocks keeps neighbouring tiles and slot ranges,
// which share halo rows and gather sources, in the same L2.  The map is a
// bijection of [0, n) whatever the dispatch order.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n)
{
    constexpr uint32_t kXcd = 8;
    const uint32_t per = n / kXcd, rem = n % kXcd;
    const uint32_t x = b % kXcd, k = b / kXcd;
    return x * per + (x < rem ? x : rem) + k;
}

// -------------------------------------------------------------- binning
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
        double z[3] = {0.0, 0.0, 0.0}, spare;
        normal_pair(a.seed, a.step, pid, 0u, &z[0], &z[1]);
        if (D == 3)
            normal_pair(a.seed, a.step, pid, 1u, &z[2], &spare);
        T jv[3];
        make_jumps<D, T>(a, z, jv);
#pragma unroll
        for (int k = 0; k < D; ++k)
            v[k] = reflect_jump<T>(v[k], jv[k], a.lo[k], a.hi[k], a.lof[k], a.hif[k]);
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

// Counts to scan are in[c] (+ in2[c] when in2 is given).
__device__ __forceinline__ void scan_reduce_body(const uint32_t* in, const uint32_t* in2, uint32_t* bsum,
                                                 uint32_t blk)
{
    const size_t base = static_cast<size_t>(blk) * kScanTile + threadIdx.x * kScanItems;
    const uint4* p = reinterpret_cast<const uint4*>(in + base);
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
        const uint4 w = p[q];
        s += w.x + w.y + w.z + w.w;
    }
    if (in2) {
        const uint4* p2 = reinterpret_cast<const uint4*>(in2 + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const uint4 w = p2[q];
            s += w.x + w.y + w.z + w.w;
        }
    }
    const uint32_t t = block_sum<kBlock, uint32_t>(s);
    if (threadIdx.x == 0)
        bsum[blk] = t;
}

// Exclusive scan of the nb tile totals in place, by one workgroup: each
// thread takes 16 consecutive totals per round (its loads in flight
// together), so a round covers 4096 totals.
__device__ __forceinline__ void scan_top_body(uint32_t* bsum, uint32_t nb)
{
    constexpr uint32_t kTop = 16;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kBlock * kTop) {
        const uint32_t i0 = base + threadIdx.x * kTop;
        uint32_t v[kTop];
#pragma unroll
        for (uint32_t q = 0; q < kTop; ++q)
            v[q] = i0 + q < nb ? bsum[i0 + q] : 0u;
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t q = 0; q < kTop; ++q)
            sum += v[q];
        uint32_t tot;
        uint32_t run = carry + block_excl_scan(sum, &tot);
#pragma unroll
        for (uint32_t q = 0; q < kTop; ++q) {
            if (i0 + q < nb)
                bsum[i0 + q] = run;
            run += v[q];
        }
        carry += tot;
    }
}

// bsum holds the exclusive prefix of the tile totals (after the top pass),
// or with fold the raw totals, summed here over the tiles before blk.
__device__ __forceinline__ void scan_down_body(uint32_t* in, const uint32_t* in2, uint32_t* out,
                                               const uint32_t* bsum, uint32_t blk, bool zero_in,
                                               bool fold = false)
{
    __shared__ uint32_t pre_s;
    if (fold) {
        uint32_t t = 0;
        for (uint32_t b = threadIdx.x; b < blk; b += kBlock)
            t += bsum[b];
        t = block_sum<kBlock, uint32_t>(t);
        if (threadIdx.x == 0)
            pre_s = t;
        __syncthreads();
    }
    const uint32_t pre = fold ? pre_s : bsum[blk];
    const size_t base = static_cast<size_t>(blk) * kScanTile + threadIdx.x * kScanItems;
    uint4* p = reinterpret_cast<uint4*>(in + base);
    uint32_t v[kScanItems];
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
        const uint4 w = p[q];
        v[4 * q + 0] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
    }
    if (in2) {
        const uint4* p2 = reinterpret_cast<const uint4*>(in2 + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const uint4 w = p2[q];
            v[4 * q + 0] += w.x; v[4 * q + 1] += w.y; v[4 * q + 2] += w.z; v[4 * q + 3] += w.w;
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t t = v[k];
        v[k] = s;
        s += t;
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(s, &tot) + pre;
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
    const uint32_t c = a.cell[i];
    const uint32_t r = a.rank[i];
    uint32_t slot = a.starts[c];
    if (a.tcounts_valid) {
        // slots of a cell: its tile's own particles first, then the arrivals
        // from other tiles (rank flagged in bit 31)
        slot += (r >> 31) ? a.tcounts[c] : 0u;
        slot += r & 0x7fffffffu;
    } else {
        slot += r;
    }
    a.perm[slot] = static_cast<uint32_t>(i);
}

// Linear cell index of a position (x fastest), as the binning computes it.
template <int D, typename T>
__device__ __forceinline__ uint32_t cell_index(const SimArgs& a, const T* v)
{
    uint32_t c = 0;
#pragma unroll
    for (int k = D - 1; k >= 0; --k)
        c = c * static_cast<uint32_t>(a.nc[k]) +
            static_cast<uint32_t>(cell_coord(static_cast<double>(v[k]), a.glo[k], a.inv_side[k], a.nc[k]));
    return c;
}

// Slot k holds particle src after the scatter, in arbitrary order inside its
// cell.  Its final slot is the cell start plus the number of cell members
// with a smaller (x, pid) key.  The workgroup gathers the keys of its 256
// slots once into LDS; only members of a cell that straddles the range of
// the workgroup are read from global memory.
template <int D, typename T, typename M>
__device__ __forceinline__ void place_body(const SimArgs& a, uint32_t blk)
{
    __shared__ T lkx[kBlock];
    __shared__ uint32_t lkp[kBlock];
    const int64_t k0 = static_cast<int64_t>(blk) * kBlock;
    const int64_t k = k0 + threadIdx.x;
    const bool live = k < a.n;
    const T* xt0 = static_cast<const T*>(a.xt[0]);
    uint32_t src = 0, kp = 0, b = 0, e = 0;
    T xv[3];
    M mv[3];
    T jv[3];
    if (live) {
        src = a.perm[k];
#pragma unroll
        for (int d = 0; d < D; ++d)
            xv[d] = static_cast<const T*>(a.xt[d])[src];
        kp = a.pid_src[src];
        // the masses are gathered with the keys, not after the ranking
        // (unless the row-sum pass moves them)
        if (!a.src_slot) {
#pragma unroll
            for (int s = 0; s < 3; ++s)
                if (s < a.ns)
                    mv[s] = static_cast<const M*>(a.m_src[s])[src];
        }
        const uint32_t c = cell_index<D, T>(a, xv);
        b = a.starts[c];
        e = a.starts[c + 1];
        lkx[threadIdx.x] = xv[0];
        lkp[threadIdx.x] = kp;
        if (a.fuse_bin) {
            // the jumps of the step after a.step, for the transfer pass's
            // walk, drawn while the cell's offsets are in flight
            double z[3] = {0.0, 0.0, 0.0}, spare;
            normal_pair(a.seed, a.step + 1, kp, 0u, &z[0], &z[1]);
            if (D == 3)
                normal_pair(a.seed, a.step + 1, kp, 1u, &z[2], &spare);
            make_jumps<D, T>(a, z, jv);
        }
    }
    __syncthreads();
    if (!live)
        return;
    const uint32_t lo = static_cast<uint32_t>(k0);
    const uint32_t hi = static_cast<uint32_t>(min(k0 + kBlock, a.n));
    const T kx = xv[0];
    uint32_t rank = 0;
    for (uint32_t q = b; q < e; ++q) {
        T ox;
        uint32_t op;
        if (q >= lo && q < hi) {
            ox = lkx[q - lo];
            op = lkp[q - lo];
        } else {
            const uint32_t o = a.perm[q];
            ox = xt0[o];
            op = a.pid_src[o];
        }
        rank += (ox < kx || (ox == kx && op < kp)) ? 1u : 0u;
    }
    const uint32_t dst = b + rank;
#pragma unroll
    for (int d = 0; d < D; ++d)
        static_cast<T*>(a.x[d])[dst] = xv[d];
    if (a.src_slot) {
        a.src_slot[dst] = src;
    } else {
#pragma unroll
        for (int s = 0; s < 3; ++s)
            if (s < a.ns)
                static_cast<M*>(a.m_mid[s])[dst] = mv[s];
    }
    a.pid_dst[dst] = kp;
    if (a.fuse_bin) {
#pragma unroll
        for (int d = 0; d < D; ++d)
            static_cast<T*>(a.jmp[d])[dst] = jv[d];
    }
}

// ------------------------------------------------------------ tiled passes
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
    // one division for both cases (operands chosen first)
    const bool dpos = d > 0.0;
    const double num = dpos ? ca * d : ca;
    const double den = dpos ? d - cb * expm1(-a.k_react * d * a.dt) : 1.0 + a.k_react * ca * a.dt;
    const double an = num / den;
    const double bn = an - d;
    const double reacted = ca - an;
    m[0] = (sw ? bn : an) * a.to_m;
    m[1] = (sw ? an : bn) * a.to_m;
    m[2] = m[2] + reacted * a.to_m;
}

// Rows are trimmed to the particle's x-window (per row, from its y/z
// distance) before the candidate loop when rows are long (a.trim_rows, set
// by the host from the mean cell occupancy); short rows are scanned whole.

template <typename T> __device__ __forceinline__ T win2_of(const SimArgs& a);
template <> __device__ __forceinline__ double win2_of<double>(const SimArgs& a) { return a.win2d; }
template <> __device__ __forceinline__ float win2_of<float>(const SimArgs& a) { return a.win2f; }
template <typename T> __device__ __forceinline__ T wmargin_of(const SimArgs& a);
template <> __device__ __forceinline__ double wmargin_of<double>(const SimArgs& a) { return a.wmargind; }
template <> __device__ __forceinline__ float wmargin_of<float>(const SimArgs& a) { return a.wmarginf; }

// Per-particle accumulator of the two passes.
template <int PREC, int NS, bool TRANSFER> struct Acc;

template <int PREC, int NS> struct Acc<PREC, NS, false> {
    using T = typename Types<PREC>::T;
    T s = T(0);
    uint32_t cnt = 0;
};

template <int PREC, int NS> struct Acc<PREC, NS, true> {
    using T = typename Types<PREC>::T;
    using M = typename Types<PREC>::M;
    using A = typename Types<PREC>::A;
    T si;
    M mi[NS];
    A dl[NS];
    A comp[NS];
};

// Candidates of one halo row: positions p[k] (k in [b, e), x-sorted), and for
// the transfer pass row sums sr[k] and masses ms[c][k]; slot j = k + jofs.
// Only the x-window [xlo, xhi] is visited.  rec(k) sees every candidate
// within the cutoff other than the particle itself.
template <int D, int PREC, int NS, bool TRANSFER, bool TN, typename PX, typename PS, typename PM, typename PR>
__device__ __forceinline__ void scan_row(const SimArgs& a, PX p, PS sr, PM ms, uint32_t b, uint32_t e,
                                         uint32_t jofs, const typename Types<PREC>::T* xi,
                                         typename Types<PREC>::T xlo, typename Types<PREC>::T xhi,
                                         uint32_t i, Acc<PREC, NS, TRANSFER>& acc, PR rec)
{
    using T = typename Types<PREC>::T;
    using M = typename Types<PREC>::M;
    using A = typename Types<PREC>::A;
    for (uint32_t k = b; k < e; ++k) {
        T xj[3];
        xj[0] = p(0, k);
        if (xj[0] < xlo)
            continue;
        if (xj[0] > xhi)
            break;
#pragma unroll
        for (int d = 1; d < D; ++d)
            xj[d] = p(d, k);
        if (TRANSFER && k + jofs == i)
            continue;
        T r2;
        if (!Metric<D, T, TN>::inside(a, xi, xj, &r2))
            continue;
        if (k + jofs != i)
            rec(k);
        const T kv = Pair<D, T>::kernel(a, r2);
        if constexpr (!TRANSFER) {
            acc.s += kv;
            acc.cnt += 1;
        } else {
            const T w = Pair<D, T>::weight(kv, acc.si, sr(k));
#pragma unroll
            for (int c = 0; c < NS; ++c) {
                const M mj = ms(c, k);
                if (PREC == 2) {
                    // Kahan-compensated FP32 accumulation
                    const A y = static_cast<A>(w) * static_cast<A>(mj - acc.mi[c]) - acc.comp[c];
                    const A t = acc.dl[c] + y;
                    acc.comp[c] = (t - acc.dl[c]) - y;
                    acc.dl[c] = t;
                } else {
                    acc.dl[c] = __builtin_fma(static_cast<A>(w), static_cast<A>(mj - acc.mi[c]), acc.dl[c]);
                }
            }
        }
    }
}

// Walk (with the jumps the place pass drew), cell id and histogram slot of
// sorted particle i for the step after a.step (the next step's binning,
// done while its position is in registers).
// A particle that stays inside the tile (cells [tlo, thi) per axis) takes
// its slot from the tile's LDS histogram hist (two 16-bit counts per word,
// used when the tile holds fewer than 65536 particles: tile_hist); one that
// leaves takes it from the global histogram, flagged in bit 31 of its rank.
// The slot is returned, not stored: the caller stores it after other work,
// so that the atomic's round trip overlaps that work.
template <int D, typename T>
__device__ __forceinline__ uint32_t bin_next(const SimArgs& a, uint32_t i, const T* x, const T* jump,
                                             const int* tlo, const int* thi, uint32_t* hist, bool tile_hist)
{
    uint32_t c = 0, lc = 0;
    bool inside = true;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        const T v = reflect_jump<T>(x[k], jump[k], a.lo[k], a.hi[k], a.lof[k], a.hif[k]);
        static_cast<T*>(a.xt[k])[i] = v;
        const int ck = cell_coord(static_cast<double>(v), a.glo[k], a.inv_side[k], a.nc[k]);
        c = c * static_cast<uint32_t>(a.nc[k]) + static_cast<uint32_t>(ck);
        inside = inside && ck >= tlo[k] && ck < thi[k];
        // tile-local index < 2^16 (a 24-bit multiply)
        lc = __umul24(lc, static_cast<uint32_t>(thi[k] - tlo[k])) + static_cast<uint32_t>(ck - tlo[k]);
    }
    a.cell[i] = c;
    uint32_t rank;
    if (inside && tile_hist) {
        const uint32_t sh = (lc & 1u) << 4;
        rank = (atomicAdd(&hist[lc >> 1], 1u << sh) >> sh) & 0xFFFFu;
    } else {
        rank = 0x80000000u | atomicAdd(&a.counts[c], 1u);
    }
    return rank;
}

// One tile: tx * ty * tz cells (tz = 1 in 2-d).  Halo rows (cells xa..xb-1
// of rows y0-1..y1 of planes z0-1..z1) are staged in LDS with the offsets of
// their cell boundaries; a particle in cell cx visits cells cx-1..cx+1 of
// each of its 3^(d-1) neighbouring rows, restricted to the x-window.  Halo
// and own rows are numbered y fastest with a fixed pitch per plane (see
// TileLimits); rows past the tile's extent are empty.
// With EXPORT the pass changes nothing: it records, for every own particle,
// the pairs it would use -- a.nb_col == nullptr: their count plus one (self)
// into a.nb_cnt[pid]; else the pids, self first, into a.nb_col from
// a.nb_row[pid] -- and skips every store of the step.
template <int D, int PREC, int NS, bool TRANSFER, bool TN, bool EXPORT = false>
__device__ __forceinline__ void tile_body(const SimArgs& a, uint32_t blk)
{
    using T = typename Types<PREC>::T;
    using M = typename Types<PREC>::M;
    constexpr int CAP = TileCap<D, PREC, NS, TRANSFER>::value;
    constexpr int planes = D == 3 ? 3 : 1;
    constexpr int SCAP = TRANSFER ? CAP : 1;
    // rows are trimmed to the spherical cutoff's x-window; an ellipsoidal
    // cutoff scans its rows whole (the host never sets trim_rows for it)
    constexpr bool kTrim = !TN;
    // the FP64 row-sum pass evaluates its (software) exp only for the
    // candidates within the cutoff, after each chunk of 32, where rows are
    // not trimmed (about one candidate in six is in; in trimmed rows most
    // are, and the second loop costs more than it saves: measured)
    constexpr bool kExpAfter = !TRANSFER && PREC == 0;
    const bool exp_after = kExpAfter && !(kTrim && a.trim_rows);
    __shared__ T lpos[D][CAP];
    __shared__ T lsr[SCAP];
    __shared__ M lms[NS][SCAP];
    constexpr int kSegs = TileLimits<D>::segs;
    constexpr int kRows = TileLimits<D>::own_rows;   // own rows (pitch kSY per plane)
    constexpr int kSY = TileLimits<D>::seg_y;
    __shared__ uint32_t seg_gb[kSegs];
    __shared__ uint32_t seg_off[kSegs + 1];
    __shared__ uint32_t cst[kSegs][TileLimits<D>::cols];
    __shared__ uint32_t own_gb[kRows];
    __shared__ uint32_t own_pre[kRows + 1];
    // the own-row table in 2-d; in 3-d its bytes would cost both passes a
    // workgroup per CU, and a search over at most 36 own rows finds the row
    constexpr bool kRowTab = D == 2 || MTPT_ROW_TABLE_3D != 0;
    __shared__ uint8_t row_of[kRowTab ? CAP : 1];   // own row of each own particle
    // 2-d FP64 row-sum pass: own cells in order of their candidate count, so
    // that a wave's trip count is near its lanes' mean (the pass's only sum
    // over particles, the pair count, is an integer: the order changes no
    // result).  The FP32 pass's candidates are too cheap to repay the ordering.
    constexpr bool kCellOrder = D == 2 && !TRANSFER && (PREC == 0 ? MTPT_CELL_ORDER_2D : MTPT_CELL_ORDER_2D_F32) != 0;
    constexpr int kCells = kCellOrder ? TileLimits<D>::max_x * TileLimits<D>::max_y : 1;
    __shared__ uint16_t ord[kCellOrder ? CAP : 1];
    __shared__ uint8_t ckey[kCells];
    __shared__ uint32_t obase[64];
    // per-cell counts of the particles that stay in the tile, two 16-bit
    // counts per word
    constexpr int kHist =
        TRANSFER ? (TileLimits<D>::max_x * TileLimits<D>::max_y * TileLimits<D>::max_z + 1) / 2 : 1;
    __shared__ uint32_t hist[kHist];

    const int tid = threadIdx.x;
    const int nc0 = a.nc[0], nc1 = a.nc[1], nc2 = a.nc[2];
    // this pass's tile plan
    const int* const tl = TRANSFER ? a.ttile : a.tile;
    const uint32_t tiles_x = TRANSFER ? a.ttiles_x : a.tiles_x;
    const uint32_t per_slab = tiles_x * (TRANSFER ? a.ttiles_y : a.tiles_y);
    const int tzi = static_cast<int>(blk / per_slab);
    const uint32_t rem = blk - static_cast<uint32_t>(tzi) * per_slab;
    const int tyi = static_cast<int>(rem / tiles_x);
    const int txi = static_cast<int>(rem - static_cast<uint32_t>(tyi) * tiles_x);
    const int x0 = txi * tl[0];
    const int x1 = min(x0 + tl[0], nc0);
    const int y0 = tyi * tl[1];
    const int y1 = min(y0 + tl[1], nc1);
    const int z0 = D == 3 ? tzi * tl[2] : 0;
    const int z1 = D == 3 ? min(z0 + tl[2], nc2) : 1;
    const int nrow = y1 - y0;                      // own rows per own plane
    const int nz = z1 - z0;                        // own planes (1 in 2-d)
    const int nown = nrow * nz;                    // own rows
    const int rows = nrow + 2;                     // halo rows per halo plane
    // Halo row sg = pz * kSY + py holds cells xa..xb-1 of grid row y0 - 1 + py
    // of plane z0 - 1 + pz (py < rows, pz < nz + 2; the others are empty).
    // Own row r = rz * kSY + ry holds cells x0..x1-1 of row y0 + ry of plane
    // z0 + rz (ry < nrow, rz < nz); its halo row is srow(r), and the halo rows
    // of its lowest candidate plane start at r.
    auto srow = [](int r) { return D == 3 ? r + kSY + 1 : r + 1; };
    const int xa = x0 > 0 ? x0 - 1 : 0;
    const int xb = x1 < nc0 ? x1 + 1 : nc0;
    const int ncol = xb - xa;
    const int tw = x1 - x0;
    if (TRANSFER && a.fuse_bin)
        for (int k = tid; k < (tw * nown + 1) / 2; k += kBlock)
            hist[k] = 0u;

    // every cell boundary of the halo rows in one round of loads, as global
    // slots (a row outside the grid is empty); the runs of the halo rows and
    // of the own rows follow from it.  A thread issues all its loads before
    // its first LDS store, so that they are in flight together (one round
    // trip instead of one per entry: measured 3.8 -> ~1.5 us of a 3-d tile).
    const int ncb = ncol + 1;
    // Thread k of a round takes boundary c = k % kCP of halo row k / kCP (a
    // power-of-two pitch: no integer division).  The loaded global slots stay
    // in registers until the rows' LDS offsets are known, then are stored
    // converted (kept as global slots when the tile does not fit the LDS).
    constexpr int kCP = TileLimits<D>::col_p;
    constexpr int kCstIt = (kSegs * kCP + kBlock - 1) / kBlock;
    uint32_t cv[kCstIt];
#pragma unroll
    for (int it = 0; it < kCstIt; ++it) {
        const int idx = tid + it * kBlock;
        const int sg = idx / kCP;
        const int c = idx % kCP;
        const int pzr = D == 3 ? sg / kSY : 0;
        const int pyr = D == 3 ? sg % kSY : sg;
        const int pz = z0 - 1 + pzr;
        const int py = y0 - 1 + pyr;
        const bool in = sg < kSegs && c < ncb && pyr < rows && (D == 2 || pzr < nz + 2) && py >= 0 &&
                        py < nc1 && (D == 2 || (pz >= 0 && pz < nc2));
        cv[it] = in ? a.starts[(static_cast<uint32_t>(D == 3 ? pz : 0) * nc1 + py) * nc0 + xa + c] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kCstIt; ++it) {
        const int idx = tid + it * kBlock;
        if (idx / kCP < kSegs && idx % kCP < ncb)
            cst[idx / kCP][idx % kCP] = cv[it];
    }
    __syncthreads();
    uint32_t slen = 0;
    if (tid < kSegs) {
        seg_gb[tid] = cst[tid][0];
        slen = cst[tid][ncol] - cst[tid][0];
    }
    uint32_t total;
    const uint32_t soff = block_excl_scan(slen, &total);
    if (tid < kSegs)
        seg_off[tid] = soff;
    if (tid == 0)
        seg_off[kSegs] = total;
    uint32_t olen = 0;
    if (tid < kRows) {
        const int ry = D == 3 ? tid % kSY : tid;
        const int rz = D == 3 ? tid / kSY : 0;
        uint32_t gb = 0;
        if (ry < nrow && rz < nz) {
            const int sr = srow(tid);
            gb = cst[sr][x0 - xa];
            olen = cst[sr][x1 - xa] - gb;
        }
        own_gb[tid] = gb;
    }
    uint32_t own_total;
    const uint32_t ooff = block_excl_scan(olen, &own_total);
    if (tid < kRows)
        own_pre[tid] = ooff;
    if (tid == 0)
        own_pre[kRows] = own_total;
    __syncthreads();

    const bool use_lds = total <= static_cast<uint32_t>(CAP);
    // cell boundaries of every halo row as LDS offsets (read by the particle
    // loop after the staging barrier)
    if (use_lds) {
#pragma unroll
        for (int it = 0; it < kCstIt; ++it) {
            const int idx = tid + it * kBlock;
            const int sg = idx / kCP;
            if (sg < kSegs && idx % kCP < ncb)
                cst[sg][idx % kCP] = cv[it] - seg_gb[sg] + seg_off[sg];
        }
    }
    // own row of every own particle, when they fit the table (2-d)
    const bool rows_tab = kRowTab && own_total <= static_cast<uint32_t>(CAP);
    if (rows_tab)
        for (int r = tid >> 6; r < kRows; r += kBlock / 64)
            for (uint32_t j = static_cast<uint32_t>(tid & 63); j < own_pre[r + 1] - own_pre[r]; j += 64)
                row_of[own_pre[r] + j] = static_cast<uint8_t>(r);
    if (use_lds) {
        // Each halo row is one contiguous run in HBM and in LDS.  A thread
        // stages slots tid, tid + kBlock, ...: it finds every slot's row
        // first (the searches advance together), then issues all its loads,
        // then all its LDS stores, so that its loads are in flight at once.
        constexpr int kIt = (CAP + kBlock - 1) / kBlock;
        uint32_t sidx[kIt];
        int sb[kIt];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            sidx[it] = static_cast<uint32_t>(tid + it * kBlock);
            sb[it] = 0;
        }
        // last row whose first slot is <= the slot (seg_off[0] = 0; an empty
        // row shares its offset with the next one, which then wins); the range
        // [sb, sb + len) always holds it
#pragma unroll
        for (int len = kSegs; len > 1;) {
            const int half = len >> 1;
#pragma unroll
            for (int it = 0; it < kIt; ++it)
                sb[it] = seg_off[sb[it] + half] <= sidx[it] ? sb[it] + half : sb[it];
            len -= half;
        }
        T vx[kIt][D];
        T vs[kIt];
        M vm[kIt][NS];
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            if (sidx[it] < total) {
                const uint32_t g = seg_gb[sb[it]] + (sidx[it] - seg_off[sb[it]]);
#pragma unroll
                for (int d = 0; d < D; ++d)
                    vx[it][d] = static_cast<const T*>(a.x[d])[g];
                if (TRANSFER) {
                    vs[it] = static_cast<const T*>(a.srow)[g];
#pragma unroll
                    for (int c = 0; c < NS; ++c)
                        vm[it][c] = static_cast<const M*>(a.m_mid[c])[g];
                }
            }
        }
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            if (sidx[it] < total) {
                const uint32_t idx = sidx[it];
#pragma unroll
                for (int d = 0; d < D; ++d)
                    lpos[d][idx] = vx[it][d];
                if (TRANSFER) {
                    lsr[idx] = vs[it];
#pragma unroll
                    for (int c = 0; c < NS; ++c)
                        lms[c][idx] = vm[it][c];
                }
            }
        }
    }
    __syncthreads();

    const bool cell_order = kCellOrder && use_lds && rows_tab;
    if constexpr (kCellOrder) {
        if (cell_order) {
            if (tid < 64)
                obase[tid] = 0;
            __syncthreads();
            // own row r is halo row r + 1; own column cx is staged column x0 - xa + cx
            for (int j = tid; j < tw * nrow; j += kBlock) {
                const int r = j / tw;
                const int cxr = x0 - xa + (j - r * tw);
                const int cl = cxr > 0 ? cxr - 1 : 0;
                const int ch = cxr + 2 < ncol ? cxr + 2 : ncol;
                uint32_t tot = 0;
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    tot += cst[r + q][ch] - cst[r + q][cl];
                const uint32_t key = min(tot, 63u);
                ckey[j] = static_cast<uint8_t>(key);
                atomicAdd(&obase[key], cst[r + 1][cxr + 1] - cst[r + 1][cxr]);
            }
            __syncthreads();
            if (tid < 64) {
                const uint32_t v = obase[tid];
                obase[tid] = wave_incl_scan(v) - v;
            }
            __syncthreads();
            for (int j = tid; j < tw * nrow; j += kBlock) {
                const int r = j / tw;
                const int cxr = x0 - xa + (j - r * tw);
                const uint32_t c0 = cst[r + 1][cxr];
                const uint32_t nin = cst[r + 1][cxr + 1] - c0;
                if (nin == 0)
                    continue;
                const uint32_t pos = atomicAdd(&obase[ckey[j]], nin);
                const uint32_t t0 = own_pre[r] + (c0 - cst[r + 1][x0 - xa]);
                for (uint32_t q = 0; q < nin; ++q)
                    ord[pos + q] = static_cast<uint16_t>(t0 + q);
            }
            __syncthreads();
        }
    }

    uint32_t pairs = 0;
    double msum[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c)
        msum[c] = 0.0;
    // Every lane of a wave runs every pass the wave takes (own_total is
    // uniform, and the loop holds no workgroup barrier), so the wave-wide
    // maxima below see only live lanes.  A wave leaves once all its lanes are
    // past the last own particle.
    for (uint32_t base = 0; base < own_total; base += kBlock) {
        if (base + static_cast<uint32_t>(tid & ~63) >= own_total)
            break;
        const uint32_t t = base + tid;
        const bool act = t < own_total;
        uint32_t tt = act ? t : own_total - 1u;
        if constexpr (kCellOrder) {
            if (cell_order)
                tt = ord[tt];
        }
        int r = 0;
        if (rows_tab) {
            r = row_of[kRowTab ? tt : 0u];
        } else {
            // last own row whose first particle is <= tt (an empty row shares
            // its offset with the next one, which then wins), in fixed steps
#pragma unroll
            for (int len = kRows; len > 1;) {
                const int half = len >> 1;
                r = own_pre[r + half] <= tt ? r + half : r;
                len -= half;
            }
        }
        const uint32_t i = own_gb[r] + (tt - own_pre[r]);
        // the particle's LDS slot; its own position (and, in the transfer
        // pass, row sum and masses) from there when the tile is staged, else
        // coalesced global loads (LDS reads and global loads stay separate
        // instructions: a select of the two addresses would make them flat
        // loads)
        const int smid0 = srow(r);
        const uint32_t lself = i - seg_gb[smid0] + seg_off[smid0];
        const uint32_t lq = use_lds ? lself : 0u;
        // first halo row of the particle's lowest candidate plane
        const int rbase = r;
        T xi[3];
#pragma unroll
        for (int d = 0; d < D; ++d)
            xi[d] = lpos[d][lq];
        if (!use_lds) {
#pragma unroll
            for (int d = 0; d < D; ++d)
                xi[d] = static_cast<const T*>(a.x[d])[i];
        }
        const int cxr = cell_coord(static_cast<double>(xi[0]), a.glo[0], a.inv_side[0], nc0) - xa;
        const int cl = cxr > 0 ? cxr - 1 : 0;
        const int ch = cxr + 2 < ncol ? cxr + 2 : ncol;
        Acc<PREC, NS, TRANSFER> acc;
        // export: the particle's pid and its next column in a.nb_col
        uint32_t ecnt = 0;
        int64_t ebase = 0;
        uint32_t epid = 0;
        if constexpr (EXPORT) {
            if (act) {
                epid = a.pid_dst[i];
                if (a.nb_col)
                    ebase = a.nb_row[epid] + 1;
            }
        }
        // one pair of particle i with sorted slot g
        auto record = [&](uint32_t g) {
            if constexpr (EXPORT) {
                if (a.nb_col)
                    a.nb_col[ebase + ecnt] = static_cast<int64_t>(a.pid_dst[g]);
                ++ecnt;
            }
        };
        // the particle's jumps and neighbour masks are loaded before its
        // candidate loops, all at once (issued later, each would stall the
        // wave in front of its use: measured 10 % of the 3-d three-species
        // transfer pass)
        constexpr bool kEarly = TRANSFER;
        T jv[3] = {T(0), T(0), T(0)};
        uint64_t mkp[planes], wkp[planes];
#pragma unroll
        for (int pzr = 0; pzr < planes; ++pzr)
            mkp[pzr] = wkp[pzr] = 0ull;
        if constexpr (TRANSFER) {
            const uint32_t ls = lq < SCAP ? lq : 0u;
            acc.si = lsr[ls];
#pragma unroll
            for (int c = 0; c < NS; ++c) {
                acc.mi[c] = lms[c][ls];
                acc.dl[c] = 0;
                acc.comp[c] = 0;
            }
            if (!use_lds) {
                acc.si = static_cast<const T*>(a.srow)[i];
#pragma unroll
                for (int c = 0; c < NS; ++c)
                    acc.mi[c] = static_cast<const M*>(a.m_mid[c])[i];
            }
            if (kEarly && a.fuse_bin) {
#pragma unroll
                for (int d = 0; d < D; ++d)
                    jv[d] = static_cast<const T*>(a.jmp[d])[i];
            }
            if (kEarly && act) {
#pragma unroll
                for (int pzr = 0; pzr < planes; ++pzr)
                    mkp[pzr] = a.cmask[static_cast<size_t>(pzr) * static_cast<size_t>(a.n) + i];
            }
            if (kEarly && NS == 1 && use_lds && kTrim && a.trim_rows && act) {
#pragma unroll
                for (int pzr = 0; pzr < planes; ++pzr)
                    wkp[pzr] = a.cwin[static_cast<size_t>(pzr) * static_cast<size_t>(a.n) + i];
            }
        }
        if (use_lds) {
            // LDS slot of particle i itself (the self pair is skipped by slot)
            const uint32_t li = lself;
            if constexpr (!TRANSFER)
                acc.cnt = 1;   // self; the neighbours are counted from the masks
            // distances from the particle to the y (and z) slabs of the rows
            // below and above its own, less a rounding margin (for trimming)
            T dyv[3] = {T(0), T(0), T(0)};
            T dzv[3] = {T(0), T(0), T(0)};
            if (kTrim && a.trim_rows) {
                const int cyc = cell_coord(static_cast<double>(xi[1]), a.glo[1], a.inv_side[1], nc1);
                const T ylo = static_cast<T>(a.glo[1] + cyc * a.side[1]);
                dyv[0] = xi[1] - ylo - wmargin_of<T>(a);
                dyv[2] = ylo + static_cast<T>(a.side[1]) - xi[1] - wmargin_of<T>(a);
                if (D == 3) {
                    const int czc = cell_coord(static_cast<double>(xi[2]), a.glo[2], a.inv_side[2], nc2);
                    const T zlo = static_cast<T>(a.glo[2] + czc * a.side[2]);
                    dzv[0] = xi[2] - zlo - wmargin_of<T>(a);
                    dzv[2] = zlo + static_cast<T>(a.side[2]) - xi[2] - wmargin_of<T>(a);
                }
            }
#pragma unroll
            for (int pzr = 0; pzr < planes; ++pzr) {
                const int s0 = rbase + pzr * kSY;
                uint32_t b0 = cst[s0][cl], l0 = cst[s0][ch] - b0;
                uint32_t b1 = cst[s0 + 1][cl], l1 = cst[s0 + 1][ch] - b1;
                uint32_t b2 = cst[s0 + 2][cl], l2 = cst[s0 + 2][ch] - b2;
                if (kTrim && a.trim_rows) {
                    uint32_t bb[3] = {b0, b1, b2}, ll[3] = {l0, l1, l2};
                    uint64_t* const pwin = a.cwin + static_cast<size_t>(pzr) * static_cast<size_t>(a.n);
                    // the one-species transfer pass takes the windows the
                    // row-sum pass recorded when every lane's fit the packing
                    // (offset into the row and length, 10 bits each per row,
                    // bit 63 set); otherwise the wave searches again, to the
                    // same result (the three-species kernels always search:
                    // their registers are the tighter limit)
                    bool have = false;
                    if constexpr (TRANSFER && NS == 1) {
                        const uint64_t wv = act ? (kEarly ? wkp[pzr] : pwin[i]) : (1ull << 63);
                        have = __builtin_amdgcn_ballot_w64((wv >> 63) == 0ull) == 0ull;
                        if (have) {
#pragma unroll
                            for (int q = 0; q < 3; ++q) {
                                bb[q] += static_cast<uint32_t>(wv >> (20 * q)) & 0x3ffu;
                                ll[q] = static_cast<uint32_t>(wv >> (20 * q + 10)) & 0x3ffu;
                            }
                        }
                    }
                    if (!have) {
                        // x-window of each row from its y/z distance: |dx|^2 <= psi^2 - dy^2 - dz^2
                        const T dz = dzv[D == 3 ? pzr : 1] > T(0) ? dzv[D == 3 ? pzr : 1] : T(0);
                        T wlo[3], whi[3];
                        uint32_t lmax = 0;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const T dy = dyv[q] > T(0) ? dyv[q] : T(0);
                            const T w2 = win2_of<T>(a) - dy * dy - dz * dz;
                            const T w = w2 > T(0) ? static_cast<T>(sqrt(w2)) + wmargin_of<T>(a) : T(0);
                            wlo[q] = xi[0] - w;
                            whi[q] = xi[0] + w;
                            if (!(w2 > T(0)))
                                ll[q] = 0;
                            lmax = max(lmax, ll[q]);
                        }
                        lmax = wave_max_u32(lmax);
                        const int nsteps = 32 - __builtin_clz(lmax | 1u);
                        // per row, the first slot with x >= wlo and the first with
                        // x > whi, both searched over the whole (x-sorted) row:
                        // wlo <= whi, so the second is never before the first, and
                        // the six searches advance together
                        uint32_t slo[3], nlo[3], shi[3], nhi[3];
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            slo[q] = shi[q] = bb[q];
                            nlo[q] = nhi[q] = ll[q];
                        }
                        for (int st = 0; st < nsteps; ++st) {
#pragma unroll
                            for (int q = 0; q < 3; ++q) {
                                const uint32_t hl = nlo[q] >> 1, ml = slo[q] + hl;
                                const uint32_t hh = nhi[q] >> 1, mh = shi[q] + hh;
                                const bool gl = nlo[q] > 0u && lpos[0][ml < CAP ? ml : CAP - 1] < wlo[q];
                                const bool gh = nhi[q] > 0u && !(lpos[0][mh < CAP ? mh : CAP - 1] > whi[q]);
                                slo[q] = gl ? ml + 1u : slo[q];
                                nlo[q] = gl ? nlo[q] - hl - 1u : hl;
                                shi[q] = gh ? mh + 1u : shi[q];
                                nhi[q] = gh ? nhi[q] - hh - 1u : hh;
                            }
                        }
                        uint64_t pack = 1ull << 63;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const uint32_t off = slo[q] - bb[q];
                            bb[q] = slo[q];
                            ll[q] = shi[q] - slo[q];
                            pack = (off < 1024u && ll[q] < 1024u)
                                       ? pack | (static_cast<uint64_t>(off) << (20 * q)) |
                                             (static_cast<uint64_t>(ll[q]) << (20 * q + 10))
                                       : 0ull;
                        }
                        if constexpr (!TRANSFER && !EXPORT) {
                            if (act)
                                pwin[i] = pack;
                        }
                    }
                    b0 = bb[0]; l0 = ll[0];
                    b1 = bb[1]; l1 = ll[1];
                    b2 = bb[2]; l2 = ll[2];
                }
                const uint32_t tot = act ? l0 + l1 + l2 : 0u;
                // LDS byte offset of candidate k of the concatenated rows: k
                // sizeof(T) plus its row's offset (kept opaque so that the
                // scaling is not folded back into the candidate loops); a
                // candidate past the lane's rows reads the particle's own slot
                constexpr uint32_t kT = static_cast<uint32_t>(sizeof(T));
                uint32_t ob0 = b0 * kT, ob1 = (b1 - l0) * kT, ob2 = (b2 - l0 - l1) * kT, obs = li * kT;
                asm volatile("" : "+v"(ob0), "+v"(ob1), "+v"(ob2), "+v"(obs));
                const uint32_t e0 = l0, e1 = l0 + l1;
                auto slot_of = [ob0, ob1, ob2, obs, e0, e1](uint32_t k, bool valid) {
                    const uint32_t off = k * kT + (k < e0 ? ob0 : (k < e1 ? ob1 : ob2));
                    return valid ? off : obs;
                };
                auto ld = [](const auto* base, uint32_t off) {
                    return *reinterpret_cast<const std::remove_cv_t<std::remove_reference_t<decltype(*base)>>*>(
                        reinterpret_cast<const char*>(base) + off);
                };
                // the recorded neighbours serve the wave when every lane has
                // them (its row-sum tile was staged) and no lane has more
                // than 63 candidates (ballots: the wave-wide maximum is needed
                // only by the candidate loop)
                uint64_t mk = 0ull;
                bool use_mask = false, fits32 = false;
                if constexpr (TRANSFER) {
                    mk = kEarly ? mkp[pzr] : (act ? a.cmask[static_cast<size_t>(pzr) * static_cast<size_t>(a.n) + i] : 0ull);
                    use_mask = __builtin_amdgcn_ballot_w64(tot > 63u || (mk & kMaskInvalid) != 0ull) == 0ull;
                    fits32 = __builtin_amdgcn_ballot_w64(tot > 32u) == 0ull;
                }
                const uint32_t kmax = use_mask ? 0u : wave_max_u32(tot);
                constexpr int kUnroll = D == 3 ? (TRANSFER && NS == 3 ? MTPT_CAND_UNROLL_3D_S3 : MTPT_CAND_UNROLL_3D)
                                               : (PREC == 0 ? MTPT_CAND_UNROLL_2D_F64 : MTPT_CAND_UNROLL_2D);
                // one candidate at LDS byte offset off (of the T arrays), pair
                // counted when in
                auto visit = [&](uint32_t off, bool in, T r2) {
                    if constexpr (EXPORT) {
                        // LDS slot -> sorted slot: the halo row holding it
                        if (in && off != obs && act) {
                            const uint32_t lidx = off / kT;
                            int sgi = 0;
                            for (int q = 1; q < kSegs; ++q)
                                sgi = seg_off[q] <= lidx ? q : sgi;
                            record(seg_gb[sgi] + (lidx - seg_off[sgi]));
                        }
                    }
                    if constexpr (!TRANSFER) {
                        // the FP64 pass sums its kernel values after each
                        // chunk, over the chunk's neighbours only
                        if (!exp_after) {
                            const T kv = Pair<D, T>::kernel(a, r2);
                            acc.s += in ? kv : T(0);
                        }
                    } else {
                        const T kv = Pair<D, T>::kernel(a, r2);
                        using A = typename Types<PREC>::A;
                        const T w = Pair<D, T>::weight(kv, acc.si, ld(lsr, off));
#pragma unroll
                        for (int c = 0; c < NS; ++c) {
                            const M mj = ld(lms[c], off * static_cast<uint32_t>(sizeof(M) / sizeof(T)));
                            if (PREC == 2) {
                                const A y = static_cast<A>(w) * static_cast<A>(mj - acc.mi[c]) - acc.comp[c];
                                const A tk = acc.dl[c] + y;
                                const A cn = (tk - acc.dl[c]) - y;
                                acc.comp[c] = in ? cn : acc.comp[c];
                                acc.dl[c] = in ? tk : acc.dl[c];
                            } else {
                                // one rounding per increment, in the mask loop
                                // and the full loop alike
                                const A dm = static_cast<A>(mj - acc.mi[c]);
                                acc.dl[c] = __builtin_fma(static_cast<A>(w), in ? dm : A(0), acc.dl[c]);
                            }
                        }
                    }
                };
                uint64_t* const pmask = a.cmask + static_cast<size_t>(pzr) * static_cast<size_t>(a.n);
                if (TRANSFER && use_mask) {
                    // neighbours recorded by the row-sum pass: bit k of the
                    // mask is candidate k (same rows, same order) within psi
                    uint32_t cmax = static_cast<uint32_t>(__builtin_popcountll(mk));
                    cmax = wave_max_u32(cmax);
                    // a lane without a neighbour left visits its own slot:
                    // r^2 = 0 and m_j - m_i = 0 give an increment of exactly
                    // zero, which only the compensated sum has to skip
                    auto visit_bit = [&](uint32_t k, bool valid) {
                        const uint32_t off = slot_of(k, valid);
                        T xj[3];
#pragma unroll
                        for (int d = 0; d < D; ++d)
                            xj[d] = ld(lpos[d], off);
                        visit(off, PREC == 2 ? valid : true, Metric<D, T, TN>::r2(a, xi, xj));
                    };
                    if (fits32) {
                        // every lane's candidates fit the low word
                        uint32_t m32 = static_cast<uint32_t>(mk);
#pragma unroll kUnroll
                        for (uint32_t q = 0; q < cmax; ++q) {
                            const bool valid = m32 != 0u;
                            const uint32_t k = valid ? static_cast<uint32_t>(__builtin_ctz(m32)) : 0u;
                            m32 &= m32 - 1u;
                            visit_bit(k, valid);
                        }
                    } else {
#pragma unroll kUnroll
                        for (uint32_t q = 0; q < cmax; ++q) {
                            const bool valid = mk != 0ull;
                            const uint32_t k = valid ? static_cast<uint32_t>(__builtin_ctzll(mk)) : 0u;
                            mk &= mk - 1ull;
                            visit_bit(k, valid);
                        }
                    }
                    continue;
                }
                uint32_t mlo = 0, mhi = 0;
                // candidates in chunks of 32 (the chunk's mask word is
                // built without a branch: shifted in, first candidate
                // highest, then bit-reversed)
                for (uint32_t k0 = 0; k0 < kmax; k0 += 32u) {
                    const uint32_t kend = min(kmax, k0 + 32u);
                    uint32_t mw = 0;
#pragma unroll kUnroll
                    for (uint32_t k = k0; k < kend; ++k) {
                        const bool valid = k < tot;
                        const uint32_t off = slot_of(k, valid);
                        T xj[3];
#pragma unroll
                        for (int d = 0; d < D; ++d)
                            xj[d] = ld(lpos[d], off);
                        T r2;
                        bool in = Metric<D, T, TN>::inside(a, xi, xj, &r2) && valid;
                        if (TRANSFER)
                            in = in && off != obs;
                        visit(off, in, r2);
                        if constexpr (!TRANSFER)
                            mw = (mw << 1) | (in ? 1u : 0u);
                    }
                    if constexpr (!TRANSFER) {
                        // candidate k0 + j at bit j
                        mw = __builtin_bitreverse32(mw) >> (32u - (kend - k0));
                        if (exp_after) {
                            // kernel values of the chunk's candidates within
                            // the cutoff (the particle itself included), in
                            // candidate order: the same sum as adding every
                            // candidate's value or zero, with the software
                            // FP64 exp evaluated for about one candidate in
                            // six instead of all
                            uint32_t mr = mw;
                            uint32_t rmax = static_cast<uint32_t>(__builtin_popcount(mr));
                            rmax = wave_max_u32(rmax);
                            for (uint32_t q = 0; q < rmax; ++q) {
                                const bool valid = mr != 0u;
                                const uint32_t kb = valid ? static_cast<uint32_t>(__builtin_ctz(mr)) : 0u;
                                mr &= mr - 1u;
                                const uint32_t off = slot_of(k0 + kb, valid);
                                T xj[3];
#pragma unroll
                                for (int d = 0; d < D; ++d)
                                    xj[d] = ld(lpos[d], off);
                                const T kv = Pair<D, T>::kernel(a, Metric<D, T, TN>::r2(a, xi, xj));
                                acc.s += valid ? kv : T(0);
                            }
                        }
                        // the particle itself is candidate l0 + (li - b1) of
                        // its own plane's middle row
                        if (pzr == planes / 2) {
                            const uint32_t ks = l0 + (li - b1) - k0;
                            mw &= (act && ks < 32u) ? ~(1u << ks) : ~0u;
                        }
                        acc.cnt += static_cast<uint32_t>(__builtin_popcount(mw));
                        mlo = k0 == 0u ? mw : mlo;
                        mhi = k0 == 32u ? mw : mhi;
                    }
                }
                if (!TRANSFER && !EXPORT && act)
                    pmask[i] = tot <= 63u ? ((static_cast<uint64_t>(mhi) << 32) | mlo) : kMaskInvalid;
            }
        } else {
#pragma unroll
            for (int pzr = 0; pzr < planes; ++pzr) {
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int sg = rbase + pzr * kSY + dy;
                    const uint32_t b = cst[sg][cl];
                    const uint32_t e = act ? cst[sg][ch] : b;
                    T xlo, xhi;
                    Window<T>::make(xi[0], a.win, &xlo, &xhi);
                    scan_row<D, PREC, NS, TRANSFER, TN>(
                        a, [&](int d, uint32_t k) { return static_cast<const T*>(a.x[d])[k]; },
                        [&](uint32_t k) { return static_cast<const T*>(a.srow)[k]; },
                        [&](int c, uint32_t k) { return static_cast<const M*>(a.m_mid[c])[k]; }, b, e, 0u, xi,
                        xlo, xhi, i, acc, [&](uint32_t k) { if (act) record(k); });
                }
            }
            // no recorded neighbours or windows for the transfer pass (whose
            // tile may be staged)
            if (!TRANSFER && !EXPORT && act) {
#pragma unroll
                for (int pzr = 0; pzr < planes; ++pzr) {
                    a.cmask[static_cast<size_t>(pzr) * static_cast<size_t>(a.n) + i] = kMaskInvalid;
                    if (kTrim && a.trim_rows)
                        a.cwin[static_cast<size_t>(pzr) * static_cast<size_t>(a.n) + i] = 0ull;
                }
            }
        }
        if (!act)
            continue;
        if constexpr (EXPORT) {
            if (a.nb_col)
                a.nb_col[ebase - 1] = static_cast<int64_t>(epid);
            else
                a.nb_cnt[epid] = ecnt + 1u;
            continue;
        }
        if constexpr (!TRANSFER) {
            static_cast<T*>(a.srow)[i] = acc.s;
            pairs += acc.cnt - 1u;
            if (a.src_slot) {
                // the masses of the sorted slot, from the order before
                // re-binning (the place pass recorded the source slot): a
                // gather whose latency the arithmetic of the other waves hides
                const uint32_t src = a.src_slot[i];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (c < a.ns)
                        static_cast<M*>(a.m_mid[c])[i] = static_cast<const M*>(a.m_src[c])[src];
            }
        } else {
            // the next step's walk and binning first: the slot's atomic (for
            // a particle that leaves the tile) is in flight during the mass
            // update and the reaction
            uint32_t nrank = 0;
            if (a.fuse_bin) {
                const int tlo[3] = {x0, y0, z0};
                const int thi[3] = {x1, y1, z1};
                if (!kEarly) {
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        jv[d] = static_cast<const T*>(a.jmp[d])[i];
                }
                nrank = bin_next<D, T>(a, i, xi, jv, tlo, thi, hist, own_total < 65536u);
            }
            double mo[3];
#pragma unroll
            for (int c = 0; c < NS; ++c) {
                if (PREC == 2) {
                    const float nv = acc.mi[c] + a.betaf * acc.dl[c];
                    mo[c] = static_cast<double>(nv);
                } else {
                    mo[c] = static_cast<double>(acc.mi[c]) + a.beta * static_cast<double>(acc.dl[c]);
                }
            }
            if (NS == 3 && a.k_react > 0.0)
                react3(mo, a);
#pragma unroll
            for (int c = 0; c < NS; ++c) {
                const M st = static_cast<M>(mo[c]);
                static_cast<M*>(a.m_dst[c])[i] = st;
                msum[c] += static_cast<double>(st);
            }
            if (a.fuse_bin)
                a.rank[i] = nrank;
        }
    }
    if constexpr (EXPORT)
        return;
    if (TRANSFER && a.fuse_bin) {
        // counts of the tile's cells from the particles that stayed in it
        __syncthreads();
        const float inv_tw = 1.0f / static_cast<float>(tw);
        const float inv_nrow = 1.0f / static_cast<float>(nrow);
        for (int k = tid; k < tw * nown; k += kBlock) {
            const int rr = small_div(k, inv_tw);   // own row, y fastest (dense)
            const int rz = small_div(rr, inv_nrow);
            const uint32_t c = (static_cast<uint32_t>(z0 + rz) * nc1 + (y0 + rr - rz * nrow)) * nc0 + x0 + (k - rr * tw);
            a.tcounts[c] = (hist[k >> 1] >> ((k & 1) << 4)) & 0xFFFFu;
        }
    }
    if constexpr (!TRANSFER) {
        const uint32_t p = block_sum<kBlock, uint32_t>(pairs);
        if (tid == 0)
            a.pair_part[blk] = p;
    } else {
        block_sum_n_final<kBlock, NS, double>(msum);
        if (tid == 0) {
#pragma unroll
            for (int c = 0; c < NS; ++c)
                a.partials[static_cast<size_t>(blk) * NS + c] = msum[c];
        }
    }
}

// Totals and pair counters of one step (mode 0) or totals only (mode 1),
// summed over the per-workgroup partials in a fixed order.
template <int NT>
__device__ __forceinline__ void finalize_body(const SimArgs& a, uint32_t nparts, int mode)
{
    const int ns = a.ns;
    DevStats* st = a.st;
    unsigned long long pairs = 0;
    if (mode == 0 && a.recompute_s) {
        unsigned long long p = 0;
#pragma unroll 8
        for (uint32_t b = threadIdx.x; b < a.ntiles; b += NT)
            p += a.pair_part[b];
        pairs = block_sum<NT, unsigned long long>(p);
    }
    for (int c = 0; c < ns; ++c) {
        double s = 0.0;
#pragma unroll 8
        for (uint32_t b = threadIdx.x; b < nparts; b += NT)
            s += a.partials[static_cast<size_t>(b) * ns + c];
        const double t = block_sum<NT, double>(s);
        if (threadIdx.x == 0) {
            st->totals[c] = t;
            if (!isfinite(t))
                st->nonfinite = 1;
        }
    }
    if (threadIdx.x == 0 && mode == 0) {
        if (a.recompute_s)
            st->pairs_last = pairs;
        st->pairs_total += st->pairs_last;
        st->steps += 1;
    }
}

// ---------------------------------------------------------- tiled kernels
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

#define MTPT_BATCH_PROLOGUE                                                                     \
    uint32_t l;                                                                                 \
    const SimArgs& a = b.args[find_sim(b, xcd_block(blockIdx.x, gridDim.x), &l)]

// The 3-d FP32W isotropic row-sum pass is held to the seven waves per SIMD
// that its LDS allows (72 registers).
template <int D, int PREC, bool TN>
__global__ __launch_bounds__(kBlock, D == 3 && PREC == 1 && !TN ? 7 : 1) void rowsum_k(SimArgs a)
{
    tile_body<D, PREC, 1, false, TN>(a, xcd_block(blockIdx.x, gridDim.x));
}
template <int D, int PREC, bool TN>
__global__ __launch_bounds__(kBlock, D == 3 && PREC == 1 && !TN ? 7 : 1) void rowsum_kb(Batch b)
{
    MTPT_BATCH_PROLOGUE;
    tile_body<D, PREC, 1, false, TN>(a, l);
}

// the 2-d FP64 one-species transfer kernel is held to the registers of 5
// workgroups per CU, which its LDS allows
#ifndef MTPT_S3_MIN_BLOCKS
#define MTPT_S3_MIN_BLOCKS 1
#endif
template <int D, int PREC, int NS>
constexpr int transfer_min_blocks()
{
    return PREC == 0 && D == 2 && NS == 1 ? 5 : (D == 3 && PREC == 1 && NS == 3 ? MTPT_S3_MIN_BLOCKS : 1);
}
template <int D, int PREC, int NS, bool TN>
__global__ __launch_bounds__(kBlock, (transfer_min_blocks<D, PREC, NS>())) void transfer_k(SimArgs a)
{
    tile_body<D, PREC, NS, true, TN>(a, xcd_block(blockIdx.x, gridDim.x));
}
template <int D, int PREC, int NS, bool TN>
__global__ __launch_bounds__(kBlock, (transfer_min_blocks<D, PREC, NS>())) void transfer_kb(Batch b)
{
    MTPT_BATCH_PROLOGUE;
    tile_body<D, PREC, NS, true, TN>(a, l);
}

// Launch of the row-sum (ph = PH_ROWSUM) or transfer (PH_TRANSFER) pass of
// dimension D and metric TN: one sim (a) or a batch (b).  Instantiated by
// the mtpt_tiles_*.hip units, one per (D, TN).
template <int D, bool TN>
hipError_t launch_tiles(int ph, int prec, int ns, const SimArgs* a, const Batch* b, hipStream_t s)
{
    const uint32_t grid = a ? (ph == PH_ROWSUM ? a->ntiles : a->nttiles) : b->total_blocks;
    if (grid == 0 || (b && b->nsims == 0) || (a && a->n <= 0))
        return hipSuccess;
#define MTPT_TILE_LAUNCH(KSIM, KBAT)                                                             \
    do {                                                                                         \
        if (a) KSIM<<<grid, kBlock, 0, s>>>(*a);                                                 \
        else KBAT<<<grid, kBlock, 0, s>>>(*b);                                                   \
    } while (0)
    if (ph == PH_ROWSUM) {
        if (prec == 0) MTPT_TILE_LAUNCH((rowsum_k<D, 0, TN>), (rowsum_kb<D, 0, TN>));
        else if (prec == 1) MTPT_TILE_LAUNCH((rowsum_k<D, 1, TN>), (rowsum_kb<D, 1, TN>));
        else MTPT_TILE_LAUNCH((rowsum_k<D, 2, TN>), (rowsum_kb<D, 2, TN>));
    } else if (ph == PH_TRANSFER) {
        if (ns == 1) {
            if (prec == 0) MTPT_TILE_LAUNCH((transfer_k<D, 0, 1, TN>), (transfer_kb<D, 0, 1, TN>));
            else if (prec == 1) MTPT_TILE_LAUNCH((transfer_k<D, 1, 1, TN>), (transfer_kb<D, 1, 1, TN>));
            else MTPT_TILE_LAUNCH((transfer_k<D, 2, 1, TN>), (transfer_kb<D, 2, 1, TN>));
        } else {
            if (prec == 0) MTPT_TILE_LAUNCH((transfer_k<D, 0, 3, TN>), (transfer_kb<D, 0, 3, TN>));
            else if (prec == 1) MTPT_TILE_LAUNCH((transfer_k<D, 1, 3, TN>), (transfer_kb<D, 1, 3, TN>));
            else MTPT_TILE_LAUNCH((transfer_k<D, 2, 3, TN>), (transfer_kb<D, 2, 3, TN>));
        }
    } else {
        return hipErrorInvalidValue;
    }
#undef MTPT_TILE_LAUNCH
    return hipGetLastError();
}

// Export launches (mtpt_step_neighbors): the row-sum or transfer pass of
// the last step, recording instead of storing.
template <int D, int PREC, bool TN>
__global__ __launch_bounds__(kBlock) void rowsum_export_k(SimArgs a)
{
    tile_body<D, PREC, 1, false, TN, true>(a, xcd_block(blockIdx.x, gridDim.x));
}
template <int D, int PREC, int NS, bool TN>
__global__ __launch_bounds__(kBlock) void transfer_export_k(SimArgs a)
{
    tile_body<D, PREC, NS, true, TN, true>(a, xcd_block(blockIdx.x, gridDim.x));
}

template <int D, bool TN>
hipError_t launch_tiles_export(int ph, int prec, int ns, const SimArgs& a, hipStream_t s)
{
    const uint32_t grid = ph == PH_ROWSUM ? a.ntiles : a.nttiles;
    if (grid == 0 || a.n <= 0)
        return hipSuccess;
    if (ph == PH_ROWSUM) {
        if (prec == 0) rowsum_export_k<D, 0, TN><<<grid, kBlock, 0, s>>>(a);
        else if (prec == 1) rowsum_export_k<D, 1, TN><<<grid, kBlock, 0, s>>>(a);
        else rowsum_export_k<D, 2, TN><<<grid, kBlock, 0, s>>>(a);
    } else if (ph == PH_TRANSFER) {
        if (ns == 1) {
            if (prec == 0) transfer_export_k<D, 0, 1, TN><<<grid, kBlock, 0, s>>>(a);
            else if (prec == 1) transfer_export_k<D, 1, 1, TN><<<grid, kBlock, 0, s>>>(a);
            else transfer_export_k<D, 2, 1, TN><<<grid, kBlock, 0, s>>>(a);
        } else {
            if (prec == 0) transfer_export_k<D, 0, 3, TN><<<grid, kBlock, 0, s>>>(a);
            else if (prec == 1) transfer_export_k<D, 1, 3, TN><<<grid, kBlock, 0, s>>>(a);
            else transfer_export_k<D, 2, 3, TN><<<grid, kBlock, 0, s>>>(a);
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mtpt
