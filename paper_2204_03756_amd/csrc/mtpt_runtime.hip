// mtpt_runtime.hip -- host runtime and C-ABI of libmtpt.so.
//
// A simulation owns one device allocation carved into the buffers listed in
// mtpt_kernels.h, a stream, and the host-side step counter that decides which
// of the double buffers is current.  mtpt_step enqueues the phases of a step
// and never waits; exports enqueue a gather by pid and a device-to-host copy,
// then wait.
#include "../../include/mtpt.h"
#include "mtpt_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace mtpt;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(MTPT_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));             \
    } while (0)

struct Alloc {
    mtpt_allocator a{};
    bool custom = false;
    void* get(size_t bytes)
    {
        if (bytes == 0)
            bytes = 256;
        if (custom)
            return a.alloc(bytes, a.ctx);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void* p)
    {
        if (!p)
            return;
        if (custom)
            a.free(p, a.ctx);
        else
            (void)hipFree(p);
    }
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Buffer plan of one simulation: grid and byte offsets inside one allocation.
struct Plan {
    int dim = 2, ns = 1, prec = 0;
    int64_t n = 0;
    double psi = 0;
    int nc[3] = {1, 1, 1};
    double inv_side[3] = {0, 0, 0};
    uint32_t ncells = 1;
    uint32_t scan_blocks = 1, part_blocks = 0;
    int tile[3] = {1, 1, 1};                  // row-sum pass
    uint32_t tiles_x = 1, tiles_y = 1, ntiles = 0;
    int ttile[3] = {1, 1, 1};                 // transfer pass
    uint32_t ttiles_x = 1, ttiles_y = 1, nttiles = 0;
    bool trim_rows = false;
    bool tensor = false;
    size_t tsz = 8, msz = 8;
    size_t off_x[3]{}, off_xt[3]{}, off_m[2][3]{}, off_p[2]{}, off_s = 0, off_cell = 0, off_rank = 0,
           off_perm = 0, off_jmp[3]{}, off_cmask = 0, off_cwin = 0, off_counts = 0, off_tcounts = 0,
           off_starts = 0, off_bsum = 0, off_part = 0, off_pair = 0, off_stats = 0;
    size_t bytes = 0;
};

// Shape tensor T of the dispersion (D_RW = d_rw T, D_MT = d_mt T), its
// Cholesky factor L and M = L^-1, each entry formed in the fixed order of
// the C-ABI's note: L00 = sqrt(T00), L10 = T10 / L00, L11 = sqrt(T11 - L10 L10),
// L20 = T20 / L00, L21 = (T21 - L20 L10) / L11, L22 = sqrt((T22 - L20 L20) - L21 L21);
// M00 = 1/L00, M11 = 1/L11, M22 = 1/L22, M10 = -((L10 M00) M11),
// M21 = -((L21 M11) M22), M20 = -(((L20 M00) + (L21 M10)) M22).
struct Tensor {
    bool on = false;          // false: isotropic (T = I)
    double t[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double l[6] = {1, 0, 1, 0, 0, 1};
    double m[6] = {1, 0, 1, 0, 0, 1};
    double cond = 9.0;        // trace(T^-1) trace(T), the FP32 error factor of q
};

// 0, or -1 with a message in *why when T is not a symmetric positive-definite
// tensor (all zero is the isotropic default)
int tensor_of(const mtpt_params& p, Tensor* out, const char** why)
{
#pragma clang fp contract(off)
    Tensor g;
    const int d = p.dim;
    bool any = false;
    for (int k = 0; k < 9; ++k) {
        if (!std::isfinite(p.disp[k])) {
            *why = "disp must be finite";
            return -1;
        }
        const int r = k / 3, c = k % 3;
        if (r < d && c < d)
            any = any || p.disp[k] != 0.0;
    }
    if (!any) {
        g.cond = static_cast<double>(d * d);
        *out = g;
        return 0;
    }
    for (int r = 0; r < d; ++r)
        for (int c = 0; c < d; ++c)
            if (p.disp[r * 3 + c] != p.disp[c * 3 + r]) {
                *why = "disp must be symmetric";
                return -1;
            }
    g.on = true;
    for (int k = 0; k < 9; ++k)
        g.t[k] = (k / 3 < d && k % 3 < d) ? p.disp[k] : (k / 3 == k % 3 ? 1.0 : 0.0);
    const double* t = g.t;
    double* l = g.l;
    double* m = g.m;
    *why = "disp must be positive definite";
    if (!(t[0] > 0.0))
        return -1;
    l[0] = std::sqrt(t[0]);
    l[1] = t[3] / l[0];
    const double p1 = t[4] - l[1] * l[1];
    if (!(p1 > 0.0))
        return -1;
    l[2] = std::sqrt(p1);
    m[0] = 1.0 / l[0];
    m[2] = 1.0 / l[2];
    m[1] = -((l[1] * m[0]) * m[2]);
    l[3] = l[4] = m[3] = m[4] = 0.0;
    l[5] = m[5] = 1.0;
    if (d == 3) {
        l[3] = t[6] / l[0];
        l[4] = (t[7] - l[3] * l[1]) / l[2];
        const double p2 = (t[8] - l[3] * l[3]) - l[4] * l[4];
        if (!(p2 > 0.0))
            return -1;
        l[5] = std::sqrt(p2);
        m[5] = 1.0 / l[5];
        m[4] = -((l[4] * m[2]) * m[5]);
        m[3] = -(((l[3] * m[0]) + (l[4] * m[1])) * m[5]);
    }
    // trace(T^-1) = |M|_F^2 (T^-1 = M^T M) times trace(T)
    double fro = 0.0, tr = 0.0;
    for (int k = 0; k < 6; ++k)
        fro += (k == 3 || k == 4 || k == 5) && d == 2 ? 0.0 : m[k] * m[k];
    for (int k = 0; k < d; ++k)
        tr += t[k * 3 + k];
    g.cond = fro * tr;
    *why = "";
    *out = g;
    return 0;
}

int validate(const mtpt_params* p)
{
    if (!p)
        return fail(MTPT_E_ARG, "params is NULL");
    if (p->abi_version != MTPT_ABI_VERSION)
        return fail(MTPT_E_ABI, "abi_version %u, library has %d", p->abi_version, MTPT_ABI_VERSION);
    if (p->dim != 2 && p->dim != 3)
        return fail(MTPT_E_ARG, "dim must be 2 or 3 (got %d)", p->dim);
    if (p->n < 0 || p->n > 0x7FFFFF00ll)
        return fail(MTPT_E_ARG, "n must be in [0, 2^31 - 256] (got %lld)", (long long)p->n);
    if (p->n_species != 1 && p->n_species != 3)
        return fail(MTPT_E_ARG, "n_species must be 1 or 3 (got %d)", p->n_species);
    if (p->precision < 0 || p->precision > 2)
        return fail(MTPT_E_ARG, "precision must be 0, 1 or 2 (got %d)", p->precision);
    for (int k = 0; k < p->dim; ++k)
        if (!std::isfinite(p->lo[k]) || !std::isfinite(p->hi[k]) || !(p->hi[k] > p->lo[k]))
            return fail(MTPT_E_ARG, "box dimension %d: need finite lo < hi", k);
    if (!std::isfinite(p->d_rw) || p->d_rw < 0)
        return fail(MTPT_E_ARG, "d_rw must be finite and >= 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->vel[k]))
            return fail(MTPT_E_ARG, "vel must be finite");
    {
        Tensor g;
        const char* why = "";
        if (tensor_of(*p, &g, &why) != 0)
            return fail(MTPT_E_ARG, "%s", why);
    }
    if (!std::isfinite(p->d_mt) || !(p->d_mt > 0))
        return fail(MTPT_E_ARG, "d_mt must be finite and > 0");
    if (!std::isfinite(p->dt) || !(p->dt > 0))
        return fail(MTPT_E_ARG, "dt must be finite and > 0");
    if (!std::isfinite(p->beta) || !(p->beta > 0) || p->beta > 1.0)
        return fail(MTPT_E_ARG, "beta must be in (0, 1]");
    if (!std::isfinite(p->psi))
        return fail(MTPT_E_ARG, "psi must be finite");
    if (!std::isfinite(p->k_react) || p->k_react < 0)
        return fail(MTPT_E_ARG, "k_react must be finite and >= 0");
    if (p->start_step < 0)
        return fail(MTPT_E_ARG, "start_step must be >= 0");
    return MTPT_OK;
}

double psi_of(const mtpt_params& p) { return p.psi > 0 ? p.psi : 3.0 * std::sqrt(4.0 * p.d_mt * p.dt); }

// Fewest tiles of a sim's mass-transfer passes: MTPT_MIN_TILES from the
// environment when it holds a whole number in [1, 2^20], else 256 (one tile
// per compute unit).  1 keeps the throughput shape at every size.
int64_t tile_min_tiles()
{
    const char* e = std::getenv("MTPT_MIN_TILES");
    if (e && *e) {
        char* end = nullptr;
        const long long v = std::strtoll(e, &end, 10);
        if (end && *end == '\0' && v >= 1 && v <= (1ll << 20))
            return v;
    }
    return 256;
}

Plan make_plan(const mtpt_params& p)
{
    Plan q;
    q.dim = p.dim;
    q.ns = p.n_species;
    q.prec = p.precision;
    q.n = p.n;
    q.psi = psi_of(p);
    q.tsz = p.precision == MTPT_FP64 ? 8 : 4;
    q.msz = p.precision == MTPT_FP32_KAHAN ? 4 : 8;
    // cells of side >= psi (1 + 1e-6) along every axis -- psi sqrt(T_kk)
    // (1 + 1e-6), the reach of the ellipsoid q <= psi^2 along axis k, with a
    // dispersion tensor: every pair within the cutoff then lies in
    // neighbouring cells even after rounding of the cell coordinate
    Tensor g;
    const char* why = "";
    (void)tensor_of(p, &g, &why);
    q.tensor = g.on;
    for (int k = 0; k < q.dim; ++k) {
        const double L = p.hi[k] - p.lo[k];
        const double side_min = q.psi * std::sqrt(g.t[k * 3 + k]) * (1.0 + 1e-6);
        double c = std::floor(L / side_min);
        c = std::min(std::max(c, 1.0), 1048576.0);
        q.nc[k] = static_cast<int>(c);
    }
    // at most ~4 cells per particle (and 2^30 cells): larger cells are also correct
    const double cap = std::min(1073741824.0, std::max(64.0, 4.0 * static_cast<double>(q.n)));
    for (;;) {
        double tot = 1.0;
        for (int k = 0; k < q.dim; ++k)
            tot *= q.nc[k];
        if (tot <= cap)
            break;
        for (int k = 0; k < q.dim; ++k)
            q.nc[k] = std::max(1, q.nc[k] - std::max(1, q.nc[k] / 8));
    }
    q.ncells = 1;
    for (int k = 0; k < q.dim; ++k) {
        q.ncells *= static_cast<uint32_t>(q.nc[k]);
        q.inv_side[k] = static_cast<double>(q.nc[k]) / (p.hi[k] - p.lo[k]);
    }
    q.scan_blocks = static_cast<uint32_t>((static_cast<uint64_t>(q.ncells) + 1 + kScanTile - 1) / kScanTile);
    q.part_blocks = static_cast<uint32_t>((q.n + kBlock - 1) / kBlock);
    // tiles of the mass-transfer passes, the tile plus its one-cell halo
    // expected to fill at most 1/1.25 of the LDS staging capacity (a fuller
    // tile falls back to global reads).  2-d: about 640 own particles, square.
    // 3-d: the shape within the limits of least estimated cost per own
    // particle: wave passes (64 lanes; a wave with no particle left leaves)
    // over the own particles (with a margin of two standard deviations of
    // their count), staging of the halo and a fixed setup, in units of one
    // lane's candidate loop.  A sim too small to give every compute unit a
    // tile that way is cut into at least min_tiles tiles (or one tile per
    // cell): its step time is then the time of one small tile, not that of a
    // few large tiles on a mostly idle chip.
    {
        const double rho_c = static_cast<double>(q.n) / static_cast<double>(q.ncells);
        const int64_t min_tiles = tile_min_tiles();
        auto tiles_of = [&](int x, int y, int z) {
            return static_cast<int64_t>((q.nc[0] + x - 1) / x) * ((q.nc[1] + y - 1) / y) *
                   (q.dim == 3 ? (q.nc[2] + z - 1) / z : 1);
        };
#ifndef MTPT_TILE_OWN
#define MTPT_TILE_OWN 640.0
#endif
#ifndef MTPT_TILE_LANES
#define MTPT_TILE_LANES 64.0
#endif
        // the tile shape for a staging capacity of capn particles
        auto choose = [&](int capn, int* t) {
            const double cap = static_cast<double>(capn) / 1.25;
            int tx = 1, ty = 1, tz = 1;
            if (q.dim == 2) {
                const double cells_own = std::max(1.0, MTPT_TILE_OWN / std::max(rho_c, 1e-9));
                const int tt = static_cast<int>(std::lround(std::sqrt(cells_own)));
                tx = std::max(1, std::min(tt, std::min(q.nc[0], tile_max(2, 0))));
                ty = std::max(1, std::min(tt, std::min(q.nc[1], tile_max(2, 1))));
                while (((tx + 2.0) * (ty + 2.0) * rho_c > cap || tiles_of(tx, ty, 1) < min_tiles) &&
                       (tx > 1 || ty > 1)) {
                    if (tx >= ty)
                        --tx;
                    else
                        --ty;
                }
            } else {
                double best = 0.0;
                for (int z = 1; z <= std::min(q.nc[2], tile_max(3, 2)); ++z)
                    for (int y = 1; y <= std::min(q.nc[1], tile_max(3, 1)); ++y)
                        for (int x = 1; x <= std::min(q.nc[0], tile_max(3, 0)); ++x) {
                            const double halo = (x + 2.0) * (y + 2.0) * (z + 2.0) * rho_c;
                            const bool unit = x == 1 && y == 1 && z == 1;
                            if ((halo > cap || tiles_of(x, y, z) < min_tiles) && !unit)
                                continue;
                            const double own = std::max(1e-9, x * y * static_cast<double>(z) * rho_c);
                            const double passes = std::ceil((own + 2.0 * std::sqrt(own)) / MTPT_TILE_LANES);
                            const double cost = (passes * MTPT_TILE_LANES + 0.02 * halo + 25.0) / own;
                            if (best == 0.0 || cost < best) {
                                best = cost;
                                tx = x;
                                ty = y;
                                tz = z;
                            }
                        }
            }
            t[0] = tx;
            t[1] = ty;
            t[2] = tz;
        };
        // the row-sum pass stages positions only (its capacity is that of the
        // one-species transfer pass); the transfer pass stages row sums and
        // every species too
        choose(tile_capacity(q.dim, q.prec, 1), q.tile);
        choose(tile_capacity(q.dim, q.prec, q.ns), q.ttile);
        auto count = [&](const int* t, uint32_t* txs, uint32_t* tys) {
            *txs = static_cast<uint32_t>((q.nc[0] + t[0] - 1) / t[0]);
            *tys = static_cast<uint32_t>((q.nc[1] + t[1] - 1) / t[1]);
            return *txs * *tys * static_cast<uint32_t>(q.dim == 3 ? (q.nc[2] + t[2] - 1) / t[2] : 1);
        };
        q.ntiles = count(q.tile, &q.tiles_x, &q.tiles_y);
        q.nttiles = count(q.ttile, &q.ttiles_x, &q.ttiles_y);
        // rows of three cells long enough that trimming them to the x-window
        // saves more candidates than its two binary searches cost
        q.trim_rows = !q.tensor && 3.0 * rho_c >= MTPT_TRIM_MIN_ROW;
    }
    const size_t n = static_cast<size_t>(q.n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    for (int k = 0; k < 3; ++k)
        q.off_x[k] = k < q.dim ? take(n * q.tsz) : 0;
    for (int k = 0; k < 3; ++k)
        q.off_xt[k] = k < q.dim ? take(n * q.tsz) : 0;
    for (int k = 0; k < 3; ++k)
        q.off_jmp[k] = k < q.dim ? take(n * q.tsz) : 0;
    for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 3; ++c)
            q.off_m[b][c] = c < q.ns ? take(n * q.msz) : 0;
    q.off_p[0] = take(n * 4);
    q.off_p[1] = take(n * 4);
    q.off_s = take(n * q.tsz);
    q.off_cell = take(n * 4);
    q.off_rank = take(n * 4);
    q.off_perm = take(n * 4);
    q.off_cmask = take(n * 8 * (q.dim == 3 ? 3 : 1));
    if (q.trim_rows)
        q.off_cwin = take(n * 8 * (q.dim == 3 ? 3 : 1));
    const size_t padded = static_cast<size_t>(q.scan_blocks) * kScanTile;
    q.off_counts = take(padded * 4);
    q.off_tcounts = take(padded * 4);
    q.off_starts = take(padded * 4);
    q.off_bsum = take(static_cast<size_t>(q.scan_blocks) * 4);
    q.off_part = take(static_cast<size_t>(std::max<uint32_t>(std::max(q.part_blocks, q.nttiles), 1)) * 3 * 8);
    q.off_pair = take(static_cast<size_t>(std::max<uint32_t>(q.ntiles, 1)) * 4);
    q.off_stats = take(sizeof(DevStats));
    q.bytes = off;
    return q;
}

struct PhaseEv {
    int phase;
    hipEvent_t a, b;
};

}  // namespace

struct mtpt_sim {
    mtpt_params p{};
    Tensor tens;              // dispersion tensor (isotropic: tens.on == false)
    int device = 0;           // the HIP device current at create
    Plan q;
    Alloc alloc;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* base = nullptr;
    void* X[3]{};
    void* XT[3]{};
    void* J[3]{};
    void* M[2][3]{};
    uint32_t* P[2]{};
    void* S = nullptr;
    uint32_t *cell = nullptr, *rank = nullptr, *perm = nullptr, *counts = nullptr, *tcounts = nullptr,
             *starts = nullptr, *bsum = nullptr;
    uint64_t* cmask = nullptr;
    uint64_t* cwin = nullptr;
    double* partials = nullptr;
    uint32_t* pair_part = nullptr;
    DevStats* st = nullptr;
    int64_t steps_done = 0;   // steps enqueued since create
    bool moving = false;
    bool s_valid = false;
    bool bin_ready = false;   // the last transfer already binned for this step
    // the last step's totals and counters (PH_FINALIZE) are enqueued with the
    // next step's place launch, or on their own before anything reads them
    bool fin_pending = false;
    SimArgs fin_args{};
    double mass_initial[3]{};
    bool mass_initial_known = false;   // else in DevStats.initial
    hipEvent_t done_ev = nullptr;      // serving: recorded behind the sim's last step
    // profiling
    bool profiling = false;
    std::vector<PhaseEv> evs;
    double ph_ms[PH_COUNT]{};
    int64_t ph_n[PH_COUNT]{};
    // pool bookkeeping
    int64_t steps_target = -1;
};

namespace {

void carve(mtpt_sim* s)
{
    const Plan& q = s->q;
    char* b = s->base;
    for (int k = 0; k < 3; ++k) {
        s->X[k] = k < q.dim ? b + q.off_x[k] : nullptr;
        s->XT[k] = k < q.dim ? b + q.off_xt[k] : nullptr;
        s->J[k] = k < q.dim ? b + q.off_jmp[k] : nullptr;
    }
    for (int bb = 0; bb < 2; ++bb)
        for (int c = 0; c < 3; ++c)
            s->M[bb][c] = c < q.ns ? b + q.off_m[bb][c] : nullptr;
    s->P[0] = reinterpret_cast<uint32_t*>(b + q.off_p[0]);
    s->P[1] = reinterpret_cast<uint32_t*>(b + q.off_p[1]);
    s->S = b + q.off_s;
    s->cell = reinterpret_cast<uint32_t*>(b + q.off_cell);
    s->rank = reinterpret_cast<uint32_t*>(b + q.off_rank);
    s->perm = reinterpret_cast<uint32_t*>(b + q.off_perm);
    s->counts = reinterpret_cast<uint32_t*>(b + q.off_counts);
    s->tcounts = reinterpret_cast<uint32_t*>(b + q.off_tcounts);
    s->cmask = reinterpret_cast<uint64_t*>(b + q.off_cmask);
    s->cwin = q.trim_rows ? reinterpret_cast<uint64_t*>(b + q.off_cwin) : nullptr;
    s->starts = reinterpret_cast<uint32_t*>(b + q.off_starts);
    s->bsum = reinterpret_cast<uint32_t*>(b + q.off_bsum);
    s->partials = reinterpret_cast<double*>(b + q.off_part);
    s->pair_part = reinterpret_cast<uint32_t*>(b + q.off_pair);
    s->st = reinterpret_cast<DevStats*>(b + q.off_stats);
}

// SimArgs with every constant filled; buffer roles are set by the caller.
SimArgs base_args(const mtpt_sim* s)
{
    const Plan& q = s->q;
    const mtpt_params& p = s->p;
    SimArgs a{};
    a.n = q.n;
    a.ns = q.ns;
    a.moving = s->moving ? 1 : 0;
    for (int k = 0; k < 3; ++k) {
        a.glo[k] = p.lo[k];
        a.inv_side[k] = q.inv_side[k];
        a.nc[k] = q.nc[k];
        a.lo[k] = p.lo[k];
        a.hi[k] = p.hi[k];
        a.lof[k] = static_cast<float>(p.lo[k]);
        a.hif[k] = static_cast<float>(p.hi[k]);
    }
    a.ncells = q.ncells;
    a.tile[0] = q.tile[0];
    a.tile[1] = q.tile[1];
    a.tile[2] = q.tile[2];
    a.tiles_x = q.tiles_x;
    a.tiles_y = q.tiles_y;
    a.ntiles = q.ntiles;
    for (int k = 0; k < 3; ++k)
        a.ttile[k] = q.ttile[k];
    a.ttiles_x = q.ttiles_x;
    a.ttiles_y = q.ttiles_y;
    a.nttiles = q.nttiles;
    a.trim_rows = q.trim_rows ? 1 : 0;
    a.sdev = std::sqrt(2.0 * p.d_rw * p.dt);
    for (int k = 0; k < 3; ++k)
        a.drift[k] = k < q.dim ? p.vel[k] * p.dt : 0.0;
    a.seed = p.seed;
    a.psi = q.psi;
    a.psi2 = q.psi * q.psi;
    a.win = q.psi * std::sqrt(s->tens.t[0]) * (1.0 + 1e-6);
    a.win2d = a.win * a.win;
    a.win2f = static_cast<float>(a.win2d);
    {
        // rounding margin of the per-row windows: 8 ulps of the largest
        // coordinate plus 8 ulps of the window, in the type of the positions
        double xmax = 0.0;
        for (int k = 0; k < q.dim; ++k)
            xmax = std::max(xmax, std::max(std::fabs(p.lo[k]), std::fabs(p.hi[k])));
        const int e = xmax > 0.0 ? std::ilogb(xmax) : 0;
        a.wmarginf = static_cast<float>(8.0 * std::ldexp(1.0, e - 23) + 8.0 * 1.1920928955078125e-7 * a.win);
        a.wmargind = 8.0 * std::ldexp(1.0, e - 52) + 8.0 * 2.220446049250313e-16 * a.win;
    }
    for (int k = 0; k < 3; ++k)
        a.side[k] = q.inv_side[k] > 0.0 ? 1.0 / q.inv_side[k] : 0.0;
    // relative band of the FP32 cutoff test: the isotropic FP32 r^2 is within
    // 1e-6 of the FP64 one; the FP32 Mahalanobis form within
    // (10 sqrt(cond) + 3) 2^-24, cond = trace(T^-1) trace(T), with a factor 4 of margin
    const double band = s->tens.on ? std::max(1e-5, 4.0 * (10.0 * std::sqrt(s->tens.cond) + 3.0) * 5.960464477539063e-08)
                                   : 1e-5;
    a.psi2_in = static_cast<float>(a.psi2 * (1.0 - band));
    a.psi2_out = static_cast<float>(a.psi2 * (1.0 + band));
    a.tensor = s->tens.on ? 1 : 0;
    for (int k = 0; k < 6; ++k) {
        a.lch[k] = s->tens.l[k];
        a.minv[k] = s->tens.m[k];
        a.minvf[k] = static_cast<float>(s->tens.m[k]);
    }
    a.kc = p.beta / (4.0 * p.d_mt * p.dt);
    a.kcf = static_cast<float>(a.kc);
    a.kcf2 = static_cast<float>(-a.kc * 1.4426950408889634);
    a.beta = p.beta;
    a.betaf = static_cast<float>(p.beta);
    a.k_react = p.k_react;
    double vol = 1.0;
    for (int k = 0; k < q.dim; ++k)
        vol *= p.hi[k] - p.lo[k];
    a.to_c = q.n > 0 ? static_cast<double>(q.n) / vol : 0.0;
    a.to_m = q.n > 0 ? vol / static_cast<double>(q.n) : 0.0;
    a.dt = p.dt;
    for (int k = 0; k < 3; ++k) {
        a.x[k] = s->X[k];
        a.xt[k] = s->XT[k];
        a.jmp[k] = s->J[k];
    }
    a.srow = s->S;
    a.cell = s->cell;
    a.rank = s->rank;
    a.perm = s->perm;
    a.counts = s->counts;
    a.tcounts = s->tcounts;
    a.cmask = s->cmask;
    a.cwin = s->cwin;
    a.starts = s->starts;
    a.bsum = s->bsum;
    a.partials = s->partials;
    a.pair_part = s->pair_part;
    a.st = s->st;
    a.scan_blocks = q.scan_blocks;
    a.scan_fold = q.scan_blocks <= kScanFold ? 1 : 0;
    a.part_blocks = q.part_blocks;
    return a;
}

// Current sorted pids and masses after steps_done steps.
//   moving sims: the gather alternates the pid buffers (P[t&1] current) and
//     the masses go M0 -> (gather) M1 -> (transfer) M0;
//   static sims: binned once at create (P0), the masses alternate M[t&1].
uint32_t* cur_pid(const mtpt_sim* s) { return s->moving ? s->P[s->steps_done & 1] : s->P[0]; }
void* const* cur_mass(const mtpt_sim* s) { return s->moving ? s->M[0] : s->M[s->steps_done & 1]; }

// Arguments of step number steps_done (0-based since create).
SimArgs step_args(const mtpt_sim* s, bool* rowsum_needed)
{
    SimArgs a = base_args(s);
    const int64_t t = s->steps_done;
    a.step = s->p.start_step + t;
    a.walk = s->moving ? 1 : 0;
    if (s->moving) {
        a.pid_src = s->P[t & 1];
        a.pid_dst = s->P[(t + 1) & 1];
        for (int c = 0; c < 3; ++c) {
            a.m_src[c] = s->M[0][c];
            a.m_mid[c] = s->M[1][c];
            a.m_dst[c] = s->M[0][c];
        }
        a.recompute_s = 1;
        // the row-sum pass (run every step of a moving sim) moves the three
        // species' masses instead of the place pass (measured on the 3.2e7-
        // particle reacting workload: place 0.92 -> 0.64 ms, row-sum 1.27 ->
        // 1.45 ms; with one species the row-sum pass lost more than the place
        // pass gained: 4e6-particle 2-d step 0.271 -> 0.279 ms)
        a.src_slot = s->q.ns == 3 ? s->cell : nullptr;
    } else {
        a.pid_src = s->P[0];
        a.pid_dst = s->P[0];
        for (int c = 0; c < 3; ++c) {
            a.m_src[c] = s->M[t & 1][c];
            a.m_mid[c] = s->M[t & 1][c];
            a.m_dst[c] = s->M[(t + 1) & 1][c];
        }
        a.recompute_s = s->s_valid ? 0 : 1;
    }
    a.fuse_bin = s->moving ? 1 : 0;
    a.tcounts_valid = (s->moving && s->bin_ready) ? 1 : 0;
    *rowsum_needed = a.recompute_s != 0;
    return a;
}

// Launch one phase of a sim; with prev (PH_PLACE only) the same launch also
// finalizes the step that prev describes.
int launch(mtpt_sim* s, int ph, const SimArgs& a, const SimArgs* prev = nullptr)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s->profiling) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, s->stream));
    }
    if (prev)
        HIP_TRY(launch_place_fin(s->q.dim, s->q.prec, a, *prev, s->stream));
    else
        HIP_TRY(launch_phase(ph, s->q.dim, s->q.prec, a, s->stream));
    if (s->profiling) {
        HIP_TRY(hipEventRecord(e1, s->stream));
        s->evs.push_back({ph, e0, e1});
    }
    return MTPT_OK;
}

// The pending finalize, on its own.
int flush_finalize(mtpt_sim* s)
{
    if (!s->fin_pending)
        return MTPT_OK;
    s->fin_pending = false;
    return launch(s, PH_FINALIZE, s->fin_args);
}

// Binning; the bin phase itself is skipped when the previous transfer pass
// already walked and binned every particle for this step.  With prev, the
// place launch also finalizes the step that prev describes (before this
// step's row-sum and transfer passes rewrite its partial sums).
int enqueue_binning(mtpt_sim* s, const SimArgs& a, bool with_bin, const SimArgs* prev = nullptr)
{
    static const int phases[] = {PH_BIN, PH_SCAN_REDUCE, PH_SCAN_TOP, PH_SCAN_DOWN,
                                 PH_SCATTER, PH_PLACE};
    for (int ph : phases) {
        if (ph == PH_BIN && !with_bin)
            continue;
        if (ph == PH_SCAN_TOP && a.scan_fold)
            continue;
        const int rc = launch(s, ph, a, ph == PH_PLACE ? prev : nullptr);
        if (rc)
            return rc;
    }
    return MTPT_OK;
}

int enqueue_step(mtpt_sim* s)
{
    bool need_rowsum = false;
    SimArgs a = step_args(s, &need_rowsum);
    // the previous step's finalize joins this step's place launch when the
    // step has one (a moving sim whose particles are binned)
    const bool merge = s->fin_pending && s->moving && s->bin_ready;
    if (s->fin_pending && !merge) {
        const int rc = flush_finalize(s);
        if (rc)
            return rc;
    }
    if (s->moving) {
        const SimArgs prev = s->fin_args;
        s->fin_pending = false;
        const int rc = enqueue_binning(s, a, !s->bin_ready, merge ? &prev : nullptr);
        if (rc)
            return rc;
    }
    if (need_rowsum) {
        const int rc = launch(s, PH_ROWSUM, a);
        if (rc)
            return rc;
    }
    const int rc = launch(s, PH_TRANSFER, a);
    if (rc)
        return rc;
    s->fin_args = a;
    s->fin_pending = true;
    s->steps_done += 1;
    if (!s->moving)
        s->s_valid = true;
    else
        s->bin_ready = true;
    return MTPT_OK;
}

int sync(mtpt_sim* s)
{
    const int rc = flush_finalize(s);
    if (rc)
        return rc;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return MTPT_OK;
}

int collect_events(mtpt_sim* s)
{
    for (auto& e : s->evs) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
        s->ph_ms[e.phase] += ms;
        s->ph_n[e.phase] += 1;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    s->evs.clear();
    return MTPT_OK;
}

void release(mtpt_sim* s)
{
    if (!s)
        return;
    for (auto& e : s->evs) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    s->evs.clear();
    s->alloc.put(s->base);
    s->base = nullptr;
    if (s->done_ev)
        (void)hipEventDestroy(s->done_ev);
    if (s->own_stream && s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
}

// Pinned host staging of one admission (serving pool): reused once the
// event recorded behind its copies has fired.
struct PinnedStage {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool armed = false;
};

// Upload inputs and bin them (the state at step 0).  Positions (and Kahan
// masses) are converted on the host into staging; the pids are filled on the
// device; the binning, the initial totals and their copy into DevStats.initial
// are enqueued on the sim's stream.  Without st (mtpt_create) the staging is
// pageable, the copies block, and create waits for the binning and reads the
// initial totals.  With st (pool admission) the staging is pinned, the copies
// are asynchronous, the event st->ev is recorded behind them, and nothing
// waits: the initial totals are read when the statistics are first asked for.
int create_into(mtpt_sim* s, const double* pos, const double* mass, PinnedStage* st = nullptr)
{
    const Plan& q = s->q;
    const size_t n = static_cast<size_t>(q.n);
    HIP_TRY(hipMemsetAsync(s->st, 0, sizeof(DevStats), s->stream));
    HIP_TRY(hipMemsetAsync(s->counts, 0, static_cast<size_t>(q.scan_blocks) * kScanTile * 4, s->stream));
    HIP_TRY(hipMemsetAsync(s->tcounts, 0, static_cast<size_t>(q.scan_blocks) * kScanTile * 4, s->stream));
    if (n > 0) {
        std::vector<unsigned char> pageable;
        unsigned char* stage = nullptr;
        if (st) {
            stage = static_cast<unsigned char*>(st->host);
        } else {
            pageable.resize(std::max(n * q.tsz, n * q.msz));
            stage = pageable.data();
        }
        // the pinned staging holds every array at once: [dim][n] positions, then
        // [ns][n] masses; the pageable one one array at a time
        size_t off = 0;
        auto upload = [&](void* dst, size_t bytes, const unsigned char* src) -> hipError_t {
            return st ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream)
                      : hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        };
        for (int k = 0; k < q.dim; ++k) {
            // coordinate k, rounded once to the position type
            unsigned char* h = stage + off;
            if (q.tsz == 8) {
                double* d = reinterpret_cast<double*>(h);
                for (size_t i = 0; i < n; ++i)
                    d[i] = pos[i * q.dim + k];
            } else {
                float* f = reinterpret_cast<float*>(h);
                for (size_t i = 0; i < n; ++i)
                    f[i] = static_cast<float>(pos[i * q.dim + k]);
            }
            HIP_TRY(upload(s->X[k], n * q.tsz, h));
            if (st)
                off += n * q.tsz;
        }
        for (int c = 0; c < q.ns; ++c) {
            unsigned char* h = stage + off;
            if (q.msz == 8) {
                if (st) {
                    std::memcpy(h, mass + c * n, n * 8);
                    HIP_TRY(upload(s->M[1][c], n * 8, h));
                } else {
                    HIP_TRY(hipMemcpy(s->M[1][c], mass + c * n, n * 8, hipMemcpyHostToDevice));
                }
            } else {
                float* f = reinterpret_cast<float*>(h);
                for (size_t i = 0; i < n; ++i)
                    f[i] = static_cast<float>(mass[c * n + i]);
                HIP_TRY(upload(s->M[1][c], n * 4, h));
            }
            if (st)
                off += n * q.msz;
        }
        HIP_TRY(launch_iota(s->P[1], q.n, s->stream));
        // initial binning: positions in pid order, no jump; pids P1 -> P0,
        // masses M1 -> M0
        SimArgs a = base_args(s);
        a.walk = 0;
        a.step = s->p.start_step;
        a.pid_src = s->P[1];
        a.pid_dst = s->P[0];
        for (int c = 0; c < 3; ++c) {
            a.m_src[c] = s->M[1][c];
            a.m_mid[c] = s->M[0][c];
            a.m_dst[c] = s->M[0][c];
        }
        const int rc = enqueue_binning(s, a, true);
        if (rc)
            return rc;
        HIP_TRY(launch_totals(q.prec, a, s->M[0], s->stream));
        HIP_TRY(hipMemcpyAsync(&s->st->initial[0], &s->st->totals[0], sizeof(double) * 3,
                               hipMemcpyDeviceToDevice, s->stream));
    }
    if (st) {
        HIP_TRY(hipEventRecord(st->ev, s->stream));
        st->armed = true;
        s->mass_initial_known = false;
        return MTPT_OK;
    }
    const int rc = sync(s);
    if (rc)
        return rc;
    if (s->profiling)
        collect_events(s);
    DevStats h{};
    HIP_TRY(hipMemcpy(&h, s->st, sizeof h, hipMemcpyDeviceToHost));
    for (int c = 0; c < 3; ++c)
        s->mass_initial[c] = c < q.ns ? h.totals[c] : 0.0;
    s->mass_initial_known = true;
    return MTPT_OK;
}

int check_inputs(const mtpt_params& p, const double* pos, const double* mass)
{
    if (p.n > 0 && (!pos || !mass))
        return fail(MTPT_E_ARG, "pos and mass must not be NULL when n > 0");
    for (int64_t i = 0; i < p.n; ++i)
        for (int k = 0; k < p.dim; ++k) {
            const double v = pos[i * p.dim + k];
            if (!(v >= p.lo[k] && v <= p.hi[k]))
                return fail(MTPT_E_ARG, "particle %lld coordinate %d = %g outside [%g, %g]",
                            (long long)i, k, v, p.lo[k], p.hi[k]);
        }
    for (int64_t i = 0; i < p.n * p.n_species; ++i)
        if (!std::isfinite(mass[i]))
            return fail(MTPT_E_ARG, "mass %lld is not finite", (long long)i);
    return MTPT_OK;
}

int new_sim(const mtpt_params* params, const double* pos, const double* mass, void* hip_stream,
            const mtpt_allocator* alloc, mtpt_sim** out, PinnedStage* st = nullptr)
{
    int rc = validate(params);
    if (rc)
        return rc;
    rc = check_inputs(*params, pos, mass);
    if (rc)
        return rc;
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(MTPT_E_ARG, "allocator needs both alloc and free");
    mtpt_sim* s = new mtpt_sim();
    s->p = *params;
    {
        const char* why = "";
        (void)tensor_of(s->p, &s->tens, &why);   // validated above
    }
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(MTPT_E_DEVICE, "hipGetDevice failed");
    }
    s->q = make_plan(s->p);
    s->moving = s->p.d_rw > 0.0;
    for (int k = 0; k < params->dim; ++k)
        s->moving = s->moving || s->p.vel[k] != 0.0;
    if (alloc) {
        s->alloc.a = *alloc;
        s->alloc.custom = true;
    }
    if (hip_stream) {
        s->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return fail(MTPT_E_DEVICE, "hipStreamCreateWithFlags failed");
        }
        s->own_stream = true;
    }
    s->base = static_cast<char*>(s->alloc.get(s->q.bytes));
    if (!s->base) {
        release(s);
        return fail(MTPT_E_NOMEM, "device allocation of %zu bytes failed", s->q.bytes);
    }
    carve(s);
    rc = create_into(s, pos, mass, st);
    if (rc) {
        std::string msg = g_err;
        (void)hipStreamSynchronize(s->stream);
        release(s);
        g_err = msg;
        return rc;
    }
    *out = s;
    return MTPT_OK;
}

}  // namespace

// ====================================================================== C-ABI
extern "C" {

const char* mtpt_last_error(void) { return g_err.c_str(); }

int mtpt_abi_version(void) { return MTPT_ABI_VERSION; }

int mtpt_sim_bytes(const mtpt_params* params, size_t* bytes)
{
    const int rc = validate(params);
    if (rc)
        return rc;
    if (!bytes)
        return fail(MTPT_E_ARG, "bytes is NULL");
    *bytes = make_plan(*params).bytes;
    return MTPT_OK;
}

int mtpt_create(const mtpt_params* params, const double* pos, const double* mass, void* hip_stream,
                const mtpt_allocator* alloc, mtpt_sim** out)
{
    if (!out)
        return fail(MTPT_E_ARG, "out is NULL");
    *out = nullptr;
    return new_sim(params, pos, mass, hip_stream, alloc, out);
}

int mtpt_step(mtpt_sim* s, int64_t n_steps)
{
    if (!s)
        return fail(MTPT_E_ARG, "sim is NULL");
    if (n_steps < 0)
        return fail(MTPT_E_ARG, "n_steps must be >= 0");
    if (s->q.n == 0) {
        s->steps_done += n_steps;
        return MTPT_OK;
    }
    for (int64_t k = 0; k < n_steps; ++k) {
        const int rc = enqueue_step(s);
        if (rc)
            return rc;
    }
    return MTPT_OK;
}

int mtpt_masses(mtpt_sim* s, double* out)
{
    if (!s || (!out && s->q.n > 0))
        return fail(MTPT_E_ARG, "NULL argument");
    const size_t n = static_cast<size_t>(s->q.n);
    if (n == 0)
        return MTPT_OK;
    const size_t bytes = n * s->q.ns * 8;
    // the totals of the last step decide MTPT_E_NONFINITE below
    const int rf = flush_finalize(s);
    if (rf)
        return rf;
    double* d = static_cast<double*>(s->alloc.get(bytes));
    if (!d)
        return fail(MTPT_E_NOMEM, "staging allocation failed");
    SimArgs a = base_args(s);
    hipError_t e = launch_unpermute_mass(s->q.prec, a, cur_mass(s), cur_pid(s), d, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s->stream);
    s->alloc.put(d);
    if (e != hipSuccess)
        return fail(MTPT_E_DEVICE, "mtpt_masses: %s", hipGetErrorString(e));
    DevStats h{};
    HIP_TRY(hipMemcpy(&h, s->st, sizeof h, hipMemcpyDeviceToHost));
    if (h.nonfinite)
        return fail(MTPT_E_NONFINITE, "a mass total became non-finite");
    return MTPT_OK;
}

int mtpt_positions(mtpt_sim* s, double* out)
{
    if (!s || (!out && s->q.n > 0))
        return fail(MTPT_E_ARG, "NULL argument");
    const size_t n = static_cast<size_t>(s->q.n);
    if (n == 0)
        return MTPT_OK;
    const size_t bytes = n * s->q.dim * 8;
    double* d = static_cast<double*>(s->alloc.get(bytes));
    if (!d)
        return fail(MTPT_E_NOMEM, "staging allocation failed");
    SimArgs a = base_args(s);
    hipError_t e = launch_unpermute_pos(s->q.dim, s->q.prec, a, cur_pid(s), d, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s->stream);
    s->alloc.put(d);
    if (e != hipSuccess)
        return fail(MTPT_E_DEVICE, "mtpt_positions: %s", hipGetErrorString(e));
    return MTPT_OK;
}

int mtpt_stats(mtpt_sim* s, mtpt_stats_t* out)
{
    if (!s || !out)
        return fail(MTPT_E_ARG, "NULL argument");
    int rc = sync(s);
    if (rc)
        return rc;
    DevStats h{};
    HIP_TRY(hipMemcpy(&h, s->st, sizeof h, hipMemcpyDeviceToHost));
    if (!s->mass_initial_known) {
        for (int c = 0; c < 3; ++c)
            s->mass_initial[c] = c < s->q.ns ? h.initial[c] : 0.0;
        s->mass_initial_known = true;
    }
    std::memset(out, 0, sizeof *out);
    out->steps_done = s->steps_done;
    out->pairs_last = static_cast<int64_t>(h.pairs_last);
    out->pairs_total = h.pairs_total;
    for (int c = 0; c < 3; ++c) {
        const bool on = c < s->q.ns && s->q.n > 0;
        out->mass_total[c] = on ? (s->steps_done > 0 ? h.totals[c] : s->mass_initial[c]) : 0.0;
        out->mass_initial[c] = on ? s->mass_initial[c] : 0.0;
    }
    // drift of the conserved quantities: each species without reaction;
    // A + C and B + C when A + B -> C runs
    double drift = 0.0;
    auto rel = [](double now, double init) {
        return init != 0.0 ? std::fabs(now - init) / std::fabs(init) : std::fabs(now);
    };
    if (s->q.ns == 3 && s->p.k_react > 0.0) {
        const double* t = out->mass_total;
        const double* i0 = out->mass_initial;
        drift = std::max(rel(t[0] + t[2], i0[0] + i0[2]), rel(t[1] + t[2], i0[1] + i0[2]));
    } else {
        for (int c = 0; c < s->q.ns; ++c)
            drift = std::max(drift, rel(out->mass_total[c], out->mass_initial[c]));
    }
    out->drift = drift;
    out->nonfinite = h.nonfinite;
    out->n_cells = static_cast<int32_t>(s->q.ncells);
    return MTPT_OK;
}

}  // extern "C"

namespace {

// CSR export in pid order: count(rowcnt) fills rowcnt[pid] with each row's
// length, fill(row_ptr, col) writes the rows (sorted ascending) from device
// row offsets.  Scratch comes from the sim's allocator.
// Device scratch of a CSR export: from the sim's allocator, or carved in
// order from one fixed buffer (base != nullptr; nothing is allocated or
// freed then, and a request beyond its size fails).
struct CsrScratch {
    mtpt_sim* s;
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    void* get(size_t bytes)
    {
        if (!base)
            return s->alloc.get(bytes);
        const size_t need = align_up(used, 256) + bytes;
        if (need > size)
            return nullptr;
        void* p = base + align_up(used, 256);
        used = need;
        return p;
    }
    void put(void* p)
    {
        if (!base)
            s->alloc.put(p);
    }
};

// Bytes of fixed scratch a CSR export of n rows and nnz entries needs.
size_t csr_scratch_bytes(int64_t n, int64_t nnz)
{
    const size_t tiles = static_cast<size_t>((n + 1 + kScanTile - 1) / kScanTile);
    return align_up(static_cast<size_t>(n) * 4, 256) + align_up(tiles * kScanTile * 4, 256) +
           align_up(tiles * 4, 256) + align_up(static_cast<size_t>(n + 1) * 8, 256) +
           static_cast<size_t>(nnz) * 8;
}

template <typename Count, typename Fill>
int csr_export(mtpt_sim* s, int64_t* row_ptr, int64_t* col, int64_t cap, int64_t* nnz_out, Count count,
               Fill fill, char* fixed = nullptr, size_t fixed_bytes = 0)
{
    const int64_t n = s->q.n;
    const int64_t tiles = (n + 1 + kScanTile - 1) / kScanTile;
    CsrScratch sc{s, fixed, fixed_bytes};
    uint32_t* rowcnt = static_cast<uint32_t*>(sc.get(static_cast<size_t>(n) * 4));
    uint32_t* tmp = static_cast<uint32_t*>(sc.get(static_cast<size_t>(tiles) * kScanTile * 4));
    uint32_t* bs = static_cast<uint32_t*>(sc.get(static_cast<size_t>(tiles) * 4));
    int64_t* drp = static_cast<int64_t*>(sc.get(static_cast<size_t>(n + 1) * 8));
    int64_t* dcol = nullptr;
    int rc = MTPT_OK;
    hipError_t e = hipSuccess;
    if (!rowcnt || !tmp || !bs || !drp) {
        rc = fixed ? fail(MTPT_E_ARG, "neighbour export of %lld rows needs %zu bytes of scratch, more than the "
                                      "static scratch's %zu", (long long)n, csr_scratch_bytes(n, 0), fixed_bytes)
                   : fail(MTPT_E_NOMEM, "neighbour export allocation failed");
        goto done;
    }
    {
        e = count(rowcnt);
        if (e == hipSuccess)
            e = launch_scan_u32_to_i64(rowcnt, drp, n, tmp, bs, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(row_ptr, drp, static_cast<size_t>(n + 1) * 8, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) {
            rc = fail(MTPT_E_DEVICE, "neighbour export: %s", hipGetErrorString(e));
            goto done;
        }
        const int64_t nnz = row_ptr[n];
        *nnz_out = nnz;
        if (col && nnz <= cap && nnz > 0) {
            dcol = static_cast<int64_t*>(sc.get(static_cast<size_t>(nnz) * 8));
            if (!dcol) {
                rc = fixed ? fail(MTPT_E_ARG, "neighbour export of %lld entries needs %zu bytes of scratch, more "
                                              "than the static scratch's %zu (row_ptr is written)",
                                  (long long)nnz, csr_scratch_bytes(n, nnz), fixed_bytes)
                           : fail(MTPT_E_NOMEM, "neighbour export allocation failed");
                goto done;
            }
            e = fill(drp, dcol);
            if (e == hipSuccess)
                e = hipMemcpyAsync(col, dcol, static_cast<size_t>(nnz) * 8, hipMemcpyDeviceToHost, s->stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess)
                rc = fail(MTPT_E_DEVICE, "neighbour export: %s", hipGetErrorString(e));
        }
    }
done:
    (void)hipStreamSynchronize(s->stream);
    sc.put(rowcnt);
    sc.put(tmp);
    sc.put(bs);
    sc.put(drp);
    sc.put(dcol);
    return rc;
}

// ------------------------------------------------------------ static scratch
// Device scratch of mtpt_neighbors_static: one file-scope array, of which
// every GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name except to look its address up:
// hipGetSymbolAddress, once per device with that device current; the
// address is kept per device and passed to the kernels like any buffer.
constexpr size_t kStaticScratchBytes = static_cast<size_t>(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's address of the array (device: the sim's device).
int static_scratch(int device, char** out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(MTPT_E_DEVICE, "device %d beyond the static scratch's table", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != device)
            HIP_TRY(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device)
            (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(MTPT_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<char*>(g_scratch_ptr[device]);
    return MTPT_OK;
}

hipError_t export_pass(const mtpt_sim* s, int ph, const SimArgs& a)
{
    const int prec = s->q.prec, ns = s->q.ns;
    if (s->q.dim == 2)
        return s->tens.on ? launch_tiles_export<2, true>(ph, prec, ns, a, s->stream)
                          : launch_tiles_export<2, false>(ph, prec, ns, a, s->stream);
    return s->tens.on ? launch_tiles_export<3, true>(ph, prec, ns, a, s->stream)
                      : launch_tiles_export<3, false>(ph, prec, ns, a, s->stream);
}

}  // namespace

extern "C" {

int mtpt_neighbors(mtpt_sim* s, int64_t* row_ptr, int64_t* col, int64_t cap, int64_t* nnz_out)
{
    if (!s || !row_ptr || !nnz_out)
        return fail(MTPT_E_ARG, "NULL argument");
    row_ptr[0] = 0;
    *nnz_out = 0;
    if (s->q.n == 0)
        return MTPT_OK;
    const SimArgs a = base_args(s);
    const int dim = s->q.dim, prec = s->q.prec;
    const uint32_t* pid = cur_pid(s);
    return csr_export(
        s, row_ptr, col, cap, nnz_out,
        [&](uint32_t* rowcnt) { return launch_nb_count(dim, prec, a, pid, rowcnt, s->stream); },
        [&](const int64_t* drp, int64_t* dcol) { return launch_nb_fill(dim, prec, a, pid, drp, dcol, s->stream); });
}

int mtpt_neighbors_static(mtpt_sim* s, int64_t* row_ptr, int64_t* col, int64_t cap, int64_t* nnz_out)
{
    if (!s || !row_ptr || !nnz_out)
        return fail(MTPT_E_ARG, "NULL argument");
    row_ptr[0] = 0;
    *nnz_out = 0;
    if (s->q.n == 0)
        return MTPT_OK;
    if (csr_scratch_bytes(s->q.n, 0) > kStaticScratchBytes)
        return fail(MTPT_E_ARG, "neighbour export of %lld rows needs %zu bytes of scratch, more than the "
                                "static scratch's %zu", (long long)s->q.n, csr_scratch_bytes(s->q.n, 0),
                    kStaticScratchBytes);
    char* base = nullptr;
    const int rc = static_scratch(s->device, &base);
    if (rc)
        return rc;
    const SimArgs a = base_args(s);
    const int dim = s->q.dim, prec = s->q.prec;
    const uint32_t* pid = cur_pid(s);
    return csr_export(
        s, row_ptr, col, cap, nnz_out,
        [&](uint32_t* rowcnt) { return launch_nb_count(dim, prec, a, pid, rowcnt, s->stream); },
        [&](const int64_t* drp, int64_t* dcol) { return launch_nb_fill(dim, prec, a, pid, drp, dcol, s->stream); },
        base, kStaticScratchBytes);
}

int mtpt_step_neighbors(mtpt_sim* s, int32_t which, int64_t* row_ptr, int64_t* col, int64_t cap,
                        int64_t* nnz_out)
{
    if (!s || !row_ptr || !nnz_out)
        return fail(MTPT_E_ARG, "NULL argument");
    if (which != 0 && which != 1)
        return fail(MTPT_E_ARG, "which must be 0 (row-sum pass) or 1 (transfer pass)");
    row_ptr[0] = 0;
    *nnz_out = 0;
    if (s->q.n == 0)
        return MTPT_OK;
    if (s->steps_done == 0)
        return fail(MTPT_E_STATE, "no step has run yet");
    // the last step's arguments: its sorted positions, cell offsets, row
    // sums, neighbour bits and windows are still in place until the next step
    SimArgs a = s->fin_args;
    const int ph = which == 0 ? PH_ROWSUM : PH_TRANSFER;
    const int64_t n = s->q.n;
    return csr_export(
        s, row_ptr, col, cap, nnz_out,
        [&](uint32_t* rowcnt) {
            a.nb_cnt = rowcnt;
            a.nb_row = nullptr;
            a.nb_col = nullptr;
            return export_pass(s, ph, a);
        },
        [&](const int64_t* drp, int64_t* dcol) {
            a.nb_cnt = nullptr;
            a.nb_row = drp;
            a.nb_col = dcol;
            hipError_t e = export_pass(s, ph, a);
            if (e == hipSuccess)
                e = launch_nb_sort(n, drp, dcol, s->stream);
            return e;
        });
}

int mtpt_destroy(mtpt_sim* s)
{
    if (!s)
        return MTPT_OK;
    (void)hipStreamSynchronize(s->stream);
    release(s);
    return MTPT_OK;
}

int mtpt_set_profiling(mtpt_sim* s, int32_t on)
{
    if (!s)
        return fail(MTPT_E_ARG, "sim is NULL");
    s->profiling = on != 0;
    return MTPT_OK;
}

int mtpt_phase_times(mtpt_sim* s, const char** names, double* ms, int64_t* launches, int32_t cap,
                     int32_t* count)
{
    if (!s || !count)
        return fail(MTPT_E_ARG, "NULL argument");
    int rc = sync(s);
    if (rc)
        return rc;
    rc = collect_events(s);
    if (rc)
        return rc;
    int32_t k = 0;
    for (int ph = 0; ph < PH_COUNT; ++ph) {
        if (s->ph_n[ph] == 0)
            continue;
        if (k < cap) {
            if (names)
                names[k] = phase_name(ph);
            if (ms)
                ms[k] = s->ph_ms[ph];
            if (launches)
                launches[k] = s->ph_n[ph];
        }
        ++k;
        s->ph_ms[ph] = 0.0;
        s->ph_n[ph] = 0;
    }
    *count = k;
    return MTPT_OK;
}

}  // extern "C"

// ==================================================================== serving
// A pool keeps independent simulations resident and advances all active ones
// together.  One tick enqueues, for every group of sims sharing (dim,
// precision, species, moving, row sums needed), one launch per phase that
// covers all sims of the group: block b of a launch finds its sim by binary
// search in a prefix of blocks per sim.  The per-tick argument arrays travel
// through a ring of pinned host buffers and device buffers; a ring slot is
// reused only after the event recorded behind its last launch has fired.
namespace {

struct RingSlot {
    void* host = nullptr;    // pinned
    void* dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool armed = false;
};

}  // namespace

struct mtpt_pool {
    size_t budget = 0;
    size_t held = 0;
    int32_t max_slots = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Alloc alloc;
    std::map<int64_t, mtpt_sim*> sims;   // ticket -> sim, ordered by admission
    std::map<int64_t, size_t> bytes_of;
    int64_t next_ticket = 1;
    RingSlot ring[4];
    int64_t ticks = 0;
    std::deque<PinnedStage> stages;      // admission staging (at most kStages)
    hipStream_t xstream = nullptr;       // exports of finished sims
};

namespace {

int ring_reserve(mtpt_pool* p, RingSlot& r, size_t bytes)
{
    if (r.armed) {
        HIP_TRY(hipEventSynchronize(r.ev));
        r.armed = false;
    }
    if (!r.ev)
        HIP_TRY(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
    if (r.cap >= bytes)
        return MTPT_OK;
    if (r.host)
        (void)hipHostFree(r.host);
    p->alloc.put(r.dev);
    r.host = nullptr;
    r.dev = nullptr;
    r.cap = 0;
    const size_t cap = align_up(std::max<size_t>(bytes, 65536), 4096);
    HIP_TRY(hipHostMalloc(&r.host, cap, hipHostMallocDefault));
    r.dev = p->alloc.get(cap);
    if (!r.dev)
        return fail(MTPT_E_NOMEM, "pool argument buffer allocation failed");
    r.cap = cap;
    return MTPT_OK;
}

// A pinned staging buffer of at least bytes whose previous copies have
// finished: a free one (grown if needed), else a new one while there are
// fewer than kStages, else the oldest once its copies are done.
constexpr size_t kStages = 4;
int stage_acquire(mtpt_pool* p, size_t bytes, PinnedStage** out)
{
    PinnedStage* pick = nullptr;
    for (auto& g : p->stages) {
        if (g.armed) {
            const hipError_t e = hipEventQuery(g.ev);
            if (e == hipErrorNotReady) {
                (void)hipGetLastError();
                continue;
            }
            if (e != hipSuccess)
                return fail(MTPT_E_DEVICE, "staging event: %s", hipGetErrorString(e));
            g.armed = false;
        }
        if (!pick || (pick->cap < bytes && g.cap >= bytes))
            pick = &g;
    }
    if (!pick && p->stages.size() < kStages) {
        p->stages.emplace_back();
        pick = &p->stages.back();
        HIP_TRY(hipEventCreateWithFlags(&pick->ev, hipEventDisableTiming));
    }
    if (!pick) {
        pick = &p->stages.front();
        HIP_TRY(hipEventSynchronize(pick->ev));
        pick->armed = false;
    }
    if (pick->cap < bytes) {
        if (pick->host)
            (void)hipHostFree(pick->host);
        pick->host = nullptr;
        pick->cap = 0;
        const size_t cap = align_up(std::max<size_t>(bytes, 1 << 20), 1 << 16);
        HIP_TRY(hipHostMalloc(&pick->host, cap, hipHostMallocDefault));
        pick->cap = cap;
    }
    *out = pick;
    return MTPT_OK;
}

// Run fn for sim s on the pool's export stream when s has finished (the
// stream first waits for the event behind s's last step, so that fn does not
// wait for the ticks of the other sims), else on the pool stream.
template <typename F>
int on_export_stream(mtpt_pool* p, mtpt_sim* s, F fn)
{
    if (!(s->done_ev && s->steps_done >= s->steps_target && p->xstream))
        return fn();
    HIP_TRY(hipStreamWaitEvent(p->xstream, s->done_ev, 0));
    hipStream_t keep = s->stream;
    s->stream = p->xstream;
    const int rc = fn();
    s->stream = keep;
    return rc;
}

struct GroupKey {
    int dim, prec, ns, tensor, moving, rowsum, bin;
    bool operator<(const GroupKey& o) const
    {
        if (dim != o.dim) return dim < o.dim;
        if (tensor != o.tensor) return tensor < o.tensor;
        if (prec != o.prec) return prec < o.prec;
        if (ns != o.ns) return ns < o.ns;
        if (moving != o.moving) return moving < o.moving;
        if (rowsum != o.rowsum) return rowsum < o.rowsum;
        return bin < o.bin;
    }
};

}  // namespace

extern "C" {

int mtpt_pool_create(size_t hbm_budget, int32_t max_slots, void* hip_stream, const mtpt_allocator* alloc,
                     mtpt_pool** out)
{
    if (!out)
        return fail(MTPT_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_slots < 1)
        return fail(MTPT_E_ARG, "max_slots must be >= 1");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(MTPT_E_ARG, "allocator needs both alloc and free");
    mtpt_pool* p = new mtpt_pool();
    p->max_slots = max_slots;
    if (alloc) {
        p->alloc.a = *alloc;
        p->alloc.custom = true;
    }
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            delete p;
            return fail(MTPT_E_DEVICE, "hipMemGetInfo failed");
        }
        hbm_budget = fr / 10 * 9;
    }
    p->budget = hbm_budget;
    if (hip_stream) {
        p->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
            delete p;
            return fail(MTPT_E_DEVICE, "hipStreamCreateWithFlags failed");
        }
        p->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&p->xstream, hipStreamNonBlocking) != hipSuccess) {
        if (p->own_stream)
            (void)hipStreamDestroy(p->stream);
        delete p;
        return fail(MTPT_E_DEVICE, "hipStreamCreateWithFlags failed");
    }
    *out = p;
    return MTPT_OK;
}

int mtpt_pool_admit(mtpt_pool* p, const mtpt_params* params, const double* pos, const double* mass,
                    int64_t n_steps, int64_t* ticket)
{
    if (!p || !ticket)
        return fail(MTPT_E_ARG, "NULL argument");
    if (n_steps < 1)
        return fail(MTPT_E_ARG, "n_steps must be >= 1");
    int rc = validate(params);
    if (rc)
        return rc;
    const Plan q = make_plan(*params);
    // the result export stages n*S doubles next to the sim
    const size_t need = q.bytes + static_cast<size_t>(q.n) * q.ns * 8;
    if (static_cast<int32_t>(p->sims.size()) >= p->max_slots)
        return fail(MTPT_E_NOMEM, "no free slot (%d active)", static_cast<int>(p->sims.size()));
    if (p->held + need > p->budget)
        return fail(MTPT_E_NOMEM, "budget: %zu held + %zu needed > %zu", p->held, need, p->budget);
    // inputs staged through pinned memory and uploaded asynchronously: the
    // admission does not wait for the ticks in flight
    PinnedStage* stage = nullptr;
    rc = stage_acquire(p, static_cast<size_t>(q.n) * (static_cast<size_t>(q.dim) * q.tsz + static_cast<size_t>(q.ns) * q.msz),
                       &stage);
    if (rc)
        return rc;
    mtpt_sim* s = nullptr;
    rc = new_sim(params, pos, mass, p->stream, p->alloc.custom ? &p->alloc.a : nullptr, &s, stage);
    if (rc)
        return rc;
    s->steps_target = n_steps;
    const int64_t t = p->next_ticket++;
    p->sims[t] = s;
    p->bytes_of[t] = need;
    p->held += need;
    *ticket = t;
    return MTPT_OK;
}

int mtpt_pool_tick(mtpt_pool* p, int32_t* n_completed)
{
    if (!p)
        return fail(MTPT_E_ARG, "pool is NULL");
    std::map<GroupKey, std::vector<mtpt_sim*>> groups;
    for (auto& kv : p->sims) {
        mtpt_sim* s = kv.second;
        if (s->steps_done >= s->steps_target || s->q.n == 0)
            continue;
        const GroupKey k{s->q.dim, s->q.prec, s->q.ns, s->tens.on ? 1 : 0, s->moving ? 1 : 0, (s->moving || !s->s_valid) ? 1 : 0,
                         (s->moving && !s->bin_ready) ? 1 : 0};
        groups[k].push_back(s);
    }
    // layout of the argument block: per group, SimArgs[ns] then PH_COUNT
    // prefixes of (ns + 1) u32
    size_t bytes = 0;
    std::vector<size_t> goff;
    for (auto& g : groups) {
        goff.push_back(bytes);
        const size_t ns = g.second.size();
        bytes = align_up(bytes + ns * sizeof(SimArgs), 256);
        bytes = align_up(bytes + PH_COUNT * (ns + 1) * sizeof(uint32_t), 256);
    }
    int32_t completed = 0;
    if (!groups.empty()) {
        RingSlot& r = p->ring[p->ticks % 4];
        int rc = ring_reserve(p, r, bytes);
        if (rc)
            return rc;
        char* h = static_cast<char*>(r.host);
        size_t gi = 0;
        for (auto& g : groups) {
            const size_t ns = g.second.size();
            SimArgs* args = reinterpret_cast<SimArgs*>(h + goff[gi]);
            uint32_t* pre = reinterpret_cast<uint32_t*>(h + align_up(goff[gi] + ns * sizeof(SimArgs), 256));
            for (size_t i = 0; i < ns; ++i) {
                bool need = false;
                args[i] = step_args(g.second[i], &need);
            }
            for (int ph = 0; ph < PH_COUNT; ++ph) {
                uint32_t* o = pre + ph * (ns + 1);
                o[0] = 0;
                for (size_t i = 0; i < ns; ++i)
                    o[i + 1] = o[i] + phase_blocks(ph, args[i]);
            }
            ++gi;
        }
        HIP_TRY(hipMemcpyAsync(r.dev, r.host, bytes, hipMemcpyHostToDevice, p->stream));
        gi = 0;
        for (auto& g : groups) {
            const GroupKey& k = g.first;
            const size_t ns = g.second.size();
            char* d = static_cast<char*>(r.dev);
            const SimArgs* dargs = reinterpret_cast<const SimArgs*>(d + goff[gi]);
            const uint32_t* dpre = reinterpret_cast<const uint32_t*>(d + align_up(goff[gi] + ns * sizeof(SimArgs), 256));
            const uint32_t* hpre = reinterpret_cast<const uint32_t*>(h + align_up(goff[gi] + ns * sizeof(SimArgs), 256));
            const SimArgs* hargs = reinterpret_cast<const SimArgs*>(h + goff[gi]);
            bool any_unfolded = false;
            for (size_t i = 0; i < ns; ++i)
                any_unfolded = any_unfolded || !hargs[i].scan_fold;
            std::vector<int> phases;
            if (k.bin)
                phases.push_back(PH_BIN);
            if (k.moving)
                for (int ph : {PH_SCAN_REDUCE, PH_SCAN_TOP, PH_SCAN_DOWN, PH_SCATTER, PH_PLACE})
                    if (ph != PH_SCAN_TOP || any_unfolded)
                        phases.push_back(ph);
            if (k.rowsum)
                phases.push_back(PH_ROWSUM);
            phases.push_back(PH_TRANSFER);
            phases.push_back(PH_FINALIZE);
            for (int ph : phases) {
                Batch b;
                b.args = dargs;
                b.blk_off = dpre + ph * (ns + 1);
                b.nsims = static_cast<int32_t>(ns);
                b.total_blocks = hpre[ph * (ns + 1) + ns];
                HIP_TRY(launch_phase_batched(ph, k.dim, k.prec, k.ns, k.tensor, b, p->stream));
            }
            for (mtpt_sim* s : g.second) {
                s->steps_done += 1;
                if (!s->moving)
                    s->s_valid = true;
                else
                    s->bin_ready = true;
                if (s->steps_done == s->steps_target) {
                    ++completed;
                    // done() and the exports wait for this event only
                    if (!s->done_ev)
                        HIP_TRY(hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming));
                    HIP_TRY(hipEventRecord(s->done_ev, p->stream));
                }
            }
            ++gi;
        }
        HIP_TRY(hipEventRecord(r.ev, p->stream));
        r.armed = true;
        p->ticks += 1;
    }
    if (n_completed)
        *n_completed = completed;
    return MTPT_OK;
}

int mtpt_pool_done(mtpt_pool* p, int64_t ticket, int32_t* done)
{
    if (!p || !done)
        return fail(MTPT_E_ARG, "NULL argument");
    auto it = p->sims.find(ticket);
    if (it == p->sims.end())
        return fail(MTPT_E_ARG, "unknown ticket %lld", (long long)ticket);
    mtpt_sim* s = it->second;
    *done = 0;
    if (s->steps_done >= s->steps_target) {
        if (!s->done_ev) {
            HIP_TRY(hipStreamSynchronize(p->stream));
            *done = 1;
            return MTPT_OK;
        }
        // a query, not a wait: the ticks of the other sims keep running
        const hipError_t e = hipEventQuery(s->done_ev);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();
            return MTPT_OK;
        }
        if (e != hipSuccess)
            return fail(MTPT_E_DEVICE, "mtpt_pool_done: %s", hipGetErrorString(e));
        *done = 1;
    }
    return MTPT_OK;
}

int mtpt_pool_stats(mtpt_pool* p, int64_t ticket, mtpt_stats_t* out)
{
    if (!p || !out)
        return fail(MTPT_E_ARG, "NULL argument");
    auto it = p->sims.find(ticket);
    if (it == p->sims.end())
        return fail(MTPT_E_ARG, "unknown ticket %lld", (long long)ticket);
    mtpt_sim* s = it->second;
    return on_export_stream(p, s, [&] { return mtpt_stats(s, out); });
}

int mtpt_pool_result(mtpt_pool* p, int64_t ticket, double* mass_out)
{
    if (!p)
        return fail(MTPT_E_ARG, "pool is NULL");
    auto it = p->sims.find(ticket);
    if (it == p->sims.end())
        return fail(MTPT_E_ARG, "unknown ticket %lld", (long long)ticket);
    mtpt_sim* s = it->second;
    if (s->steps_done < s->steps_target)
        return fail(MTPT_E_STATE, "ticket %lld has %lld of %lld steps", (long long)ticket,
                    (long long)s->steps_done, (long long)s->steps_target);
    const int rc = on_export_stream(p, s, [&] { return mtpt_masses(s, mass_out); });
    if (rc && rc != MTPT_E_NONFINITE)
        return rc;
    if (!s->done_ev)
        (void)hipStreamSynchronize(p->stream);
    release(s);
    p->held -= p->bytes_of[ticket];
    p->bytes_of.erase(ticket);
    p->sims.erase(it);
    return rc;
}

int mtpt_pool_usage(mtpt_pool* p, int32_t* active, size_t* bytes_held, size_t* budget)
{
    if (!p)
        return fail(MTPT_E_ARG, "pool is NULL");
    if (active)
        *active = static_cast<int32_t>(p->sims.size());
    if (bytes_held)
        *bytes_held = p->held;
    if (budget)
        *budget = p->budget;
    return MTPT_OK;
}

int mtpt_pool_destroy(mtpt_pool* p)
{
    if (!p)
        return MTPT_OK;
    (void)hipStreamSynchronize(p->stream);
    if (p->xstream)
        (void)hipStreamSynchronize(p->xstream);
    for (auto& kv : p->sims)
        release(kv.second);
    p->sims.clear();
    for (auto& g : p->stages) {
        if (g.host)
            (void)hipHostFree(g.host);
        if (g.ev)
            (void)hipEventDestroy(g.ev);
    }
    p->stages.clear();
    if (p->xstream)
        (void)hipStreamDestroy(p->xstream);
    for (auto& r : p->ring) {
        if (r.host)
            (void)hipHostFree(r.host);
        p->alloc.put(r.dev);
        if (r.ev)
            (void)hipEventDestroy(r.ev);
    }
    if (p->own_stream && p->stream)
        (void)hipStreamDestroy(p->stream);
    delete p;
    return MTPT_OK;
}

}  // extern "C"
