// C ABI of the S-TPLS time step (declared in include/stp.h): context,
// workspace carving, the SRJ schedule, the Poisson drivers and the step
// sequence.  All arithmetic runs in the kernels of stp_kernels.hip; this file
// only orders launches on the caller's stream and reads back scalars.
#include "stp.h"
#include "stp_internal.h"
#include "stp_net.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace stp;

struct stp_ctx {
    stp_config cfg{};
    Geo g{};
    hipStream_t s = nullptr;
    int device = 0;
    // FP64 fields
    double *u = nullptr, *v = nullptr, *w = nullptr, *p = nullptr, *ptmp = nullptr, *b = nullptr, *nut = nullptr;
    double* rhs[3] = {nullptr, nullptr, nullptr};
    double* tmp = nullptr;  // Crank-Nicolson ping-pong partner (nw values)
    double *p1 = nullptr, *p2 = nullptr;  // p^{n-1}, p^{n-2} (extrapolated warm start)
    int nhist = 0;                        // of them, the solutions held
    // least-squares history: the solution of step j and its right-hand side
    // sit in slot j mod proj_depth; nproj of the latest steps are held
    double* hp[kMaxProj] = {};
    double* hb[kMaxProj] = {};
    int nproj = 0;
    double* e[3][3] = {};   // Adams-Bashforth history, [slot][component] (FP64 mode)
    float* e32[3][3] = {};  // the same in FP32 (mixed mode)
    float *u32 = nullptr, *v32 = nullptr, *w32 = nullptr;  // FP32 copies of the state (mixed mode stencils)
    double* ub = nullptr;  // plane means of u; u32 holds u minus them (mixed mode)
    // FP32 work arrays of the mixed solve
    float *e0 = nullptr, *e1 = nullptr, *r32 = nullptr;
    _Float16* r16 = nullptr;  // mixed_rhs16: scaled FP16 copy of r32
    // FP32 arrays of the mixed-mode Crank-Nicolson solve: nu_T, h L R, increments
    float *nut32 = nullptr, *cnd = nullptr, *cna = nullptr, *cnb = nullptr;
    double* part = nullptr;  // reduction partials
    double* res = nullptr;   // device scalar results
    double* host = nullptr;  // pinned host copy of res
    std::vector<double> omega;  // the relaxation cycle (weights)
    double kmin = 0.0, kmax = 0.0;                     // spectrum of L_p / D
    std::map<int, std::vector<double>> cycles;        // adaptive cycles by degree
    double D = 0.0;             // Jacobi diagonal 2/dx^2 + 2/dy^2 + 2/dz^2
    int step = 0;
    stp::NetModel* net = nullptr;
    // step start, solve start/end, step end; sweep sequence start/end; ends of
    // the eddy-viscosity, momentum and divergence phases
    hipEvent_t ev[9] = {};
    bool trace_sync = false;  // STP_TRACE_SYNC=1: phase ranges end after their device work
    std::string err;
};

namespace {

constexpr size_t kAlign = 256;
constexpr double kCnTol32 = 1e-7;  // FP32 resolution of the Crank-Nicolson increment
// least per-pass residual reduction asked of a pass whose right-hand side is
// stored in FP16 (unit roundoff 2^-11 = 4.9e-4 on every element)
constexpr double kRhs16Floor = 1e-3;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Effective configuration: defaults applied to the zero-valued optional fields.
stp_config effective(const stp_config& c)
{
    stp_config e = c;
    if (e.srj_reduction == 0.0) e.srj_reduction = 1e-3;
    if (e.mixed_inner == 0) e.mixed_inner = 1;
    if (e.cn_tol == 0.0) e.cn_tol = 1e-13;
    return e;
}

Geo make_geo(int nx, int ny, int nz, double lx, double ly, double lz)
{
    Geo g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.plane = (long long)nx * ny;
    g.n = g.plane * nz;
    g.nw = g.plane * (nz + 1);
    const double dx = lx / nx, dy = ly / ny, dz = lz / nz;
    g.idx = 1.0 / dx; g.idy = 1.0 / dy; g.idz = 1.0 / dz;
    g.idx2 = 1.0 / (dx * dx); g.idy2 = 1.0 / (dy * dy); g.idz2 = 1.0 / (dz * dz);
    return g;
}

// Grid and domain checks shared by every entry point that takes a grid.
const char* validate_grid(int nx, int ny, int nz, double lx, double ly, double lz)
{
    if (nx < 1 || ny < 1 || nz < 2) return "grid: need nx >= 1, ny >= 1, nz >= 2";
    if ((long long)nx * ny * (nz + 1) > (1LL << 40)) return "grid too large";
    if ((long long)nx * ny >= (1LL << 31)) return "grid plane too large (nx*ny >= 2^31)";
    if (!finite_pos(lx) || !finite_pos(ly) || !finite_pos(lz)) return "domain lengths must be finite and > 0";
    // the column-marching reductions keep up to 8 partials per workgroup in
    // kMaxPartBlocks * 8 slots, and every z-chunk holds at least one plane
    if ((long long)march_shape(make_geo(nx, ny, nz, lx, ly, lz), 2048).nblocks() > kMaxPartBlocks)
        return "grid plane too large for the reductions (more than 65536 column tiles of 64 x 4)";
    return nullptr;
}

const char* validate(const stp_config& c)
{
    if (const char* e = validate_grid(c.nx, c.ny, c.nz, c.lx, c.ly, c.lz)) return e;
    if (!finite_pos(c.nu)) return "nu must be finite and > 0";
    if (!finite_pos(c.dt)) return "dt must be finite and > 0";
    if (!std::isfinite(c.dpdx)) return "dpdx must be finite";
    if (c.les != 0 && c.les != 1) return "les must be 0 or 1";
    if (c.les && (!(c.cs >= 0.0) || !std::isfinite(c.cs) || !finite_pos(c.vd_a))) return "les: need cs >= 0, vd_a > 0";
    if (c.precision != STP_FP64 && c.precision != STP_MIXED) return "precision must be STP_FP64 or STP_MIXED";
    if (c.warm_start != STP_WS_PREV && c.warm_start != STP_WS_ZERO && c.warm_start != STP_WS_LEARNED)
        return "warm_start must be STP_WS_PREV, STP_WS_ZERO or STP_WS_LEARNED";
    if (!(c.poisson_rtol >= 0.0) || !std::isfinite(c.poisson_rtol)) return "poisson_rtol must be >= 0";
    if (c.poisson_maxit < 1) return "poisson_maxit must be >= 1";
    if (c.srj_m < 0) return "srj_m must be >= 0";
    if (c.srj_m > 0) {
        if (!c.srj_omega) return "srj_omega is NULL with srj_m > 0";
        for (int k = 0; k < c.srj_m; ++k)
            if (!std::isfinite(c.srj_omega[k])) return "srj_omega holds a non-finite weight";
    } else if (!(c.srj_reduction > 0.0 && c.srj_reduction < 1.0)) {
        return "srj_reduction must lie in (0, 1)";
    }
    if (c.mixed_inner < 1) return "mixed_inner must be >= 1";
    if (c.srj_adaptive != 0 && c.srj_adaptive != 1) return "srj_adaptive must be 0 or 1";
    if (c.srj_adaptive && c.srj_m > 0) return "srj_adaptive needs the built-in schedule (srj_m = 0)";
    if (c.tblock < 0 || c.tblock > kMaxFused) return "tblock must lie in 0..5";
    if (!(c.cn_tol > 0.0 && c.cn_tol < 1.0)) return "cn_tol must lie in (0, 1)";
    if (c.learned_correction != 0 && c.learned_correction != 1) return "learned_correction must be 0 or 1";
    if (c.extrap_order < 0 || c.extrap_order > 2) return "extrap_order must be 0, 1 or 2";
    if (c.extrap_order > 0 && c.warm_start == STP_WS_ZERO) return "extrap_order needs STP_WS_PREV or STP_WS_LEARNED";
    if (c.proj_depth < 0 || c.proj_depth > kMaxProj) return "proj_depth must lie in 0..8";
    if (c.proj_depth > 0 && c.warm_start == STP_WS_ZERO) return "proj_depth needs STP_WS_PREV or STP_WS_LEARNED";
    if (c.mixed_rhs16 != 0 && c.mixed_rhs16 != 1) return "mixed_rhs16 must be 0 or 1";
    if (c.mixed_rhs16 && c.precision != STP_MIXED) return "mixed_rhs16 needs STP_MIXED";
    if (c.stencils32 != 0 && c.stencils32 != 1) return "stencils32 must be 0 or 1";
    if (c.stencils32 && c.precision != STP_MIXED) return "stencils32 needs STP_MIXED";
    return nullptr;
}

// Byte offsets of every array in the workspace.
struct Layout {
    size_t u, v, w, p, ptmp, b, nut, rhs[3], tmp, p1, p2, hp[kMaxProj], hb[kMaxProj], e[3][3], e32[3][3], u32, v32,
        w32, ub, e0, e1, r32, r16, nut32, cnd, cna, cnb, part, res, total;
};

Layout layout(const stp_config& c)
{
    const size_t n = (size_t)c.nx * c.ny * c.nz, nw = (size_t)c.nx * c.ny * (c.nz + 1);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.u = take(n * 8);
    L.v = take(n * 8);
    L.w = take(nw * 8);
    L.p = take(n * 8);
    L.ptmp = take(n * 8);
    L.b = take(n * 8);
    // FP32 eddy viscosity, explicit terms and history (stencils32)
    const bool st32 = c.precision == STP_MIXED && c.stencils32;
    if (!st32) L.nut = take(n * 8);
    for (int q = 0; q < 3; ++q) L.rhs[q] = take((q == 2 ? nw : n) * 8);
    L.tmp = take(nw * 8);
    if (c.extrap_order >= 1) L.p1 = take(n * 8);
    if (c.extrap_order >= 2) L.p2 = take(n * 8);
    for (int j = 0; j < c.proj_depth; ++j) {
        L.hp[j] = take(n * 8);
        L.hb[j] = take(n * 8);
    }
    for (int sl = 0; sl < 3; ++sl)
        for (int q = 0; q < 3; ++q) {
            if (st32) L.e32[sl][q] = take((q == 2 ? nw : n) * 4);
            else L.e[sl][q] = take((q == 2 ? nw : n) * 8);
        }
    if (st32) {
        L.u32 = take(n * 4);
        L.v32 = take(n * 4);
        L.w32 = take(nw * 4);
        L.ub = take((size_t)c.nz * 8);
    }
    L.e0 = take(n * 4);
    L.e1 = take(n * 4);
    L.r32 = take(n * 4);
    if (c.precision == STP_MIXED && c.mixed_rhs16) L.r16 = take(n * 2);
    if (c.precision == STP_MIXED) {
        L.nut32 = take(n * 4);
        L.cnd = take(nw * 4);
        L.cna = take(nw * 4);
        L.cnb = take(nw * 4);
    }
    L.part = take((size_t)kMaxPartBlocks * 8 * 8);
    L.res = take(RES_COUNT * 8);
    L.total = off;
    return L;
}

// ---- the relaxation schedule ------------------------------------------------
// The paper (Sec. 3.4) uses an SRJ cycle of M Jacobi-SOR sweeps whose weights
// it takes from an external script without printing them.  The built-in
// cycle here: one sweep multiplies the error along an eigenvector of -L_p
// (eigenvalue lambda, kappa = lambda/D) by (1 - omega kappa), so the cycle of
// least worst-case factor over [kappa_min, kappa_max] has omega_k = 1/x_k at
// the Chebyshev nodes x_k of that interval (the many-level limit of SRJ).
// M is the smallest degree whose bound 1/T_M((b+a)/(b-a)) meets the requested
// reduction; the sweeps run in Leja order of the nodes, which keeps the
// intermediate amplification of the cycle moderate.

void kappa_range(const Geo& g, double D, double* kmin, double* kmax)
{
    const double pi = M_PI;
    double lmin = INFINITY, lmax = 0.0;
    auto dir = [&](double ih2, int n, bool cosine_modes) {
        if (n < 2) return;  // a single cell carries only the constant mode
        const double period = cosine_modes ? 2.0 * n : (double)n;
        const double s1 = std::sin(pi / period);
        lmin = std::min(lmin, 4.0 * ih2 * s1 * s1);
        const int mtop = cosine_modes ? n - 1 : n / 2;
        const double st = std::sin(pi * mtop / period);
        lmax += 4.0 * ih2 * st * st;
    };
    dir(g.idx2, g.nx, false);
    dir(g.idy2, g.ny, false);
    dir(g.idz2, g.nz, true);
    *kmin = lmin / D;
    *kmax = lmax / D;
}

int chebyshev_degree(double a, double b, double reduction)
{
    const double s = (b + a) / (b - a);
    return std::max(1, (int)std::ceil(std::acosh(1.0 / reduction) / std::acosh(s)));
}

// max of a[0..n): four independent running maxima (a max does not depend on
// the order), so the compare chain does not serialise the scan
static double max_of(const double* a, int n)
{
    double t[4] = {-1e300, -1e300, -1e300, -1e300};
    int k = 0;
    for (; k + 4 <= n; k += 4)
        for (int q = 0; q < 4; ++q) t[q] = a[k + q] > t[q] ? a[k + q] : t[q];
    for (; k < n; ++k) t[0] = a[k] > t[0] ? a[k] : t[0];
    return std::max(std::max(t[0], t[1]), std::max(t[2], t[3]));
}

std::vector<double> chebyshev_leja_nodes(double a, double b, int m)
{
    std::vector<double> x(m);
    for (int k = 1; k <= m; ++k) x[k - 1] = 0.5 * (a + b) + 0.5 * (b - a) * std::cos(M_PI * (2.0 * k - 1.0) / (2.0 * m));
    // Leja order: largest magnitude first, then maximise the product of
    // distances to the nodes already placed (sum of logs).  Candidates within
    // a relative 1e-9 of the best count as tied (the nodes are symmetric, so
    // exact ties occur and round-off must not decide them); ties go to the
    // lower index.
    // The logs come from a table: with theta_i = pi (2i + 1) / (2m) and
    // h = (b - a) / 2, x_i - x_j = -2h sin(pi (i + j + 1) / (2m)) sin(pi (i - j) / (2m)),
    // so log|x_i - x_j| = log(2h) + T[i + j + 1] + T[|i - j|] with
    // T[n] = log sin(pi n / (2m)), 0 < n < 2m: 2m logs instead of m^2 / 2.
    const double l2h = std::log(b - a);
    std::vector<double> T(2 * m + 1, 0.0);  // T[0], T[2m] are never read
    for (int n = 1; n < 2 * m; ++n) T[n] = std::log(std::sin(M_PI * n / (2.0 * m)));
    constexpr double kPlaced = -1e300;  // finite, below any sum of logs
    std::vector<double> logd(m, 0.0);
    std::vector<double> out;
    out.reserve(m);
    int cur = 0;
    for (int k = 1; k < m; ++k)
        if (std::fabs(x[k]) > std::fabs(x[cur])) cur = k;
    for (int t = 0; t < m; ++t) {
        logd[cur] = kPlaced;
        out.push_back(1.0 / x[cur]);
        if (t == m - 1) break;
        double* L = logd.data();
        const double* Tp = T.data() + cur + 1;  // T[k + cur + 1]
        const double* Tm = T.data() + cur;      // T[cur - k] = Tm[-k]
        for (int k = 0; k < cur; ++k) L[k] += (l2h + Tp[k]) + Tm[-k];
        for (int k = cur + 1; k < m; ++k) L[k] += (l2h + Tp[k]) + T[k - cur];
        const double top = max_of(L, m);
        const double tol = 1e-9 * std::max(1.0, std::fabs(top));
        int best = 0;
        while (!(L[best] >= top - tol)) ++best;
        cur = best;
    }
    return out;
}

std::vector<double> chebyshev_leja_cycle(double a, double b, double reduction)
{
    return chebyshev_leja_nodes(a, b, chebyshev_degree(a, b, reduction));
}

#define CHK(expr)                                                                   \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);           \
            return STP_EDEVICE;                                                     \
        }                                                                           \
    } while (0)

stp_status readback(stp_ctx* ctx)
{
    CHK(hipMemcpyAsync(ctx->host, ctx->res, RES_COUNT * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
    CHK(hipStreamSynchronize(ctx->s));
    return STP_OK;
}

// Run `count` sweeps of the schedule starting at sweep index `first` (mod M),
// ping-ponging between *cur and *other; on return *cur holds the iterate.
// The cycle for the next pass: the fixed cycle, or (adaptive) the Chebyshev/
// Leja cycle whose degree, rounded up to a multiple of 16, bounds the residual
// reduction by rho = max(rtol ||b|| / ||r||, floor), rho <= 1/2: the residual
// is mean-free, so each of its modes has kappa in [kmin, kmax] and is scaled
// by at most 1/T_M, and one cycle meets the reduction still needed.
const std::vector<double>& next_cycle(stp_ctx* ctx, double rtol, double fb, double rn, double floor_rho)
{
    if (!ctx->cfg.srj_adaptive || !(rtol > 0.0) || !(rn > 0.0)) return ctx->omega;
    double rho = rtol * fb / rn;
    rho = std::min(0.5, std::max(floor_rho, rho));
    int m = chebyshev_degree(ctx->kmin, ctx->kmax, rho);
    m = (m + 15) / 16 * 16;
    auto it = ctx->cycles.find(m);
    if (it == ctx->cycles.end()) it = ctx->cycles.emplace(m, chebyshev_leja_nodes(ctx->kmin, ctx->kmax, m)).first;
    return it->second;
}

template <typename T, typename TB = T>
stp_status run_sweeps(stp_ctx* ctx, const TB* b, T** cur, T** other, const double* omega, int m, long long first,
                      long long count, int* launches = nullptr)
{
    // tblock sweeps per launch where the grid allows it (FP64: at most 4;
    // tblock = 0: FP32 sweeps take relax_auto_depth, FP64 four), the
    // remainder in one shorter launch.
    const int want = ctx->cfg.tblock != 0 ? ctx->cfg.tblock : (sizeof(T) == 4 ? relax_auto_depth(ctx->g) : 4);
    const int tb = relax_fusable(ctx->g) ? std::min(want, sizeof(T) == 4 ? kMaxFused : 4) : 1;
    long long s = 0;
    while (s < count) {
        const int nf = (int)std::min<long long>(tb, count - s);
        Weights wts{};
        for (int f = 0; f < nf; ++f) wts.omega[f] = omega[(first + s + f) % m];
        CHK(relax(ctx->g, b, (const T*)*cur, *other, wts, nf, ctx->s));
        std::swap(*cur, *other);
        s += nf;
        if (launches) ++*launches;
    }
    return STP_OK;
}

// run_sweeps between two events; adds the device time to st->ms_relax after
// the next synchronisation (timed_flush).
template <typename T, typename TB = T>
stp_status timed_sweeps(stp_ctx* ctx, const TB* b, T** cur, T** other, const std::vector<double>& omega, long long count,
                        stp_solve_stats* st)
{
    CHK(hipEventRecord(ctx->ev[4], ctx->s));
    stp_status rc = run_sweeps<T, TB>(ctx, b, cur, other, omega.data(), (int)omega.size(), 0, count, &st->launches);
    if (rc != STP_OK) return rc;
    CHK(hipEventRecord(ctx->ev[5], ctx->s));
    return STP_OK;
}

stp_status timed_flush(stp_ctx* ctx, stp_solve_stats* st)
{
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, ctx->ev[4], ctx->ev[5]));
    st->ms_relax += ms;
    return STP_OK;
}

// FP64 SRJ solve of L_p p = b; p and ptmp ping-pong; result lands in p.
// Assumes res[RES_B2] = ||b||^2 already computed.
stp_status solve_fp64(stp_ctx* ctx, const double* b, double* p, double* ptmp, double rtol, int maxit,
                      stp_solve_stats* st)
{
    const int m = (int)ctx->omega.size();
    double* cur = p;
    double* oth = ptmp;
    stp_status rc;
    CHK(residual(ctx->g, b, cur, nullptr, ctx->part, ctx->res, ctx->s));
    if ((rc = readback(ctx)) != STP_OK) return rc;
    const double bn = std::sqrt(ctx->host[RES_B2]);
    const double fb = bn > 1e-300 ? bn : 1e-300;
    double rn = std::sqrt(ctx->host[RES_R2]);
    st->bnorm = bn;
    st->relres0 = rn / fb;
    st->status = STP_OK;
    int cycles = 0, checks = 0;
    long long sweeps = 0;
    if (rtol > 0.0) {
        while (!(rn <= rtol * fb)) {
            if (!std::isfinite(rn)) { st->status = STP_ENAN; break; }
            if (cycles >= maxit) { st->status = STP_ENOCONV; break; }
            const std::vector<double>& cyc = next_cycle(ctx, rtol, fb, rn, 1e-10);
            if ((rc = timed_sweeps<double>(ctx, b, &cur, &oth, cyc, (long long)cyc.size(), st)) != STP_OK) return rc;
            sweeps += (long long)cyc.size();
            ++cycles;
            CHK(residual(ctx->g, b, cur, nullptr, ctx->part, ctx->res, ctx->s));
            if ((rc = readback(ctx)) != STP_OK) return rc;
            if ((rc = timed_flush(ctx, st)) != STP_OK) return rc;
            rn = std::sqrt(ctx->host[RES_R2]);
            ++checks;
        }
    } else {
        if ((rc = timed_sweeps<double>(ctx, b, &cur, &oth, ctx->omega, (long long)m * maxit, st)) != STP_OK) return rc;
        sweeps = (long long)m * maxit;
        cycles = maxit;
        CHK(residual(ctx->g, b, cur, nullptr, ctx->part, ctx->res, ctx->s));
        if ((rc = readback(ctx)) != STP_OK) return rc;
        if ((rc = timed_flush(ctx, st)) != STP_OK) return rc;
        rn = std::sqrt(ctx->host[RES_R2]);
        checks = 1;
        if (!std::isfinite(rn)) st->status = STP_ENAN;
    }
    if (cur != p) CHK(copy(p, cur, ctx->g.n, ctx->s));
    CHK(sum_into(p, ctx->g.n, ctx->part, ctx->res, RES_SUM_P, ctx->s));
    CHK(remove_mean(p, ctx->g.n, ctx->res + RES_SUM_P, -1, ctx->part, ctx->res, ctx->s));
    st->relres = rn / fb;
    st->cycles = cycles;
    st->outer = checks;
    st->sweeps = (int32_t)sweeps;
    return STP_OK;
}

// Mixed solve: FP64 residual r = b - L p, FP32 SRJ cycles on L e = r from
// e = 0, FP64 update p += e, repeated until the FP64 residual test passes.
stp_status solve_mixed(stp_ctx* ctx, const double* b, double* p, double rtol, int maxit, stp_solve_stats* st)
{
    const int inner = ctx->cfg.mixed_inner;
    stp_status rc;
    CHK(residual(ctx->g, b, p, ctx->r32, ctx->part, ctx->res, ctx->s));
    if ((rc = readback(ctx)) != STP_OK) return rc;
    const double bn = std::sqrt(ctx->host[RES_B2]);
    const double fb = bn > 1e-300 ? bn : 1e-300;
    double rn = std::sqrt(ctx->host[RES_R2]);
    st->bnorm = bn;
    st->relres0 = rn / fb;
    st->status = STP_OK;
    int outer = 0;
    long long sweeps = 0;
    // The FP32 pass solves L e = s r for a power of two s (r32 holds s r, which
    // rounds exactly like r) and the correction is e / s: the scale keeps the
    // copy of a tiny or huge residual inside FP32's normal range, and being a
    // power of two it changes no rounding.  The copy is written with the scale
    // of the residual before the previous pass (rms 1 at that pass, so the
    // reduction of one pass below it); it is rewritten when its rms has left
    // [2^-40, 2^40].  With mixed_rhs16 the pass reads an FP16 copy brought to
    // about unit rms by a further power of two, which bounds what one pass can
    // reduce.
    const bool rhs16 = ctx->cfg.mixed_rhs16 != 0;
    const double floor_rho = rhs16 ? std::max(ctx->cfg.srj_reduction, kRhs16Floor) : ctx->cfg.srj_reduction;
    const double sqrt_n = std::sqrt((double)ctx->g.n);
    auto unit_scale = [&](double rms) {  // power of two nearest 1/rms (rms > 0, finite)
        return std::ldexp(1.0, (int)std::lround(-std::log2(rms)));
    };
    double r32_scale = 1.0;  // ctx->r32 holds r32_scale * r
    auto pass = [&]() -> stp_status {
        float* cur = ctx->e0;
        float* oth = ctx->e1;
        CHK(fill(cur, 0.0f, ctx->g.n, ctx->s));
        const std::vector<double>& cyc = rtol > 0.0 ? next_cycle(ctx, rtol, fb, rn, floor_rho) : ctx->omega;
        const long long count = (long long)cyc.size() * inner;
        sweeps += count;
        stp_status r2;
        const double rms = rn / sqrt_n;  // of the FP64 residual r
        const bool scalable = rms > 0.0 && std::isfinite(rms);
        if (scalable && !(r32_scale * rms >= 0x1p-40 && r32_scale * rms <= 0x1p40)) {
            r32_scale = unit_scale(rms);
            CHK(residual(ctx->g, b, p, ctx->r32, ctx->part, ctx->res, ctx->s, r32_scale));
        }
        if (rhs16 && scalable) {
            // every element of the FP16 copy is at most about sqrt(n) (below
            // FP16's 65504 for n < 2e9)
            const double t = unit_scale(r32_scale * rms);
            CHK(half_scaled(ctx->r16, ctx->r32, ctx->g.n, (float)t, ctx->s));
            r2 = timed_sweeps<float, _Float16>(ctx, ctx->r16, &cur, &oth, cyc, count, st);
            if (r2 != STP_OK) return r2;
            CHK(add_correction_scaled(p, cur, ctx->g.n, 1.0 / (r32_scale * t), ctx->s));
        } else {
            r2 = timed_sweeps<float>(ctx, ctx->r32, &cur, &oth, cyc, count, st);
            if (r2 != STP_OK) return r2;
            if (r32_scale == 1.0) CHK(add_correction(p, cur, ctx->g.n, ctx->s));
            else CHK(add_correction_scaled(p, cur, ctx->g.n, 1.0 / r32_scale, ctx->s));
        }
        if (scalable) r32_scale = unit_scale(rms);
        CHK(residual(ctx->g, b, p, ctx->r32, ctx->part, ctx->res, ctx->s, r32_scale));
        r2 = readback(ctx);
        if (r2 != STP_OK) return r2;
        r2 = timed_flush(ctx, st);
        if (r2 != STP_OK) return r2;
        rn = std::sqrt(ctx->host[RES_R2]);
        ++outer;
        return STP_OK;
    };
    // Learned coarse correction: the network maps the residual r of p to an
    // estimate of L^-1 r; the proposal p + s_r y replaces p only when its FP64
    // residual is smaller (r32 is left holding the residual of whichever is kept).
    int corrections = 0;
    auto correct = [&]() -> stp_status {
        CHK(ctx->net->predict(b, p, ctx->ptmp));
        CHK(residual(ctx->g, b, ctx->ptmp, ctx->r32, ctx->part, ctx->res, ctx->s, r32_scale));
        stp_status r2 = readback(ctx);
        if (r2 != STP_OK) return r2;
        const double rg = std::sqrt(ctx->host[RES_R2]);
        if (std::isfinite(rg) && rg < rn) {
            CHK(copy(p, ctx->ptmp, ctx->g.n, ctx->s));
            rn = rg;
            ++corrections;
        } else {
            CHK(residual(ctx->g, b, p, ctx->r32, ctx->part, ctx->res, ctx->s, r32_scale));
        }
        return STP_OK;
    };
    const bool learned = ctx->cfg.learned_correction && ctx->net != nullptr;
    if (rtol > 0.0) {
        while (!(rn <= rtol * fb)) {
            if (!std::isfinite(rn)) { st->status = STP_ENAN; break; }
            if (outer >= maxit) { st->status = STP_ENOCONV; break; }
            if ((rc = pass()) != STP_OK) return rc;
            if (learned && !(rn <= rtol * fb) && std::isfinite(rn) && outer < maxit)
                if ((rc = correct()) != STP_OK) return rc;
        }
    } else {
        for (int it = 0; it < maxit; ++it)
            if ((rc = pass()) != STP_OK) return rc;
        if (!std::isfinite(rn)) st->status = STP_ENAN;
    }
    CHK(sum_into(p, ctx->g.n, ctx->part, ctx->res, RES_SUM_P, ctx->s));
    CHK(remove_mean(p, ctx->g.n, ctx->res + RES_SUM_P, -1, ctx->part, ctx->res, ctx->s));
    st->relres = rn / fb;
    st->cycles = outer * inner;
    st->outer = outer;
    st->corrections = corrections;
    st->sweeps = (int32_t)sweeps;
    return STP_OK;
}

stp_status solve(stp_ctx* ctx, const double* b, double* p, double rtol, int maxit, stp_solve_stats* st)
{
    if (ctx->cfg.precision == STP_MIXED) return solve_mixed(ctx, b, p, rtol, maxit, st);
    return solve_fp64(ctx, b, p, ctx->ptmp, rtol, maxit, st);
}

// Coefficients a of the least-squares guess from the Gram quantities of
// proj_gram (k(k+1)/2 entries <E_i, E_j>, i <= j row by row, then k entries
// <E_i, b>): the normal equations M a = g, scaled to unit diagonal and solved
// by a Cholesky factorisation that skips every E_i whose part orthogonal to
// the columns kept before it is below kProjPivot of its norm squared (a
// direction the history does not resolve).  Skipped columns get a = 0.
// Returns the number of columns kept.
constexpr long double kProjPivot = 1e-10L;

int proj_coefficients(int k, const double* q, double* a)
{
    long double M[kMaxProj][kMaxProj], g[kMaxProj], sc[kMaxProj], L[kMaxProj][kMaxProj] = {}, z[kMaxProj];
    int t = 0;
    for (int i = 0; i < k; ++i)
        for (int j = i; j < k; ++j) M[i][j] = M[j][i] = q[t++];
    for (int i = 0; i < k; ++i) g[i] = q[t++];
    bool keep[kMaxProj] = {};
    for (int i = 0; i < k; ++i) {
        a[i] = 0.0;
        const long double d = M[i][i];
        sc[i] = (std::isfinite((double)d) && d > 0.0L) ? 1.0L / std::sqrt(d) : 0.0L;
    }
    for (int i = 0; i < t; ++i)
        if (!std::isfinite(q[i])) return 0;
    int rank = 0;
    for (int i = 0; i < k; ++i) {
        if (sc[i] == 0.0L) continue;
        long double d = 1.0L;
        for (int j = 0; j < i; ++j) {
            if (!keep[j]) continue;
            long double v = M[i][j] * sc[i] * sc[j];
            for (int m = 0; m < j; ++m)
                if (keep[m]) v -= L[i][m] * L[j][m];
            L[i][j] = v / L[j][j];
            d -= L[i][j] * L[i][j];
        }
        if (!(d > kProjPivot)) continue;
        L[i][i] = std::sqrt(d);
        keep[i] = true;
        ++rank;
    }
    if (rank == 0) return 0;
    for (int i = 0; i < k; ++i) {  // L z = scaled g
        if (!keep[i]) continue;
        long double v = g[i] * sc[i];
        for (int j = 0; j < i; ++j)
            if (keep[j]) v -= L[i][j] * z[j];
        z[i] = v / L[i][i];
    }
    for (int i = k - 1; i >= 0; --i) {  // L^T y = z, a = scaled y
        if (!keep[i]) continue;
        long double v = z[i];
        for (int j = i + 1; j < k; ++j)
            if (keep[j]) v -= L[j][i] * z[j];
        z[i] = v / L[i][i];
    }
    for (int i = 0; i < k; ++i)
        if (keep[i]) a[i] = (double)(z[i] * sc[i]);
    for (int i = 0; i < k; ++i)
        if (!std::isfinite(a[i])) return 0;
    return rank;
}

// out = the least-squares guess from k held solutions xs and right-hand sides
// ys (newest first) for the right-hand side b; *rank = columns used (out is
// not written when 0).
stp_status lsq_guess(stp_ctx* ctx, int k, const double* const* xs, const double* const* ys, const double* b,
                     double* out, int* rank)
{
    stp_status rc;
    CHK(proj_gram(k, ys, b, ctx->g.n, ctx->part, ctx->res, RES_PROJ, ctx->s));
    if ((rc = readback(ctx)) != STP_OK) return rc;
    double a[kMaxProj];
    *rank = proj_coefficients(k, ctx->host + RES_PROJ, a);
    if (*rank > 0) CHK(proj_combine(k, xs, a, out, ctx->g.n, ctx->s));
    return STP_OK;
}

// The phases of one step as roctx ranges (rocprofv3 --marker-trace), in the
// order of Sec. 3.1: eddy viscosity, momentum (explicit terms and
// Crank-Nicolson), divergence, Poisson guess, Poisson solve, projection.  A
// range covers the host code of its phase; with trace_sync it also waits for
// the phase's device work, so that the ranges tile the step's device time.
class PhaseRanges {
  public:
    explicit PhaseRanges(const stp_ctx* ctx) : ctx_(ctx) {}
    ~PhaseRanges() { close(); }
    void next(const char* name)
    {
        close();
        roctxRangePushA(name);
        open_ = true;
    }
    void close()
    {
        if (!open_) return;
        if (ctx_->trace_sync) (void)hipStreamSynchronize(ctx_->s);
        roctxRangePop();
        open_ = false;
    }

  private:
    const stp_ctx* ctx_;
    bool open_ = false;
};

stp_status one_step(stp_ctx* ctx, stp_step_stats* out)
{
    const stp_config& c = ctx->cfg;
    const Geo& g = ctx->g;
    hipStream_t s = ctx->s;
    stp_step_stats st{};
    stp_status rc;
    PhaseRanges phase(ctx);
    phase.next("stp_step: eddy viscosity");
    CHK(hipEventRecord(ctx->ev[0], s));
    CHK(zero_walls(g, ctx->w, s));

    // 1. eddy viscosity at level n (Sec. 2.2); with stencils32 this and the
    //    explicit terms run on FP32 copies of the FP64 state
    const bool mixed = c.precision == STP_MIXED;
    const bool st32 = mixed && c.stencils32;
    if (st32) {
        CHK(round_departure_f32(g, ctx->u32, ctx->u, ctx->ub, s));
        CHK(round_to_f32(ctx->v32, ctx->v, g.n, s));
        CHK(round_to_f32(ctx->w32, ctx->w, g.nw, s));
    }
    double nut_max = c.nu;
    if (c.les) {
        const double delta = 2.0 * std::cbrt((c.lx / c.nx) * (c.ly / c.ny) * (c.lz / c.nz));
        const double utau = std::sqrt(0.5 * c.lz * std::fabs(c.dpdx));
        const double inv_wall_unit = utau / (c.nu * c.vd_a);
        if (st32)
            CHK(nut_smagorinsky<float>(g, ctx->u32, ctx->v32, ctx->w32, ctx->nut32, c.nu, c.cs * delta,
                                       inv_wall_unit, c.lz, ctx->ub, ctx->part, ctx->res, s));
        else
            CHK(nut_smagorinsky<double>(g, ctx->u, ctx->v, ctx->w, ctx->nut, c.nu, c.cs * delta, inv_wall_unit, c.lz,
                                        nullptr, ctx->part, ctx->res, s));
    } else if (st32) {
        CHK(fill(ctx->nut32, (float)c.nu, g.n, s));
    } else {
        CHK(fill(ctx->nut, c.nu, g.n, s));
    }
    // the mixed mode's Crank-Nicolson iterations read nu_T in FP32
    if (mixed && !st32) CHK(round_to_f32(ctx->nut32, ctx->nut, g.n, s));

    // 2. explicit terms and Crank-Nicolson right-hand sides (Sec. 3.1)
    CHK(hipEventRecord(ctx->ev[6], s));
    phase.next("stp_step: momentum");
    const int n = ctx->step;
    const int sl_n = n % 3, sl_1 = (n + 2) % 3, sl_2 = (n + 1) % 3;
    double beta[3] = {1.0, 0.0, 0.0};
    if (n == 1) { beta[0] = 1.5; beta[1] = -0.5; }
    if (n >= 2) { beta[0] = 23.0 / 12.0; beta[1] = -16.0 / 12.0; beta[2] = 5.0 / 12.0; }
    double* vel[3] = {ctx->u, ctx->v, ctx->w};
    for (int q = 0; q < 3; ++q) {
        if (st32) {
            MomArgsT<float> a{};
            a.u = ctx->u32; a.v = ctx->v32; a.w = ctx->w32; a.nut = ctx->nut32; a.ub = ctx->ub;
            a.en = ctx->e32[sl_n][q]; a.e1 = ctx->e32[sl_1][q]; a.e2 = ctx->e32[sl_2][q];
            a.rhs = ctx->rhs[q];
            a.x64 = vel[q];
            a.beta0 = beta[0]; a.beta1 = beta[1]; a.beta2 = beta[2];
            a.dt = c.dt; a.half_dt = 0.5 * c.dt; a.dpdx = c.dpdx; a.nu = c.nu;
            CHK(momentum_rhs<float>(g, q, a, s));
        } else {
            MomArgs a{};
            a.u = ctx->u; a.v = ctx->v; a.w = ctx->w; a.nut = ctx->nut;
            a.en = ctx->e[sl_n][q]; a.e1 = ctx->e[sl_1][q]; a.e2 = ctx->e[sl_2][q];
            a.rhs = ctx->rhs[q];
            a.beta0 = beta[0]; a.beta1 = beta[1]; a.beta2 = beta[2];
            a.dt = c.dt; a.half_dt = 0.5 * c.dt; a.dpdx = c.dpdx; a.nu = c.nu;
            CHK(momentum_rhs<double>(g, q, a, s));
        }
    }
    if (c.les) {
        if ((rc = readback(ctx)) != STP_OK) return rc;
        nut_max = ctx->host[RES_NUT_MAX];
        if (!std::isfinite(nut_max)) {
            ctx->err = "non-finite eddy viscosity";
            return STP_ENAN;
        }
    }

    // 3. Crank-Nicolson solve (I - dt/2 L_nu) u* = R by the iteration
    //    x <- x + (R - (I - h L) x)/(1 + h s), h = dt/2, s = Lambda/2, Lambda =
    //    4 nu_max (1/dx^2 + 1/dy^2 + 1/dz^2) >= spectral radius of -L_nu; its
    //    error contracts by rho = h s/(1 + h s) per iteration, so m iterations
    //    with rho^m <= cn_tol reach the target.  m is made odd so that the
    //    last iterate lands in the state array.
    const double lam = 4.0 * nut_max * (g.idx2 + g.idy2 + g.idz2);
    const double hs = 0.5 * c.dt * 0.5 * lam;
    const double rho = hs / (1.0 + hs);
    int mcn = (int)std::ceil(std::log(c.cn_tol) / std::log(rho));
    mcn = std::max(1, std::min(mcn, 999));
    if (mcn % 2 == 0) ++mcn;
    if (c.precision == STP_MIXED) {
        // Mixed mode: the defect form u* = R + delta, (I - h L) delta = h L R,
        // iterated in FP32 from delta = 0 (R and u* stay FP64); FP32 resolves
        // delta to about 1e-7 of itself, so the target is max(cn_tol, 1e-7).
        int m32 = (int)std::ceil(std::log(std::max(c.cn_tol, kCnTol32)) / std::log(rho));
        m32 = std::max(2, std::min(m32, 999));
        for (int q = 0; q < 3; ++q) {
            float* a = ctx->cna;
            float* bb = ctx->cnb;
            CHK(cn_defect(g, q, 0, ctx->nut32, c.nu, ctx->rhs[q], nullptr, ctx->cnd, nullptr, a, nullptr, 0.5 * c.dt,
                          1.0 / (1.0 + hs), s));
            for (int it = 1; it + 1 < m32; ++it) {
                CHK(cn_defect(g, q, 1, ctx->nut32, c.nu, ctx->rhs[q], ctx->cnd, nullptr, a, bb, nullptr, 0.5 * c.dt,
                              1.0 / (1.0 + hs), s));
                std::swap(a, bb);
            }
            CHK(cn_defect(g, q, 2, ctx->nut32, c.nu, ctx->rhs[q], ctx->cnd, nullptr, a, nullptr, vel[q], 0.5 * c.dt,
                          1.0 / (1.0 + hs), s));
        }
        st.cn_sweeps = m32;
    } else {
        for (int q = 0; q < 3; ++q) {
            for (int it = 0; it < mcn; ++it) {
                const double* x = it == 0 ? ctx->rhs[q] : (it % 2 == 1 ? vel[q] : ctx->tmp);
                double* xo = it % 2 == 0 ? vel[q] : ctx->tmp;
                CHK(cn_iterate(g, q, ctx->nut, c.nu, ctx->rhs[q], x, xo, 0.5 * c.dt, 1.0 / (1.0 + hs), s));
            }
        }
        st.cn_sweeps = mcn;
    }

    // 4. b = div(u*)/dt, mean removed; ||b||^2 into RES_B2
    CHK(hipEventRecord(ctx->ev[7], s));
    phase.next("stp_step: divergence");
    CHK(divergence_rhs(g, ctx->u, ctx->v, ctx->w, ctx->b, 1.0 / c.dt, ctx->part, ctx->res, s));
    CHK(remove_mean(ctx->b, g.n, ctx->res + RES_SUM_B, RES_B2, ctx->part, ctx->res, s));
    CHK(hipEventRecord(ctx->ev[8], s));
    phase.next("stp_step: Poisson guess");

    // 5. SRJ pressure solve from the warm start (Sec. 3.4)
    if (c.warm_start == STP_WS_ZERO) CHK(fill(ctx->p, 0.0, g.n, s));
    double guess_res = -1.0;  // residual norm of ctx->p when already known
    if (c.extrap_order > 0) {
        // candidates: p^n, 2p^n - p^{n-1} (into ptmp), 3(p^n - p^{n-1}) + p^{n-2}
        // (into tmp), as far as the history goes; the one of least FP64
        // residual becomes the guess, and p^n enters the history
        CHK(residual(g, ctx->b, ctx->p, nullptr, ctx->part, ctx->res, s));
        if ((rc = readback(ctx)) != STP_OK) return rc;
        const double bn = std::sqrt(ctx->host[RES_B2]);
        const double fb = bn > 1e-300 ? bn : 1e-300;
        const double r0 = std::sqrt(ctx->host[RES_R2]);
        double rbest = r0;
        int best = 0;
        double* cand[3] = {ctx->p, ctx->ptmp, ctx->tmp};
        for (int order = 1; order <= std::min(c.extrap_order, ctx->nhist); ++order) {
            CHK(extrapolate(ctx->p, ctx->p1, ctx->p2, order, cand[order], g.n, s));
            CHK(residual(g, ctx->b, cand[order], nullptr, ctx->part, ctx->res, s));
            if ((rc = readback(ctx)) != STP_OK) return rc;
            const double r = std::sqrt(ctx->host[RES_R2]);
            if (std::isfinite(r) && r < rbest) {
                rbest = r;
                best = order;
            }
        }
        if (c.extrap_order >= 2 && ctx->nhist >= 1) CHK(copy(ctx->p2, ctx->p1, g.n, s));
        CHK(copy(ctx->p1, ctx->p, g.n, s));
        ctx->nhist = std::min(ctx->nhist + 1, c.extrap_order);
        if (best > 0) CHK(copy(ctx->p, cand[best], g.n, s));
        st.relres_prev = r0 / fb;
        st.relres_extrap = rbest / fb;
        st.extrap_used = best;
        guess_res = rbest;
    }
    if (c.proj_depth > 0 && ctx->nproj > 0) {
        // least squares over the held solutions, newest first (slot of step j: j mod proj_depth)
        if (guess_res < 0.0) {
            CHK(residual(g, ctx->b, ctx->p, nullptr, ctx->part, ctx->res, s));
            if ((rc = readback(ctx)) != STP_OK) return rc;
            guess_res = std::sqrt(ctx->host[RES_R2]);
            st.relres_prev = guess_res / std::max(std::sqrt(ctx->host[RES_B2]), 1e-300);
        }
        const int k = std::min(c.proj_depth, ctx->nproj);
        const double* xs[kMaxProj];
        const double* ys[kMaxProj];
        for (int i = 0; i < k; ++i) {
            const int slot = ((ctx->step - 1 - i) % c.proj_depth + c.proj_depth) % c.proj_depth;
            xs[i] = ctx->hp[slot];
            ys[i] = ctx->hb[slot];
        }
        int rank = 0;
        if ((rc = lsq_guess(ctx, k, xs, ys, ctx->b, ctx->ptmp, &rank)) != STP_OK) return rc;
        st.proj_rank = rank;
        if (rank > 0) {
            CHK(residual(g, ctx->b, ctx->ptmp, nullptr, ctx->part, ctx->res, s));
            if ((rc = readback(ctx)) != STP_OK) return rc;
            const double r = std::sqrt(ctx->host[RES_R2]);
            st.relres_proj = r / std::max(std::sqrt(ctx->host[RES_B2]), 1e-300);
            if (std::isfinite(r) && r < guess_res) {
                CHK(copy(ctx->p, ctx->ptmp, g.n, s));
                guess_res = r;
                st.proj_used = 1;
                st.extrap_used = 0;
            }
        }
    }
    if (c.warm_start == STP_WS_LEARNED) {
        if (!ctx->net) {
            ctx->err = "STP_WS_LEARNED needs stp_net_init";
            return STP_EINVAL;
        }
        // guess into ptmp; keep whichever of p^n and the guess has the smaller residual
        CHK(hipEventRecord(ctx->ev[4], s));
        CHK(ctx->net->predict(ctx->b, ctx->p, ctx->ptmp));
        CHK(hipEventRecord(ctx->ev[5], s));
        if (guess_res < 0.0) {
            CHK(residual(g, ctx->b, ctx->p, nullptr, ctx->part, ctx->res, s));
            if ((rc = readback(ctx)) != STP_OK) return rc;
            guess_res = std::sqrt(ctx->host[RES_R2]);
        }
        const double r_prev = guess_res;
        CHK(residual(g, ctx->b, ctx->ptmp, nullptr, ctx->part, ctx->res, s));
        if ((rc = readback(ctx)) != STP_OK) return rc;
        const double r_net = std::sqrt(ctx->host[RES_R2]);
        const double bn = std::sqrt(ctx->host[RES_B2]);
        const double fb = bn > 1e-300 ? bn : 1e-300;
        if (st.relres_prev == 0.0) st.relres_prev = r_prev / fb;  // not yet set by a candidate above
        st.relres_learned = r_net / fb;
        if (std::isfinite(r_net) && r_net < r_prev) {
            CHK(copy(ctx->p, ctx->ptmp, g.n, s));
            st.learned_used = 1;
        }
        float msn = 0.f;
        CHK(hipEventElapsedTime(&msn, ctx->ev[4], ctx->ev[5]));
        st.ms_net = msn;
    }
    CHK(hipEventRecord(ctx->ev[1], s));
    phase.next("stp_step: Poisson solve");
    if ((rc = solve(ctx, ctx->b, ctx->p, c.poisson_rtol, c.poisson_maxit, &st.poisson)) != STP_OK) {
        ctx->nproj = 0;
        return rc;
    }
    CHK(hipEventRecord(ctx->ev[2], s));
    phase.next("stp_step: projection");
    if (c.proj_depth > 0) {
        // only converged solutions enter the least-squares history
        if (st.poisson.status == STP_OK) {
            const int slot = ctx->step % c.proj_depth;
            CHK(copy(ctx->hp[slot], ctx->p, g.n, s));
            CHK(copy(ctx->hb[slot], ctx->b, g.n, s));
            ctx->nproj = std::min(ctx->nproj + 1, c.proj_depth);
        } else {
            ctx->nproj = 0;
        }
    }

    // 6. correction u = u* - dt grad p (Sec. 3.1)
    CHK(project(g, ctx->p, ctx->u, ctx->v, ctx->w, c.dt, s));

    // 7. diagnostics
    CHK(diagnostics(g, ctx->u, ctx->v, ctx->w, c.dt, ctx->part, ctx->res, s));
    CHK(hipEventRecord(ctx->ev[3], s));
    if ((rc = readback(ctx)) != STP_OK) return rc;
    phase.close();
    st.max_div = ctx->host[RES_DIAG + 0];
    st.u_bulk = ctx->host[RES_DIAG + 1] / (double)g.n;
    st.u_max = ctx->host[RES_DIAG + 2];
    st.cfl = ctx->host[RES_DIAG + 3];
    st.u_centre = ctx->host[RES_DIAG + 4] / (double)g.plane;
    st.nut_max = nut_max;
    float ms = 0.f;
    CHK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]));
    st.ms_total = ms;
    CHK(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
    st.ms_poisson = ms;
    const int bound[7] = {0, 6, 7, 8, 1, 2, 3};  // events between the phases, in order
    double* phase_ms[6] = {&st.ms_nut, &st.ms_momentum, &st.ms_divergence, &st.ms_guess, &st.ms_poisson,
                           &st.ms_projection};
    for (int q = 0; q < 6; ++q) {
        CHK(hipEventElapsedTime(&ms, ctx->ev[bound[q]], ctx->ev[bound[q + 1]]));
        *phase_ms[q] = ms;
    }
    ++ctx->step;
    st.step = ctx->step;
    if (out) *out = st;
    return (stp_status)st.poisson.status;
}

}  // namespace

// ---- static scratch of the allocation-free entry point ---------------------
// stp_residual_norm_noalloc keeps its reduction partials here instead of in a
// context's workspace: one partial per workgroup of the residual kernel (at
// most kMaxPartBlocks) and the reduced sum of squares after them.  Every GPU
// the library runs on holds its own copy, 512 KiB plus a few slots, until the
// process ends.  Host code must not pass `scratch` itself to a kernel (in
// host code the name stands for a host-side shadow, not a device address):
// it uses the address hipGetSymbolAddress returns on each device.
constexpr int kScratchDoubles = kMaxPartBlocks + 32;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};  // address of `scratch` on each device, once looked up
thread_local const char* g_noctx_err = "";  // message of the last failed context-free call

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current.
hipError_t scratch_on_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev] == nullptr) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (ptr == nullptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

stp_status noctx_fail(stp_status rc, const char* msg)
{
    g_noctx_err = msg;
    return rc;
}

}  // namespace

extern "C" {

stp_status stp_residual_norm_noalloc(int32_t nx, int32_t ny, int32_t nz, double lx, double ly, double lz,
                                     const void* b_dev, const void* p_dev, void* norm_dev, void* stream)
{
    g_noctx_err = "";
    if (!b_dev || !p_dev || !norm_dev) return noctx_fail(STP_EINVAL, "stp_residual_norm_noalloc: null pointer");
    if (const char* e = validate_grid(nx, ny, nz, lx, ly, lz)) return noctx_fail(STP_EINVAL, e);
    const Geo g = make_geo(nx, ny, nz, lx, ly, lz);
    if ((long long)march_shape(g, 2048).nblocks() + 1 > kScratchDoubles)
        return noctx_fail(STP_EINVAL, "stp_residual_norm_noalloc: grid needs more partials than the static scratch holds");
    double* sp = nullptr;
    if (scratch_on_current_device(&sp) != hipSuccess)
        return noctx_fail(STP_EDEVICE, "stp_residual_norm_noalloc: no device address for the static scratch");
    if (residual_norm_into(g, static_cast<const double*>(b_dev), static_cast<const double*>(p_dev), sp,
                           static_cast<double*>(norm_dev), static_cast<hipStream_t>(stream)) != hipSuccess)
        return noctx_fail(STP_EDEVICE, "stp_residual_norm_noalloc: kernel launch failed");
    return STP_OK;
}

size_t stp_workspace_bytes(const stp_config* cfg)
{
    if (!cfg) return 0;
    const stp_config c = effective(*cfg);
    if (validate(c)) return 0;
    return layout(c).total;
}

stp_status stp_init(const stp_config* cfg, void* ws, size_t bytes, stp_ctx** out)
{
    if (!cfg || !out) return STP_EINVAL;
    *out = nullptr;
    const stp_config c = effective(*cfg);
    if (validate(c)) return STP_EINVAL;
    const Layout L = layout(c);
    if (!ws || bytes < L.total) return STP_ENOMEM;
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return STP_EINVAL;
    stp_ctx* ctx = new (std::nothrow) stp_ctx();
    if (!ctx) return STP_ENOMEM;
    ctx->cfg = c;
    ctx->cfg.srj_omega = nullptr;  // copied below; the caller's array is not kept
    ctx->s = static_cast<hipStream_t>(c.stream);
    ctx->g = make_geo(c.nx, c.ny, c.nz, c.lx, c.ly, c.lz);
    const Geo& g = ctx->g;
    ctx->D = 2.0 * (g.idx2 + g.idy2 + g.idz2);
    char* base = static_cast<char*>(ws);
    ctx->u = (double*)(base + L.u);
    ctx->v = (double*)(base + L.v);
    ctx->w = (double*)(base + L.w);
    ctx->p = (double*)(base + L.p);
    ctx->ptmp = (double*)(base + L.ptmp);
    ctx->b = (double*)(base + L.b);
    const bool st32 = c.precision == STP_MIXED && c.stencils32;
    if (!st32) ctx->nut = (double*)(base + L.nut);
    for (int q = 0; q < 3; ++q) ctx->rhs[q] = (double*)(base + L.rhs[q]);
    ctx->tmp = (double*)(base + L.tmp);
    if (c.extrap_order >= 1) ctx->p1 = (double*)(base + L.p1);
    if (c.extrap_order >= 2) ctx->p2 = (double*)(base + L.p2);
    for (int j = 0; j < c.proj_depth; ++j) {
        ctx->hp[j] = (double*)(base + L.hp[j]);
        ctx->hb[j] = (double*)(base + L.hb[j]);
    }
    for (int sl = 0; sl < 3; ++sl)
        for (int q = 0; q < 3; ++q) {
            if (st32) ctx->e32[sl][q] = (float*)(base + L.e32[sl][q]);
            else ctx->e[sl][q] = (double*)(base + L.e[sl][q]);
        }
    if (st32) {
        ctx->u32 = (float*)(base + L.u32);
        ctx->ub = (double*)(base + L.ub);
        ctx->v32 = (float*)(base + L.v32);
        ctx->w32 = (float*)(base + L.w32);
    }
    ctx->e0 = (float*)(base + L.e0);
    ctx->e1 = (float*)(base + L.e1);
    ctx->r32 = (float*)(base + L.r32);
    if (c.precision == STP_MIXED && c.mixed_rhs16) ctx->r16 = (_Float16*)(base + L.r16);
    if (c.precision == STP_MIXED) {
        ctx->nut32 = (float*)(base + L.nut32);
        ctx->cnd = (float*)(base + L.cnd);
        ctx->cna = (float*)(base + L.cna);
        ctx->cnb = (float*)(base + L.cnb);
    }
    ctx->part = (double*)(base + L.part);
    ctx->res = (double*)(base + L.res);
    if (c.srj_m > 0) {
        ctx->omega.assign(c.srj_omega, c.srj_omega + c.srj_m);
    } else {
        double a, b;
        kappa_range(g, ctx->D, &a, &b);
        if (!(a > 0.0 && b > a)) {
            delete ctx;
            return STP_EINVAL;
        }
        ctx->kmin = a;
        ctx->kmax = b;
        ctx->omega = chebyshev_leja_cycle(a, b, c.srj_reduction);
    }
    if (hipGetDevice(&ctx->device) != hipSuccess || hipHostMalloc((void**)&ctx->host, RES_COUNT * sizeof(double)) != hipSuccess) {
        delete ctx;
        return STP_ENOMEM;
    }
    for (int q = 0; q < 9; ++q)
        if (hipEventCreate(&ctx->ev[q]) != hipSuccess) {
            stp_destroy(ctx);
            return STP_EDEVICE;
        }
    {
        const char* sync = std::getenv("STP_TRACE_SYNC");
        ctx->trace_sync = sync && sync[0] == '1';
    }
    // state at rest, empty history
    hipError_t e = hipSuccess;
    const long long nn = g.n, nw = g.nw;
    double* zero64[] = {ctx->u, ctx->v, ctx->p, ctx->ptmp, ctx->b, ctx->rhs[0], ctx->rhs[1]};
    for (double* a : zero64) if (e == hipSuccess) e = fill(a, 0.0, nn, ctx->s);
    if (e == hipSuccess) e = fill(ctx->w, 0.0, nw, ctx->s);
    if (e == hipSuccess) e = fill(ctx->rhs[2], 0.0, nw, ctx->s);
    if (e == hipSuccess) e = fill(ctx->tmp, 0.0, nw, ctx->s);
    if (e == hipSuccess && ctx->nut) e = fill(ctx->nut, c.nu, nn, ctx->s);
    if (e == hipSuccess && ctx->nut32) e = fill(ctx->nut32, (float)c.nu, nn, ctx->s);
    for (int sl = 0; sl < 3; ++sl)
        for (int q = 0; q < 3; ++q) {
            if (e == hipSuccess && ctx->e[sl][q]) e = fill(ctx->e[sl][q], 0.0, q == 2 ? nw : nn, ctx->s);
            if (e == hipSuccess && ctx->e32[sl][q]) e = fill(ctx->e32[sl][q], 0.0f, q == 2 ? nw : nn, ctx->s);
        }
    float* zero32[] = {ctx->e0, ctx->e1, ctx->r32};
    for (float* a : zero32) if (e == hipSuccess) e = fill(a, 0.0f, nn, ctx->s);
    if (e == hipSuccess) e = fill(ctx->res, 0.0, RES_COUNT, ctx->s);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->s);
    if (e != hipSuccess) {
        stp_destroy(ctx);
        return STP_EDEVICE;
    }
    *out = ctx;
    return STP_OK;
}

stp_status stp_step(stp_ctx* ctx, int32_t nsteps, stp_step_stats* last)
{
    if (!ctx) return STP_EINVAL;
    if (nsteps < 0) {
        ctx->err = "nsteps must be >= 0";
        return STP_EINVAL;
    }
    ctx->err.clear();
    for (int t = 0; t < nsteps; ++t) {
        stp_status rc = one_step(ctx, last);
        if (rc != STP_OK) {
            if (ctx->err.empty()) ctx->err = rc == STP_ENOCONV ? "Poisson solve did not converge" : "Poisson residual is not finite";
            return rc;
        }
    }
    return STP_OK;
}

stp_status stp_poisson_solve(stp_ctx* ctx, const void* b_dev, void* p_dev, double rtol, int32_t maxit,
                             stp_solve_stats* stats)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (!b_dev || !p_dev || !(rtol >= 0.0) || !std::isfinite(rtol) || maxit < 1) {
        ctx->err = "stp_poisson_solve: bad argument";
        return STP_EINVAL;
    }
    const double* b = static_cast<const double*>(b_dev);
    double* p = static_cast<double*>(p_dev);
    CHK(sumsq_into(b, ctx->g.n, ctx->part, ctx->res, RES_B2, ctx->s));
    stp_solve_stats st{};
    stp_status rc = solve(ctx, b, p, rtol, maxit, &st);
    if (rc != STP_OK) return rc;
    if (stats) *stats = st;
    if (st.status != STP_OK)
        ctx->err = st.status == STP_ENOCONV ? "Poisson solve did not converge" : "Poisson residual is not finite";
    return (stp_status)st.status;
}

stp_status stp_relax(stp_ctx* ctx, int32_t dtype, const void* b_dev, void* p_dev, const double* omega, int32_t nsweeps)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (!b_dev || !p_dev || nsweeps < 0 || (nsweeps > 0 && !omega) ||
        (dtype != STP_DTYPE_F64 && dtype != STP_DTYPE_F32 && dtype != STP_DTYPE_F32_RHS16)) {
        ctx->err = "stp_relax: bad argument";
        return STP_EINVAL;
    }
    for (int k = 0; k < nsweeps; ++k)
        if (!std::isfinite(omega[k])) {
            ctx->err = "stp_relax: non-finite weight";
            return STP_EINVAL;
        }
    stp_status rc;
    if (dtype == STP_DTYPE_F64) {
        double* p = static_cast<double*>(p_dev);
        double* cur = p;
        double* oth = ctx->ptmp;
        if ((rc = run_sweeps<double>(ctx, static_cast<const double*>(b_dev), &cur, &oth, omega, nsweeps, 0, nsweeps)) != STP_OK)
            return rc;
        if (cur != p) CHK(copy(p, cur, ctx->g.n, ctx->s));
    } else {
        float* p = static_cast<float*>(p_dev);
        float* cur = p;
        float* oth = ctx->e1;
        if (dtype == STP_DTYPE_F32)
            rc = run_sweeps<float>(ctx, static_cast<const float*>(b_dev), &cur, &oth, omega, nsweeps, 0, nsweeps);
        else
            rc = run_sweeps<float, _Float16>(ctx, static_cast<const _Float16*>(b_dev), &cur, &oth, omega, nsweeps, 0,
                                             nsweeps);
        if (rc != STP_OK) return rc;
        if (cur != p) CHK(copy(p, cur, ctx->g.n, ctx->s));
    }
    return STP_OK;
}

stp_status stp_residual_norm(stp_ctx* ctx, const void* b_dev, const void* p_dev, double* norm)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (!b_dev || !p_dev || !norm) {
        ctx->err = "stp_residual_norm: bad argument";
        return STP_EINVAL;
    }
    CHK(residual(ctx->g, static_cast<const double*>(b_dev), static_cast<const double*>(p_dev), nullptr, ctx->part,
                 ctx->res, ctx->s));
    stp_status rc = readback(ctx);
    if (rc != STP_OK) return rc;
    *norm = std::sqrt(ctx->host[RES_R2]);
    return STP_OK;
}

stp_status stp_lsq_guess(stp_ctx* ctx, int32_t k, const void* const* x_dev, const void* const* y_dev,
                         const void* b_dev, void* out_dev, int32_t* rank)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (k < 1 || k > kMaxProj || !x_dev || !y_dev || !b_dev || !out_dev || !rank) {
        ctx->err = "stp_lsq_guess: need 1 <= k <= 8 and non-null arrays";
        return STP_EINVAL;
    }
    const double* xs[kMaxProj];
    const double* ys[kMaxProj];
    for (int i = 0; i < k; ++i) {
        xs[i] = static_cast<const double*>(x_dev[i]);
        ys[i] = static_cast<const double*>(y_dev[i]);
        if (!xs[i] || !ys[i]) {
            ctx->err = "stp_lsq_guess: null history array";
            return STP_EINVAL;
        }
    }
    int r = 0;
    stp_status rc = lsq_guess(ctx, k, xs, ys, static_cast<const double*>(b_dev), static_cast<double*>(out_dev), &r);
    if (rc != STP_OK) return rc;
    *rank = r;
    CHK(hipStreamSynchronize(ctx->s));
    return STP_OK;
}

stp_status stp_fields(stp_ctx* ctx, int32_t field, void** dev_ptr, int64_t shape[3], int64_t strides[3],
                      int32_t* dtype, double offset[3])
{
    if (!ctx || !dev_ptr || !shape || !dtype) return STP_EINVAL;
    const Geo& g = ctx->g;
    const double dx = ctx->cfg.lx / g.nx, dy = ctx->cfg.ly / g.ny, dz = ctx->cfg.lz / g.nz;
    void* ptr = nullptr;
    int planes = g.nz;
    int32_t dt = STP_DTYPE_F64;
    // position of element [0][0][0] (z, y, x) on the staggered grid
    double oz = 0.5 * dz, oy = 0.5 * dy, ox = 0.5 * dx;
    switch (field) {
    case STP_U: ptr = ctx->u; ox = 0.0; break;
    case STP_V: ptr = ctx->v; oy = 0.0; break;
    case STP_W: ptr = ctx->w; planes = g.nz + 1; oz = 0.0; break;
    case STP_P: ptr = ctx->p; break;
    case STP_NUT:
        if (ctx->nut) {
            ptr = ctx->nut;
        } else {  // stencils32 keeps nu_T in FP32 only
            ptr = ctx->nut32;
            dt = STP_DTYPE_F32;
        }
        break;
    case STP_RHS: ptr = ctx->b; break;
    default:
        ctx->err = "stp_fields: unknown field";
        return STP_EINVAL;
    }
    *dev_ptr = ptr;
    shape[0] = planes;
    shape[1] = g.ny;
    shape[2] = g.nx;
    *dtype = dt;
    if (strides) {
        strides[0] = g.plane;
        strides[1] = g.nx;
        strides[2] = 1;
    }
    if (offset) {
        offset[0] = oz;
        offset[1] = oy;
        offset[2] = ox;
    }
    return STP_OK;
}

stp_status stp_plane_stats(stp_ctx* ctx, double* out)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (!out) {
        ctx->err = "stp_plane_stats: NULL output";
        return STP_EINVAL;
    }
    const size_t count = (size_t)kPlaneStats * (ctx->g.nz + 1);
    if (count > (size_t)kMaxPartBlocks * 8) {
        ctx->err = "stp_plane_stats: too many planes for the partials";
        return STP_EINVAL;
    }
    if (!ctx->nut) CHK(plane_stats(ctx->g, ctx->u, ctx->v, ctx->w, ctx->nut32, ctx->part, ctx->s));
    else CHK(plane_stats(ctx->g, ctx->u, ctx->v, ctx->w, ctx->nut, ctx->part, ctx->s));
    CHK(hipMemcpyAsync(out, ctx->part, count * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
    CHK(hipStreamSynchronize(ctx->s));
    return STP_OK;
}

stp_status stp_get_state(const stp_ctx* ctx, stp_state* out)
{
    if (!ctx || !out) return STP_EINVAL;
    out->step = ctx->step;
    out->nhist = ctx->nhist;
    out->nproj = ctx->nproj;
    return STP_OK;
}

stp_status stp_set_state(stp_ctx* ctx, const stp_state* in)
{
    if (!ctx || !in || in->step < 0 || in->nhist < 0 || in->nhist > ctx->cfg.extrap_order || in->nproj < 0 ||
        in->nproj > ctx->cfg.proj_depth)
        return STP_EINVAL;
    ctx->step = in->step;
    ctx->nhist = in->nhist;
    ctx->nproj = in->nproj;
    return STP_OK;
}

stp_status stp_schedule(const stp_ctx* ctx, double* omega, int32_t cap, int32_t* m)
{
    if (!ctx || !m || cap < 0 || (cap > 0 && !omega)) return STP_EINVAL;
    *m = (int32_t)ctx->omega.size();
    for (int k = 0; k < cap && k < *m; ++k) omega[k] = ctx->omega[k];
    return STP_OK;
}

size_t stp_net_workspace_bytes(const stp_ctx* ctx, int32_t training)
{
    if (!ctx) return 0;
    return stp::NetModel::workspace_bytes(ctx->g.nx, ctx->g.ny, ctx->g.nz, training != 0);
}

stp_status stp_net_init(stp_ctx* ctx, void* ws, size_t bytes, int32_t training, uint64_t seed)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    const size_t need = stp::NetModel::workspace_bytes(ctx->g.nx, ctx->g.ny, ctx->g.nz, training != 0);
    if (need == 0) {
        ctx->err = "stp_net_init: grid dimensions must be divisible by 4";
        return STP_EINVAL;
    }
    if (!ws || bytes < need) {
        ctx->err = "stp_net_init: workspace too small";
        return STP_ENOMEM;
    }
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
        ctx->err = "stp_net_init: workspace must be 256-byte aligned";
        return STP_EINVAL;
    }
    delete ctx->net;
    ctx->net = new (std::nothrow) stp::NetModel(ctx->g.nx, ctx->g.ny, ctx->g.nz, ctx->g.idx2, ctx->g.idy2, ctx->g.idz2,
                                                training != 0, ws, ctx->s);
    if (!ctx->net) return STP_ENOMEM;
    CHK(ctx->net->init_params(seed));
    CHK(hipStreamSynchronize(ctx->s));
    return STP_OK;
}

stp_status stp_net_params(stp_ctx* ctx, float** params, float** grads, int64_t* count)
{
    if (!ctx || !ctx->net || !params || !count) return STP_EINVAL;
    *params = ctx->net->params();
    if (grads) *grads = ctx->net->grads();
    *count = ctx->net->param_count();
    return STP_OK;
}

stp_status stp_net_layout(const stp_ctx* ctx, int32_t layer, int64_t out[6])
{
    if (!ctx || !ctx->net || !out || layer < 0 || layer >= stp::NetModel::kLayers) return STP_EINVAL;
    const stp::NetLayer& l = ctx->net->layer(layer);
    out[0] = l.w_off;
    out[1] = l.b_off;
    out[2] = l.cin;
    out[3] = l.cout;
    out[4] = l.cin_logical;
    out[5] = l.cout_logical;
    return STP_OK;
}

stp_status stp_net_sync(stp_ctx* ctx)
{
    if (!ctx || !ctx->net) return STP_EINVAL;
    ctx->err.clear();
    CHK(ctx->net->sync());
    return STP_OK;
}

stp_status stp_net_predict(stp_ctx* ctx, const void* b, const void* p_prev, void* p_guess)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (!ctx->net || !b || !p_prev || !p_guess) {
        ctx->err = "stp_net_predict: network not initialised or NULL argument";
        return STP_EINVAL;
    }
    CHK(ctx->net->predict(static_cast<const double*>(b), static_cast<const double*>(p_prev),
                          static_cast<double*>(p_guess)));
    return STP_OK;
}

stp_status stp_net_train_step(stp_ctx* ctx, const void* b, const void* p_prev, const void* p_next, float lr,
                              double* loss)
{
    if (!ctx) return STP_EINVAL;
    ctx->err.clear();
    if (!ctx->net || !b || !p_prev || !p_next || !(lr >= 0.f) || !std::isfinite(lr)) {
        ctx->err = "stp_net_train_step: network not initialised for training or bad argument";
        return STP_EINVAL;
    }
    CHK(ctx->net->train_step(static_cast<const double*>(b), static_cast<const double*>(p_prev),
                             static_cast<const double*>(p_next), lr, ctx->res + RES_NET_LOSS));
    if (loss) {
        stp_status rc = readback(ctx);
        if (rc != STP_OK) return rc;
        *loss = ctx->host[RES_NET_LOSS];
    }
    return STP_OK;
}

stp_status stp_destroy(stp_ctx* ctx)
{
    if (!ctx) return STP_OK;
    for (int q = 0; q < 9; ++q)
        if (ctx->ev[q]) (void)hipEventDestroy(ctx->ev[q]);
    if (ctx->host) (void)hipHostFree(ctx->host);
    delete ctx->net;
    delete ctx;
    return STP_OK;
}

const char* stp_last_error(const stp_ctx* ctx)
{
    if (!ctx) return g_noctx_err[0] ? g_noctx_err : "null context";
    return ctx->err.c_str();
}

}  // extern "C"
