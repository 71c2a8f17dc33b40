// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace stp {

// Grid geometry handed to every kernel by value.
struct Geo {
    int nx, ny, nz;
    long long plane;  // nx*ny
    long long n;      // nx*ny*nz cells
    long long nw;     // nx*ny*(nz+1) z-faces
    double idx, idy, idz;     // 1/h
    double idx2, idy2, idz2;  // 1/h^2
};

// Launch shape of the z-marching stencil kernels: a (bx, by) tile of columns
// per workgroup, kchunk planes per workgroup along z.
struct March {
    dim3 grid, block;
    int kchunk;
    int nblocks() const { return (int)(grid.x * grid.y * grid.z); }
};
March march_shape(const Geo& g, int min_blocks);

// Slots of the device scalar-result array.
enum ResSlot {
    RES_SUM_B = 0,   // sum b (before mean removal)
    RES_B2 = 1,      // sum (b - mean)^2
    RES_R2 = 2,      // sum r^2 of the last residual
    RES_SUM_P = 3,   // sum p
    RES_NUT_MAX = 4,
    RES_NET_LOSS = 5,
    RES_DIAG = 8,    // 5 values: max|div|, sum u, max|u|, max cfl, centreline sum
    RES_PROJ = 16,   // Gram matrix and right-hand side of the least-squares guess
    RES_COUNT = 64
};

constexpr int kMaxPartBlocks = 65536;  // partial-sum slots per reduced quantity
constexpr int kMaxFused = 5;           // sweeps fused per relaxation launch (FP64: 4)
constexpr int kMaxProj = 8;            // earlier solutions in the least-squares guess
static_assert(RES_PROJ + kMaxProj * (kMaxProj + 1) / 2 + kMaxProj <= RES_COUNT, "result slots");

struct Weights {  // omega_s of the fused sweeps of one launch
    double omega[kMaxFused];
};

// ---- launchers (all enqueue on `s`, return hipError of the launch) ----
hipError_t fill(double* a, double v, long long n, hipStream_t s);
hipError_t fill(float* a, float v, long long n, hipStream_t s);
hipError_t copy(double* dst, const double* src, long long n, hipStream_t s);
hipError_t copy(float* dst, const float* src, long long n, hipStream_t s);
// out = 2p - p1 (order 1) or 3(p - p1) + p2 (order 2)
hipError_t extrapolate(const double* p, const double* p1, const double* p2, int order, double* out, long long n,
                       hipStream_t s);
// Least-squares guess from k <= kMaxProj earlier solutions x[0..k-1] and their
// right-hand sides y[0..k-1] (newest first), both entering through their
// backward differences at the newest, E_0 = y_0, E_j = sum_i (-1)^i C(j, i) y_i.
// proj_gram writes <E_i, E_j> (i <= j, row by row) and then <E_i, b> into
// res[slot ...]; proj_combine writes out = sum_j a[j] F_j with F the
// differences of the x.
hipError_t proj_gram(int k, const double* const* y, const double* b, long long n, double* part, double* res,
                     int slot, hipStream_t s);
hipError_t proj_combine(int k, const double* const* x, const double* a, double* out, long long n, hipStream_t s);
hipError_t sumsq_into(const double* a, long long n, double* part, double* res, int slot, hipStream_t s);
hipError_t zero_walls(const Geo& g, double* w, hipStream_t s);

// nu_T from velocities stored as T (FP64, or FP32 copies in the mixed mode),
// written as T; max nu_T into res[RES_NUT_MAX].  For T = float, u holds the
// departure u - ub[k] from the FP64 plane profile ub (round_departure_f32);
// ub is unused for T = double.
template <typename T>
hipError_t nut_smagorinsky(const Geo& g, const T* u, const T* v, const T* w, T* nut, double nu, double cs_delta,
                           double inv_wall_unit, double lz, const double* ub, double* part, double* res,
                           hipStream_t s);

// Explicit terms E^n and the Crank-Nicolson right-hand side R for component
// c, with the stencils in T (velocities, nu_T and the Adams-Bashforth
// history stored as T) and R in FP64: for T = float R = x64 + the FP32
// increment, x64 the component's FP64 state, and u holds u - ub[k] (both
// unused for T = double).
template <typename T>
struct MomArgsT {
    const T *u, *v, *w, *nut;
    const double* ub;  // plane profile of u (T = float)
    T* en;          // E^n out
    const T* e1;    // E^{n-1}
    const T* e2;    // E^{n-2}
    double* rhs;    // R out
    const double* x64;
    double beta0, beta1, beta2;
    double dt, half_dt, dpdx, nu;
};
using MomArgs = MomArgsT<double>;
template <typename T>
hipError_t momentum_rhs(const Geo& g, int comp, const MomArgsT<T>& a, hipStream_t s);

// One Crank-Nicolson iteration x_out = x + (R - (I - h L) x) * inv_shift.
hipError_t cn_iterate(const Geo& g, int comp, const double* nut, double nu, const double* rhs, const double* x,
                      double* xout, double half_dt, double inv_shift, hipStream_t s);
// one Crank-Nicolson iteration in defect form (mixed mode): phase 0 from R,
// phase 1 delta -> delta, phase 2 delta -> u* = R + delta (FP64)
hipError_t cn_defect(const Geo& g, int comp, int phase, const float* nut32, double nu, const double* rhs,
                     const float* d0in, float* d0out, const float* x, float* xo, double* uo, double half_dt,
                     double inv_shift, hipStream_t s);
hipError_t round_to_f32(float* dst, const double* src, long long n, hipStream_t s);
// ub[k] = plane mean of the cell field src on plane k (nz doubles), then
// dst = FP32(src - ub[k]): the FP32 copy of u the mixed-mode stencils read
hipError_t round_departure_f32(const Geo& g, float* dst, const double* src, double* ub, hipStream_t s);

hipError_t divergence_rhs(const Geo& g, const double* u, const double* v, const double* w, double* b,
                          double inv_dt, double* part, double* res, hipStream_t s);
hipError_t remove_mean(double* a, long long n, const double* res_sum, int res_out_sq, double* part, double* res,
                       hipStream_t s);  // a -= res_sum[0]/n; optional sum of squares into res[res_out_sq]
hipError_t sum_into(const double* a, long long n, double* part, double* res, int slot, hipStream_t s);

// nfused = 1 (any grid) or 2..kMaxFused (FP64: 2..4) on grids with nx >= 64
// and ny >= 32.
bool relax_fusable(const Geo& g);
// FP32 sweeps fused per launch when the caller leaves the choice to the
// library: 5 where the tall five-sweep tiles fit (ny >= 66); on narrower
// grids 4 when a four-sweep launch fits one round of resident workgroups,
// else 5 (1 on grids that cannot fuse).
int relax_auto_depth(const Geo& g);
template <typename T>
hipError_t relax(const Geo& g, const T* b, const T* p, T* out, const Weights& wts, int nfused, hipStream_t s);
// FP32 sweeps whose right-hand side is stored in FP16 (widened exactly on load)
hipError_t relax(const Geo& g, const _Float16* b, const float* p, float* out, const Weights& wts, int nfused,
                 hipStream_t s);

// r = b - L p (FP64); sum r^2 -> res[RES_R2]; optional FP32 copy of
// r32_scale * r (r32_scale a power of two, so the copy rounds r alone).
hipError_t residual(const Geo& g, const double* b, const double* p, float* r32, double* part, double* res,
                    hipStream_t s, double r32_scale = 1.0);
// ||b - L p||_2 written to the device double *norm; part holds the partials
// (march_shape(g, 2048).nblocks() + 1 doubles, every one written before it is read).
hipError_t residual_norm_into(const Geo& g, const double* b, const double* p, double* part, double* norm,
                              hipStream_t s);
hipError_t add_correction(double* p, const float* e, long long n, hipStream_t s);
hipError_t add_correction_scaled(double* p, const float* e, long long n, double inv_scale, hipStream_t s);
// dst = FP16(scale * r), scale a power of two
hipError_t half_scaled(_Float16* dst, const float* r, long long n, float scale, hipStream_t s);

hipError_t project(const Geo& g, const double* p, double* u, double* v, double* w, double dt, hipStream_t s);
hipError_t diagnostics(const Geo& g, const double* u, const double* v, const double* w, double dt, double* part,
                       double* res, hipStream_t s);
// Plane means at every height (kPlaneStats quantities, see k_plane_stats)
// into out[q (nz + 1) + k], a device array of kPlaneStats (nz + 1) doubles.
constexpr int kPlaneStats = 8;
template <typename TN>
hipError_t plane_stats(const Geo& g, const double* u, const double* v, const double* w, const TN* nut, double* out,
                       hipStream_t s);

}  // namespace stp
