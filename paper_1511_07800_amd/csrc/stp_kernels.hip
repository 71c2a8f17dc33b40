// HIP kernels for gfx950 (CDNA4): the stencils, relaxation sweeps and
// reductions of the S-TPLS time step (arXiv 1511.07800, Sec. 2-3).
//
// Every kernel here is bandwidth-bound (a few flops per byte), so the design
// rules are: x-fastest coalesced rows, one thread per (i, j) column marching
// along z with the vertical neighbours kept in registers, periodic wrap in x
// and y computed in-kernel, and reductions as fixed-order wave64 shuffle trees
// with per-workgroup partials (bitwise reproducible, no float atomics).
#include "stp_internal.h"

#include <algorithm>
#include <type_traits>

namespace stp {

namespace {

constexpr int kBlock1d = 256;

__device__ __forceinline__ int wm(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wp(int i, int n) { return i == n - 1 ? 0 : i + 1; }

__device__ __forceinline__ long long at(const Geo& g, int i, int j, int k)
{
    return (long long)i + (long long)g.nx * j + g.plane * k;
}

// Reference profile of u in the mixed mode.  The FP32 copy of u holds the
// departure u - ub[k] from a per-plane reference (the plane mean), so the
// copy rounds the departure only and differences of it are exact in the
// mean; the stencils add the reference's own contribution from the FP64
// profile.  The odd wall ghost of u continues the profile as -ub[0] below the
// bottom plane and -ub[nz - 1] above the top one.
struct URef {
    const double* __restrict__ ub;
    int nz;
    __device__ double at(int k) const { return k < 0 ? -ub[0] : (k >= nz ? -ub[nz - 1] : ub[k]); }
    __device__ float mean(int k) const { return (float)ub[k]; }
    // ub(k + 1) - ub(k), and the mean on the z-edge between planes k and k + 1
    __device__ float dz(int k) const { return (float)(at(k + 1) - at(k)); }
    __device__ float edge(int k) const { return (float)(0.5 * (at(k) + at(k + 1))); }
};
template <typename T>
constexpr bool kRefU = std::is_same<T, float>::value;

// ---- fixed-order reductions -------------------------------------------------

template <bool MAX>
__device__ __forceinline__ double wave_reduce(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(v, off, 64);
        v = MAX ? fmax(v, o) : v + o;
    }
    return v;
}

// Reduce one value per thread of the workgroup; thread 0 gets the result.
template <bool MAX>
__device__ double block_reduce(double v, double* lds /* >= 16 */)
{
    const int lane = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
    v = wave_reduce<MAX>(v);
    __syncthreads();
    if ((lane & 63) == 0) lds[lane >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (lane == 0) {
        r = lds[0];
        for (int wv = 1; wv < (nthreads + 63) / 64; ++wv) r = MAX ? fmax(r, lds[wv]) : r + lds[wv];
    }
    return r;
}

__device__ __forceinline__ int block_id()
{
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ __forceinline__ int block_count() { return gridDim.x * gridDim.y * gridDim.z; }

// Second stage: nq quantities, each with nblk partials laid out part[q*nblk + b].
// Bit q of max_mask selects max instead of sum.  Writes res[slot + q].
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ part, int nblk, int nq,
                                                  unsigned max_mask, double* __restrict__ res, int slot)
{
    __shared__ double lds[16];
    for (int q = 0; q < nq; ++q) {
        const bool mx = (max_mask >> q) & 1u;
        double v = mx ? -INFINITY : 0.0;
        for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
            const double x = part[(long long)q * nblk + b];
            v = mx ? fmax(v, x) : v + x;
        }
        const double r = mx ? block_reduce<true>(v, lds) : block_reduce<false>(v, lds);
        if (threadIdx.x == 0) res[slot + q] = r;
        __syncthreads();
    }
}

hipError_t finalize(const double* part, int nblk, int nq, unsigned max_mask, double* res, int slot, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, part, nblk, nq, max_mask, res, slot);
    return hipGetLastError();
}

int grid1d(long long n, int cap = 4096)
{
    long long b = (n + kBlock1d - 1) / kBlock1d;
    return (int)std::max<long long>(1, std::min<long long>(b, cap));
}

// ---- elementwise ------------------------------------------------------------

template <typename T>
__global__ void k_fill(T* __restrict__ a, T v, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        a[q] = v;
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        d[q] = s[q];
}

// Polynomial extrapolation in time of the last solutions p = p^n, p1 = p^{n-1},
// p2 = p^{n-2} to the next step: order 1 gives 2p - p1, order 2 gives
// 3(p - p1) + p2.
__global__ void k_extrapolate(const double* __restrict__ p, const double* __restrict__ p1,
                              const double* __restrict__ p2, int order, double* __restrict__ out, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        out[q] = order == 1 ? 2.0 * p[q] - p1[q] : 3.0 * (p[q] - p1[q]) + p2[q];
}

// ---- least-squares guess from earlier solutions ------------------------------
// The right-hand sides y_0 (newest), y_1, ... of earlier steps and their
// solutions x_0, x_1, ... enter through backward differences at the newest
// (E_0 = y_0, E_j = sum_i (-1)^i C(j, i) y_i), formed per cell in registers.
// Along a trajectory smooth in time the differences fall off by orders of
// magnitude; in this basis, scaled to unit diagonal, the normal equations are
// well conditioned where those of the raw vectors are not.

struct HistPtrs {
    const double* a[kMaxProj];
};
struct ProjCoef {
    double a[kMaxProj];
};

// v[j] <- j-th backward difference at v[0], in place
template <int K>
__device__ __forceinline__ void backward_differences(double (&v)[K])
{
#pragma unroll
    for (int j = 1; j < K; ++j)
#pragma unroll
        for (int i = K - 1; i >= j; --i) v[i] = v[i - 1] - v[i];
}

// Per-workgroup partial sums of <E_i, E_j> (i <= j, row by row) and then
// <E_i, b>: NQ = K(K+1)/2 + K quantities, part[q * gridDim.x + block].
template <int K>
__global__ __launch_bounds__(256) void k_proj_gram(HistPtrs y, const double* __restrict__ b, long long n,
                                                   double* __restrict__ part)
{
    constexpr int NQ = K * (K + 1) / 2 + K;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        double v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = y.a[j][c];
        const double bc = b[c];
        backward_differences<K>(v);
        int q = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = i; j < K; ++j) acc[q++] += v[i] * v[j];
#pragma unroll
        for (int i = 0; i < K; ++i) acc[q++] += v[i] * bc;
    }
    __shared__ double lds[kBlock1d / 64][NQ];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double r = wave_reduce<false>(acc[q]);
        if (lane == 0) lds[wave][q] = r;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NQ; q += blockDim.x) {
        double r = lds[0][q];
        for (int w = 1; w < kBlock1d / 64; ++w) r += lds[w][q];
        part[(long long)q * gridDim.x + blockIdx.x] = r;
    }
}

// One workgroup per quantity: res[slot + q] = sum over blocks of part[q * nblk + block].
__global__ __launch_bounds__(256) void k_finalize_each(const double* __restrict__ part, int nblk,
                                                       double* __restrict__ res, int slot)
{
    __shared__ double lds[16];
    const int q = blockIdx.x;
    double v = 0.0;
    for (int blk = threadIdx.x; blk < nblk; blk += blockDim.x) v += part[(long long)q * nblk + blk];
    const double r = block_reduce<false>(v, lds);
    if (threadIdx.x == 0) res[slot + q] = r;
}

template <int K>
__global__ void k_proj_combine(HistPtrs x, ProjCoef a, double* __restrict__ out, long long n)
{
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        double v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = x.a[j][c];
        backward_differences<K>(v);
        double s = a.a[0] * v[0];
#pragma unroll
        for (int j = 1; j < K; ++j) s += a.a[j] * v[j];
        out[c] = s;
    }
}

__global__ void k_copy32(float* __restrict__ d, const float* __restrict__ s, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        d[q] = s[q];
}

__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ a, long long n, double* __restrict__ part)
{
    __shared__ double lds[16];
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        acc += a[q] * a[q];
    const double r = block_reduce<false>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void k_zero_walls(Geo g, double* __restrict__ w)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < g.plane; q += (long long)gridDim.x * blockDim.x) {
        w[q] = 0.0;
        w[g.plane * g.nz + q] = 0.0;
    }
}

// a -= sum/n; optionally partial sums of the squared result.
__global__ __launch_bounds__(256) void k_remove_mean(double* __restrict__ a, long long n,
                                                     const double* __restrict__ sum, double* __restrict__ part,
                                                     int want_sq)
{
    __shared__ double lds[16];
    const double m = sum[0] / (double)n;
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const double x = a[q] - m;
        a[q] = x;
        acc += x * x;
    }
    if (want_sq) {
        const double r = block_reduce<false>(acc, lds);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ a, long long n, double* __restrict__ part)
{
    __shared__ double lds[16];
    double acc = 0.0;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        acc += a[q];
    const double r = block_reduce<false>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void k_add_correction(double* __restrict__ p, const float* __restrict__ e, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] += (double)e[q];
}

// p += e / scale: the correction of a pass whose right-hand side was scaled by
// `scale` (a power of two, so the product is exact)
__global__ void k_add_correction_scaled(double* __restrict__ p, const float* __restrict__ e, long long n,
                                        double inv_scale)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        p[q] += inv_scale * (double)e[q];
}

// FP16 copy of scale * r (round to nearest); scale, a power of two, brings the
// rms of r to about 1
__global__ void k_half_scaled(_Float16* __restrict__ d, const float* __restrict__ r, long long n, float scale)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        d[q] = (_Float16)(scale * r[q]);
}

// ---- eddy viscosity (Sec. 2.2) ---------------------------------------------

// nu_T = nu + (C_S Delta phi_w)^2 |S| at cell centres; phi_w = 1 - exp(-z+/A)
// with z+ the distance to the nearer wall times u_tau/nu.  |S|^2 =
// 2(S11^2 + S22^2 + S33^2) + 4(<S12^2> + <S13^2> + <S23^2>), <.> the mean over
// the four edges around the centre; u, v odd and w zero at the walls.
// T: the type the velocities and nu_T are stored and computed in (FP64, or
// FP32 in the mixed mode); the maximum is reduced in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_nut(Geo g, int kchunk, const T* __restrict__ u, const T* __restrict__ v,
                                             const T* __restrict__ w, T* __restrict__ nut, double nu_d,
                                             double cs_delta_d, double inv_wall_unit_d, double lz_d,
                                             const double* __restrict__ ub, double* __restrict__ part)
{
    const URef R{ub, g.nz};  // FP32 only: u holds u - ub (see URef)
    __shared__ double lds[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double vmax = -INFINITY;
    const T idx = (T)g.idx, idy = (T)g.idy, idz = (T)g.idz;
    const T nu = (T)nu_d, cs_delta = (T)cs_delta_d, inv_wall_unit = (T)inv_wall_unit_d, lz = (T)lz_d;
    const T h = T(0.5), q = T(0.25);
    if (i < g.nx && j < g.ny) {
        const int im = wm(i, g.nx), ip = wp(i, g.nx), jm = wm(j, g.ny), jp = wp(j, g.ny);
        const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
        const T dz = T(1.0) / idz;
        // u and v with the odd wall ghosts; w's wall planes hold 0
        auto U = [&](int ii, int jj, int kk) -> T {
            if (kk < 0) return -u[at(g, ii, jj, 0)];
            if (kk >= g.nz) return -u[at(g, ii, jj, g.nz - 1)];
            return u[at(g, ii, jj, kk)];
        };
        auto V = [&](int ii, int jj, int kk) -> T {
            if (kk < 0) return -v[at(g, ii, jj, 0)];
            if (kk >= g.nz) return -v[at(g, ii, jj, g.nz - 1)];
            return v[at(g, ii, jj, kk)];
        };
        auto Wf = [&](int ii, int jj, int kk) -> T { return w[at(g, ii, jj, kk)]; };
        const int is[2] = {i, ip}, ism[2] = {im, i};
        const int js[2] = {j, jp}, jsm[2] = {jm, j};
        // x-z edge (i + di, kk) on row j and y-z edge (j + di, kk) on column i
        // d_z u across the edge above plane kk - 1 (the profile's part added
        // for the FP32 departure)
        auto duz = [&](int ii, int kk) -> T {
            if constexpr (kRefU<T>) return (U(ii, j, kk) - U(ii, j, kk - 1)) + R.dz(kk - 1);
            else return U(ii, j, kk) - U(ii, j, kk - 1);
        };
        auto s13at = [&](int di, int kk) {
            return h * (duz(is[di], kk) * idz + (Wf(is[di], j, kk) - Wf(ism[di], j, kk)) * idx);
        };
        auto s23at = [&](int di, int kk) {
            return h * ((V(i, js[di], kk) - V(i, js[di], kk - 1)) * idz + (Wf(i, js[di], kk) - Wf(i, jsm[di], kk)) * idy);
        };
        // Along the march the edges above plane k become the edges below
        // plane k + 1, and the column's values on plane k + 1 are those of the
        // next step: both stay in registers.
        T s13lo[2] = {s13at(0, k0), s13at(1, k0)}, s23lo[2] = {s23at(0, k0), s23at(1, k0)};
        T uc = U(i, j, k0), ue = U(ip, j, k0), vc = V(i, j, k0), vn = V(i, jp, k0), wc = Wf(i, j, k0);
        for (int k = k0; k < k1; ++k) {
            const T uS = U(i, jm, k), uSE = U(ip, jm, k), uN = U(i, jp, k), uNE = U(ip, jp, k);
            const T vW = V(im, j, k), vE = V(ip, j, k), vNW = V(im, jp, k), vNE = V(ip, jp, k);
            const T uc1 = U(i, j, k + 1), ue1 = U(ip, j, k + 1), vc1 = V(i, j, k + 1), vn1 = V(i, jp, k + 1);
            const T wc1 = Wf(i, j, k + 1), we1 = Wf(ip, j, k + 1), ww1 = Wf(im, j, k + 1);
            const T wn1 = Wf(i, jp, k + 1), ws1 = Wf(i, jm, k + 1);
            const T s11 = (ue - uc) * idx;
            const T s22 = (vn - vc) * idy;
            const T s33 = (wc1 - wc) * idz;
            T duc = uc1 - uc, due = ue1 - ue;
            if constexpr (kRefU<T>) {
                const T d = R.dz(k);
                duc += d;
                due += d;
            }
            const T s13hi[2] = {h * (duc * idz + (wc1 - ww1) * idx), h * (due * idz + (we1 - wc1) * idx)};
            const T s23hi[2] = {h * ((vc1 - vc) * idz + (wc1 - ws1) * idy), h * ((vn1 - vn) * idz + (wn1 - wc1) * idy)};
            // x-y edges (i + di, j + dj) on plane k
            const T s12[4] = {h * ((uc - uS) * idy + (vc - vW) * idx), h * ((ue - uSE) * idy + (vE - vc) * idx),
                              h * ((uN - uc) * idy + (vn - vNW) * idx), h * ((uNE - ue) * idy + (vNE - vn) * idx)};
            T a12 = T(0), a13 = T(0), a23 = T(0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int di = e & 1, dj = e >> 1;
                const T s13 = dj ? s13hi[di] : s13lo[di];
                const T s23 = dj ? s23hi[di] : s23lo[di];
                a12 += q * s12[e] * s12[e];
                a13 += q * s13 * s13;
                a23 += q * s23 * s23;
            }
            const T s2 = T(2.0) * (s11 * s11 + s22 * s22 + s33 * s33) + T(4.0) * (a12 + a13 + a23);
            const T zc = ((T)k + h) * dz;
            const T dwall = fmin(zc, lz - zc);
            const T l = cs_delta * (T(1.0) - exp(-dwall * inv_wall_unit));
            const T val = nu + l * l * sqrt(s2);
            nut[at(g, i, j, k)] = val;
            vmax = fmax(vmax, (double)val);
            s13lo[0] = s13hi[0];
            s13lo[1] = s13hi[1];
            s23lo[0] = s23hi[0];
            s23lo[1] = s23hi[1];
            uc = uc1;
            ue = ue1;
            vc = vc1;
            vn = vn1;
            wc = wc1;
        }
    }
    const double r = block_reduce<true>(vmax, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = r;
}

// ---- momentum: explicit terms and Crank-Nicolson right-hand side (Sec. 3.1)

// Edge viscosities: mean of the four surrounding centres; nu on wall edges.
// nu_T at centres (stored as TN) and its averages on edges, evaluated in TC
template <typename TN, typename TC>
struct NuT {
    const TN* __restrict__ t;
    Geo g;
    TC nu;
    __device__ TC c(int i, int j, int k) const { return (TC)t[at(g, i, j, k)]; }
    // x-y edge between centres (i0|i1) x (j0|j1) on plane k
    __device__ TC xy(int i0, int i1, int j0, int j1, int k) const
    {
        return TC(0.25) * (c(i0, j0, k) + c(i1, j0, k) + c(i0, j1, k) + c(i1, j1, k));
    }
    // x-z edge between centres (i0|i1) x (k-1|k) on row j; wall edges carry nu
    __device__ TC xz(int i0, int i1, int j, int k) const
    {
        if (k <= 0 || k >= g.nz) return nu;
        return TC(0.25) * (c(i0, j, k - 1) + c(i1, j, k - 1) + c(i0, j, k) + c(i1, j, k));
    }
    __device__ TC yz(int i, int j0, int j1, int k) const
    {
        if (k <= 0 || k >= g.nz) return nu;
        return TC(0.25) * (c(i, j0, k - 1) + c(i, j1, k - 1) + c(i, j0, k) + c(i, j1, k));
    }
};
using Nu = NuT<double, double>;

// L_nu x = d_j(nu_T d_j x) for velocity component COMP at face (i, j, k)
// (flat index c), in arithmetic TC: odd ghosts of u, v at the walls; w is
// not evaluated on its wall planes.
template <int COMP, typename TC, typename TX, typename TN>
__device__ __forceinline__ TC visc_apply(const Geo& g, const NuT<TN, TC>& N, const TX* __restrict__ x, long long c,
                                         int i, int j, int k, int im, int ip, int jm, int jp)
{
    const TC xc = (TC)x[c];
    const TC xE = (TC)x[at(g, ip, j, k)], xW = (TC)x[at(g, im, j, k)];
    const TC xN = (TC)x[at(g, i, jp, k)], xS = (TC)x[at(g, i, jm, k)];
    const TC idx2 = (TC)g.idx2, idy2 = (TC)g.idy2, idz2 = (TC)g.idz2;
    if (COMP == 0) {
        const TC xT = k + 1 < g.nz ? (TC)x[c + g.plane] : -xc;
        const TC xB = k > 0 ? (TC)x[c - g.plane] : -xc;
        return (N.c(i, j, k) * (xE - xc) - N.c(im, j, k) * (xc - xW)) * idx2 +
               (N.xy(im, i, j, jp, k) * (xN - xc) - N.xy(im, i, jm, j, k) * (xc - xS)) * idy2 +
               (N.xz(im, i, j, k + 1) * (xT - xc) - N.xz(im, i, j, k) * (xc - xB)) * idz2;
    } else if (COMP == 1) {
        const TC xT = k + 1 < g.nz ? (TC)x[c + g.plane] : -xc;
        const TC xB = k > 0 ? (TC)x[c - g.plane] : -xc;
        return (N.xy(i, ip, jm, j, k) * (xE - xc) - N.xy(im, i, jm, j, k) * (xc - xW)) * idx2 +
               (N.c(i, j, k) * (xN - xc) - N.c(i, jm, k) * (xc - xS)) * idy2 +
               (N.yz(i, jm, j, k + 1) * (xT - xc) - N.yz(i, jm, j, k) * (xc - xB)) * idz2;
    } else {
        const TC xT = (TC)x[c + g.plane], xB = (TC)x[c - g.plane];
        return (N.xz(i, ip, j, k) * (xE - xc) - N.xz(im, i, j, k) * (xc - xW)) * idx2 +
               (N.yz(i, j, jp, k) * (xN - xc) - N.yz(i, jm, j, k) * (xc - xS)) * idy2 +
               (N.c(i, j, k) * (xT - xc) - N.c(i, j, k - 1) * (xc - xB)) * idz2;
    }
}

// The Crank-Nicolson right-hand side R = x + dt sum_m beta_m E^{n-m} +
// (dt/2) L x at face c: in FP64 as one expression; with FP32 stencils the
// increment is formed in FP32 and added to the FP64 state x64, so R keeps the
// state's precision and only the increment carries FP32 rounding.
template <typename T>
__device__ __forceinline__ void store_mom(const MomArgsT<T>& a, long long c, T xc, T E, T Ldiff, T dt, T b0, T b1,
                                          T b2, T hdt)
{
    a.en[c] = E;
    if constexpr (std::is_same<T, double>::value) {
        a.rhs[c] = xc + dt * (b0 * E + b1 * a.e1[c] + b2 * a.e2[c]) + hdt * Ldiff;
    } else {
        a.rhs[c] = a.x64[c] + (double)(dt * (b0 * E + b1 * a.e1[c] + b2 * a.e2[c]) + hdt * Ldiff);
    }
}

// Coefficients of the momentum kernels, rounded once to the stencil type.
template <typename T>
struct MomConst {
    T idx, idy, idz, idx2, idy2, idz2, dt, hdt, b0, b1, b2, dpdx, nu;
    __device__ MomConst(const Geo& g, const MomArgsT<T>& a)
        : idx((T)g.idx), idy((T)g.idy), idz((T)g.idz), idx2((T)g.idx2), idy2((T)g.idy2), idz2((T)g.idz2),
          dt((T)a.dt), hdt((T)a.half_dt), b0((T)a.beta0), b1((T)a.beta1), b2((T)a.beta2), dpdx((T)a.dpdx),
          nu((T)a.nu)
    {
    }
};

// x-momentum on x-faces: E_u = -d_j(u_j u) + d_j(nu_T d_x u_j) - G and
// R_u = u + dt sum_m beta_m E_u^{n-m} + (dt/2) d_j(nu_T d_j u).
template <typename T>
__global__ __launch_bounds__(256) void k_mom_u(Geo g, int kchunk, MomArgsT<T> a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int im = wm(i, g.nx), ip = wp(i, g.nx), jm = wm(j, g.ny), jp = wp(j, g.ny);
    const T* __restrict__ u = a.u;
    const T* __restrict__ v = a.v;
    const T* __restrict__ w = a.w;
    const MomConst<T> K(g, a);
    const URef R{a.ub, g.nz};  // FP32 only: u holds u - ub (see URef)
    const T h = T(0.5), q = T(0.25);
    auto C = [&](int ii, int jj, int kk) { return a.nut[at(g, ii, jj, kk)]; };
    const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
    // Carried along the march (the values of plane k + 1 become those of
    // plane k): u at the face's column on k - 1 and k, w under the face's
    // x-z edge, nu_T at the two centres of the face, and the x-z edge
    // viscosity below the face.
    T uc = u[at(g, i, j, k0)], uBraw = k0 > 0 ? u[at(g, i, j, k0 - 1)] : T(0);
    T wI = w[at(g, i, j, k0)], wIm = w[at(g, im, j, k0)];
    T nC = C(i, j, k0), nWc = C(im, j, k0);
    T nB = k0 > 0 ? q * (C(im, j, k0 - 1) + C(i, j, k0 - 1) + nWc + nC) : K.nu;
    for (int k = k0; k < k1; ++k) {
        const long long c = at(g, i, j, k);
        const bool up = k + 1 < g.nz;
        const T uTraw = up ? u[c + g.plane] : T(0);
        const T uE = u[at(g, ip, j, k)], uW = u[at(g, im, j, k)];
        const T uN = u[at(g, i, jp, k)], uS = u[at(g, i, jm, k)];
        const T uT = up ? uTraw : -uc;
        const T uB = k > 0 ? uBraw : -uc;
        // convection, divergence form
        const T ue = h * (uc + uE), uw = h * (uW + uc);
        const T vImjp = v[at(g, im, jp, k)], vIjp = v[at(g, i, jp, k)];
        const T vImj = v[at(g, im, j, k)], vIj = v[at(g, i, j, k)];
        const T vn = h * (vImjp + vIjp);
        const T vs = h * (vImj + vIj);
        const T wIm1 = w[at(g, im, j, k + 1)], wI1 = w[at(g, i, j, k + 1)];
        const T wt = h * (wIm1 + wI1);
        const T wb = h * (wIm + wI);
        T cx, cy, cz;
        if constexpr (kRefU<T>) {
            // u = ub + u': the profile is constant on the plane, so
            // ue^2 - uw^2 = (ue' - uw')(2 ub + ue' + uw') and the y flux
            // difference is ub (vn - vs) + its departure part
            const T ub = R.mean(k);
            cx = (ue - uw) * (T(2) * ub + ue + uw) * K.idx;
            cy = (ub * (vn - vs) + (vn * h * (uc + uN) - vs * h * (uS + uc))) * K.idy;
            cz = (wt * (R.edge(k) + h * (uc + uT)) - wb * (R.edge(k - 1) + h * (uB + uc))) * K.idz;
        } else {
            cx = (ue * ue - uw * uw) * K.idx;
            cy = (vn * h * (uc + uN) - vs * h * (uS + uc)) * K.idy;
            cz = (wt * h * (uc + uT) - wb * h * (uB + uc)) * K.idz;
        }
        // viscous terms
        const T nE = nC, nW = nWc;
        const T nN = q * (nWc + nC + C(im, jp, k) + C(i, jp, k));
        const T nS = q * (C(im, jm, k) + C(i, jm, k) + nWc + nC);
        const T nCn = up ? C(i, j, k + 1) : T(0), nWn = up ? C(im, j, k + 1) : T(0);
        const T nT = up ? q * (nWc + nC + nWn + nCn) : K.nu;
        const T dxx = (nE * (uE - uc) - nW * (uc - uW)) * K.idx2;
        const T vy = (nN * (vIjp - vImjp) - nS * (vIj - vImj)) * (K.idx * K.idy);
        const T vz = (nT * (wI1 - wIm1) - nB * (wI - wIm)) * (K.idx * K.idz);
        const T E = -(cx + cy + cz) + (dxx + vy + vz) - K.dpdx;
        T dut = uT - uc, dub = uc - uB;
        if constexpr (kRefU<T>) {
            dut += R.dz(k);
            dub += R.dz(k - 1);
        }
        const T Ldiff = dxx + (nN * (uN - uc) - nS * (uc - uS)) * K.idy2 + (nT * dut - nB * dub) * K.idz2;
        store_mom(a, c, uc, E, Ldiff, K.dt, K.b0, K.b1, K.b2, K.hdt);
        uBraw = uc;
        uc = uTraw;
        wI = wI1;
        wIm = wIm1;
        nC = nCn;
        nWc = nWn;
        nB = nT;
    }
}

// y-momentum on y-faces: E_v = -d_j(u_j v) + d_j(nu_T d_y u_j).
template <typename T>
__global__ __launch_bounds__(256) void k_mom_v(Geo g, int kchunk, MomArgsT<T> a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int im = wm(i, g.nx), ip = wp(i, g.nx), jm = wm(j, g.ny), jp = wp(j, g.ny);
    const T* __restrict__ u = a.u;
    const T* __restrict__ v = a.v;
    const T* __restrict__ w = a.w;
    const MomConst<T> K(g, a);
    const URef R{a.ub, g.nz};  // FP32 only: u holds u - ub (see URef)
    const T h = T(0.5), q = T(0.25);
    auto C = [&](int ii, int jj, int kk) { return a.nut[at(g, ii, jj, kk)]; };
    const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
    // carried as in k_mom_u, with x and y exchanged
    T vc = v[at(g, i, j, k0)], vBraw = k0 > 0 ? v[at(g, i, j, k0 - 1)] : T(0);
    T wJ = w[at(g, i, j, k0)], wJm = w[at(g, i, jm, k0)];
    T nC = C(i, j, k0), nSc = C(i, jm, k0);
    T nB = k0 > 0 ? q * (C(i, jm, k0 - 1) + C(i, j, k0 - 1) + nSc + nC) : K.nu;
    for (int k = k0; k < k1; ++k) {
        const long long c = at(g, i, j, k);
        const bool up = k + 1 < g.nz;
        const T vTraw = up ? v[c + g.plane] : T(0);
        const T vE = v[at(g, ip, j, k)], vW = v[at(g, im, j, k)];
        const T vN = v[at(g, i, jp, k)], vS = v[at(g, i, jm, k)];
        const T vT = up ? vTraw : -vc;
        const T vB = k > 0 ? vBraw : -vc;
        const T uIpjm = u[at(g, ip, jm, k)], uIpj = u[at(g, ip, j, k)];
        const T uIjm = u[at(g, i, jm, k)], uIj = u[at(g, i, j, k)];
        const T ue = h * (uIpjm + uIpj);
        const T uw = h * (uIjm + uIj);
        T cx;
        if constexpr (kRefU<T>) cx = (R.mean(k) * (h * (vE - vW)) + (ue * h * (vc + vE) - uw * h * (vW + vc))) * K.idx;
        else cx = (ue * h * (vc + vE) - uw * h * (vW + vc)) * K.idx;
        const T vn = h * (vc + vN), vs = h * (vS + vc);
        const T cy = (vn * vn - vs * vs) * K.idy;
        const T wJm1 = w[at(g, i, jm, k + 1)], wJ1 = w[at(g, i, j, k + 1)];
        const T wt = h * (wJm1 + wJ1);
        const T wb = h * (wJm + wJ);
        const T cz = (wt * h * (vc + vT) - wb * h * (vB + vc)) * K.idz;
        const T nE = q * (nSc + C(ip, jm, k) + nC + C(ip, j, k));
        const T nW = q * (C(im, jm, k) + nSc + C(im, j, k) + nC);
        const T nN = nC, nS = nSc;
        const T nCn = up ? C(i, j, k + 1) : T(0), nSn = up ? C(i, jm, k + 1) : T(0);
        const T nT = up ? q * (nSc + nC + nSn + nCn) : K.nu;
        const T vx = (nE * (uIpj - uIpjm) - nW * (uIj - uIjm)) * (K.idx * K.idy);
        const T dyy = (nN * (vN - vc) - nS * (vc - vS)) * K.idy2;
        const T vz = (nT * (wJ1 - wJm1) - nB * (wJ - wJm)) * (K.idy * K.idz);
        const T E = -(cx + cy + cz) + (vx + dyy + vz);
        const T Ldiff = (nE * (vE - vc) - nW * (vc - vW)) * K.idx2 + dyy + (nT * (vT - vc) - nB * (vc - vB)) * K.idz2;
        store_mom(a, c, vc, E, Ldiff, K.dt, K.b0, K.b1, K.b2, K.hdt);
        vBraw = vc;
        vc = vTraw;
        wJ = wJ1;
        wJm = wJm1;
        nC = nCn;
        nSc = nSn;
        nB = nT;
    }
}

// z-momentum on interior z-faces: E_w = -d_j(u_j w) + d_j(nu_T d_z u_j);
// wall planes get E = R = 0.
template <typename T>
__global__ __launch_bounds__(256) void k_mom_w(Geo g, int kchunk, MomArgsT<T> a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int im = wm(i, g.nx), ip = wp(i, g.nx), jm = wm(j, g.ny), jp = wp(j, g.ny);
    const T* __restrict__ u = a.u;
    const T* __restrict__ v = a.v;
    const T* __restrict__ w = a.w;
    const MomConst<T> K(g, a);
    const URef R{a.ub, g.nz};  // FP32 only: u holds u - ub (see URef)
    const T h = T(0.5), q = T(0.25);
    auto C = [&](int ii, int jj, int kk) { return a.nut[at(g, ii, jj, kk)]; };
    const int k0 = blockIdx.z * kchunk, k1 = min(g.nz + 1, k0 + kchunk);
    auto wall = [&](int k) {
        const long long c = at(g, i, j, k);
        a.en[c] = T(0);
        a.rhs[c] = 0.0;
    };
    int kb = k0;
    if (kb == 0) {
        wall(0);
        kb = 1;
    }
    const int ke = min(k1, g.nz);  // interior faces [kb, ke)
    if (kb < ke) {
        // Carried along the march: w at the column on k - 1 and k; u, v and
        // nu_T on the plane of centres below the face (k - 1).
        T wB = w[at(g, i, j, kb - 1)], wc = w[at(g, i, j, kb)];
        T uIp0 = u[at(g, ip, j, kb - 1)], uI0 = u[at(g, i, j, kb - 1)];
        T vJp0 = v[at(g, i, jp, kb - 1)], vJ0 = v[at(g, i, j, kb - 1)];
        T pC = C(i, j, kb - 1), pE = C(ip, j, kb - 1), pW = C(im, j, kb - 1), pN = C(i, jp, kb - 1),
          pS = C(i, jm, kb - 1);
        for (int k = kb; k < ke; ++k) {
            const long long c = at(g, i, j, k);
            const T wE = w[at(g, ip, j, k)], wW = w[at(g, im, j, k)];
            const T wN = w[at(g, i, jp, k)], wS = w[at(g, i, jm, k)];
            const T wT = w[c + g.plane];
            const T uIp1 = u[at(g, ip, j, k)], uI1 = u[at(g, i, j, k)];
            const T vJp1 = v[at(g, i, jp, k)], vJ1 = v[at(g, i, j, k)];
            const T ue = h * (uIp0 + uIp1);
            const T uw = h * (uI0 + uI1);
            T cx;
            if constexpr (kRefU<T>)
                cx = (R.edge(k - 1) * (h * (wE - wW)) + (ue * h * (wc + wE) - uw * h * (wW + wc))) * K.idx;
            else
                cx = (ue * h * (wc + wE) - uw * h * (wW + wc)) * K.idx;
            const T vn = h * (vJp0 + vJp1);
            const T vs = h * (vJ0 + vJ1);
            const T cy = (vn * h * (wc + wN) - vs * h * (wS + wc)) * K.idy;
            const T wt = h * (wc + wT), wb = h * (wB + wc);
            const T cz = (wt * wt - wb * wb) * K.idz;
            const T cC = C(i, j, k), cE = C(ip, j, k), cW = C(im, j, k), cN = C(i, jp, k), cS = C(i, jm, k);
            const T nE = q * (pC + pE + cC + cE), nW = q * (pW + pC + cW + cC);
            const T nN = q * (pC + pN + cC + cN), nS = q * (pS + pC + cS + cC);
            const T nT = cC, nB = pC;
            T duE = uIp1 - uIp0, duW = uI1 - uI0;
            if constexpr (kRefU<T>) {
                const T d = R.dz(k - 1);
                duE += d;
                duW += d;
            }
            const T vx = (nE * duE - nW * duW) * (K.idx * K.idz);
            const T vy = (nN * (vJp1 - vJp0) - nS * (vJ1 - vJ0)) * (K.idy * K.idz);
            const T dzz = (nT * (wT - wc) - nB * (wc - wB)) * K.idz2;
            const T E = -(cx + cy + cz) + (vx + vy + dzz);
            const T Ldiff = (nE * (wE - wc) - nW * (wc - wW)) * K.idx2 + (nN * (wN - wc) - nS * (wc - wS)) * K.idy2 + dzz;
            store_mom(a, c, wc, E, Ldiff, K.dt, K.b0, K.b1, K.b2, K.hdt);
            wB = wc;
            wc = wT;
            uIp0 = uIp1;
            uI0 = uI1;
            vJp0 = vJp1;
            vJ0 = vJ1;
            pC = cC;
            pE = cE;
            pW = cW;
            pN = cN;
            pS = cS;
        }
    }
    if (k1 == g.nz + 1) wall(g.nz);
}

// L_nu x = d_j(nu_T d_j x) for component COMP along the z march of the column
// (i, j) over planes [k0, k1), with visc_apply's expression and order of
// evaluation (so the results are identical) but the column's vertical
// neighbours and the nu_T values and edge averages shared with the next
// plane kept in registers: each plane loads x at k + 1 and its four lateral
// neighbours and the nu_T values of the new plane, not the whole stencil.
// Calls upd(k, c, L, x_c) for every face the column owns, wall(k) for w's
// wall planes.  TC: arithmetic, TN: nu_T storage, TX: x storage.
template <int COMP, typename TC, typename TN, typename TX, typename Upd, typename Wall>
__device__ __forceinline__ void visc_march(const Geo& g, int i, int j, int k0, int k1, const TN* __restrict__ nut,
                                           double nu, const TX* __restrict__ X, Upd&& upd, Wall&& wall)
{
    const int im = wm(i, g.nx), ip = wp(i, g.nx), jm = wm(j, g.ny), jp = wp(j, g.ny);
    const long long P = g.plane;
    const long long oc = at(g, i, j, 0), oE = at(g, ip, j, 0), oW = at(g, im, j, 0), oN = at(g, i, jp, 0),
                    oS = at(g, i, jm, 0);
    auto C = [&](long long o, int k) -> TC { return (TC)nut[o + P * k]; };
    auto V = [&](long long o, int k) -> TC { return (TC)X[o + P * k]; };
    const TC idx2 = (TC)g.idx2, idy2 = (TC)g.idy2, idz2 = (TC)g.idz2, nuT = (TC)nu, q = TC(0.25);

    if constexpr (COMP == 0 || COMP == 1) {
        // u: centre nu_T at (i, j) and (im, j), x-y edges to the north and
        // south, x-z edges above and below.  v: the same with x and y swapped.
        const long long oA = COMP == 0 ? oW : oS;  // the other centre of the face
        TC xc = V(oc, k0), xBraw = k0 > 0 ? V(oc, k0 - 1) : TC(0);
        TC cC = C(oc, k0), cA = C(oA, k0);
        TC elo = nuT;  // vertical edge below plane k0
        if (k0 > 0) elo = q * (C(oA, k0 - 1) + C(oc, k0 - 1) + cA + cC);
        for (int k = k0; k < k1; ++k) {
            const bool up = k + 1 < g.nz;
            const TC xTraw = up ? V(oc, k + 1) : TC(0);
            const TC cCn = up ? C(oc, k + 1) : TC(0), cAn = up ? C(oA, k + 1) : TC(0);
            const TC xT = up ? xTraw : -xc, xB = k > 0 ? xBraw : -xc;
            const TC xE = V(oE, k), xW = V(oW, k), xN = V(oN, k), xS = V(oS, k);
            const TC eup = up ? q * (cA + cC + cAn + cCn) : nuT;
            TC L;
            if constexpr (COMP == 0) {
                const TC en = q * (cA + cC + C(oW + (oN - oc), k) + C(oN, k));  // edge (im|i) x (j|jp)
                const TC es = q * (C(oW + (oS - oc), k) + C(oS, k) + cA + cC);  // edge (im|i) x (jm|j)
                L = (cC * (xE - xc) - cA * (xc - xW)) * idx2 + (en * (xN - xc) - es * (xc - xS)) * idy2 +
                    (eup * (xT - xc) - elo * (xc - xB)) * idz2;
            } else {
                const TC ee = q * (cA + C(oS + (oE - oc), k) + cC + C(oE, k));  // edge (i|ip) x (jm|j)
                const TC ew = q * (C(oS + (oW - oc), k) + cA + C(oW, k) + cC);  // edge (im|i) x (jm|j)
                L = (ee * (xE - xc) - ew * (xc - xW)) * idx2 + (cC * (xN - xc) - cA * (xc - xS)) * idy2 +
                    (eup * (xT - xc) - elo * (xc - xB)) * idz2;
            }
            upd(k, oc + P * k, L, xc);
            xBraw = xc;
            xc = xTraw;
            cC = cCn;
            cA = cAn;
            elo = eup;
        }
    } else {
        // w on z-faces: nu_T at the centres below (k - 1) and above (k), x-z
        // edges east and west, y-z edges north and south
        int kb = k0;
        if (kb == 0) {
            wall(oc);
            kb = 1;
        }
        const int ke = min(k1, g.nz);  // interior planes [kb, ke)
        if (kb < ke) {
            TC xB = V(oc, kb - 1), xc = V(oc, kb);
            TC pC = C(oc, kb - 1), pE = C(oE, kb - 1), pW = C(oW, kb - 1), pN = C(oN, kb - 1), pS = C(oS, kb - 1);
            for (int k = kb; k < ke; ++k) {
                const TC xT = V(oc, k + 1);
                const TC xE = V(oE, k), xW = V(oW, k), xN = V(oN, k), xS = V(oS, k);
                const TC cC = C(oc, k), cE = C(oE, k), cW = C(oW, k), cN = C(oN, k), cS = C(oS, k);
                const TC ee = q * (pC + pE + cC + cE), ew = q * (pW + pC + cW + cC);
                const TC en = q * (pC + pN + cC + cN), es = q * (pS + pC + cS + cC);
                const TC L = (ee * (xE - xc) - ew * (xc - xW)) * idx2 + (en * (xN - xc) - es * (xc - xS)) * idy2 +
                             (cC * (xT - xc) - pC * (xc - xB)) * idz2;
                upd(k, oc + P * k, L, xc);
                xB = xc;
                xc = xT;
                pC = cC;
                pE = cE;
                pW = cW;
                pN = cN;
                pS = cS;
            }
        }
        if (k1 == g.nz + 1) wall(oc + P * g.nz);
    }
}

// Crank-Nicolson solve in defect form for the mixed mode: u* = R + delta with
// (I - h L) delta = h L R, so that the iterate is the small viscous increment
// and FP32 resolves it; R and u* stay FP64.  From delta = 0, one step of the
// same iteration as k_cn per launch:
//   PHASE 0: d0 = h L R (FP64 arithmetic, FP32 nu_T), delta_1 = d0 / (1 + h s)
//   PHASE 1: delta_out = delta + (d0 - delta + h L delta) / (1 + h s)  (FP32)
//   PHASE 2: as PHASE 1, then u* = R + delta_out in FP64.
template <int COMP, int PHASE>
__global__ __launch_bounds__(256) void k_cn_defect(Geo g, int kchunk, const float* __restrict__ nut32, double nu,
                                                   const double* __restrict__ R, const float* __restrict__ d0in,
                                                   float* __restrict__ d0out, const float* __restrict__ x,
                                                   float* __restrict__ xo, double* __restrict__ uo, double h,
                                                   double inv_shift)
{
    // PHASE 0 applies the operator to R in FP64 arithmetic, the other phases
    // to the FP32 iterate in FP32
    using TC = std::conditional_t<PHASE == 0, double, float>;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const float h32 = (float)h, inv32 = (float)inv_shift;
    const int nplanes = COMP == 2 ? g.nz + 1 : g.nz;
    const int k0 = blockIdx.z * kchunk, k1 = min(nplanes, k0 + kchunk);
    auto upd = [&](int, long long c, TC L, TC xc) {
        if constexpr (PHASE == 0) {
            const float d = (float)(h * L);
            d0out[c] = d;
            xo[c] = d * inv32;
        } else {
            const float xn = xc + (d0in[c] - xc + h32 * L) * inv32;
            if constexpr (PHASE == 1) xo[c] = xn;
            else uo[c] = R[c] + (double)xn;
        }
    };
    auto wall = [&](long long c) {
        if constexpr (PHASE == 0) d0out[c] = 0.f;
        if constexpr (PHASE < 2) xo[c] = 0.f;
        else uo[c] = 0.0;
    };
    if constexpr (PHASE == 0) visc_march<COMP, double>(g, i, j, k0, k1, nut32, nu, R, upd, wall);
    else visc_march<COMP, float>(g, i, j, k0, k1, nut32, nu, x, upd, wall);
}

// One Crank-Nicolson iteration for component COMP:
// x_out = x + (R - x + h L_nu x) * inv_shift, L_nu = d_j(nu_T d_j .).
template <int COMP>
__global__ __launch_bounds__(256) void k_cn(Geo g, int kchunk, const double* __restrict__ nut, double nu,
                                            const double* __restrict__ R, const double* __restrict__ x,
                                            double* __restrict__ xo, double h, double inv_shift)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int nplanes = COMP == 2 ? g.nz + 1 : g.nz;
    const int k0 = blockIdx.z * kchunk, k1 = min(nplanes, k0 + kchunk);
    visc_march<COMP, double>(
        g, i, j, k0, k1, nut, nu, x,
        [&](int, long long c, double L, double xc) { xo[c] = xc + (R[c] - xc + h * L) * inv_shift; },
        [&](long long c) { xo[c] = 0.0; });
}

__global__ void k_round32(float* __restrict__ d, const double* __restrict__ s, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        d[q] = (float)s[q];
}

// ub[k] = mean of s over plane k (one workgroup per plane, fixed order)
__global__ __launch_bounds__(256) void k_plane_mean(const double* __restrict__ s, long long plane,
                                                    double* __restrict__ ub)
{
    __shared__ double lds[16];
    const double* __restrict__ p = s + plane * blockIdx.x;
    double acc = 0.0;
    for (long long q = threadIdx.x; q < plane; q += blockDim.x) acc += p[q];
    const double r = block_reduce<false>(acc, lds);
    if (threadIdx.x == 0) ub[blockIdx.x] = r / (double)plane;
}

// d = FP32(s - ub[k]) on plane k = blockIdx.y
__global__ void k_round32_sub(float* __restrict__ d, const double* __restrict__ s, const double* __restrict__ ub,
                              long long plane)
{
    const long long o = plane * blockIdx.y;
    const double m = ub[blockIdx.y];
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < plane; q += (long long)gridDim.x * blockDim.x)
        d[o + q] = (float)(s[o + q] - m);
}

// ---- divergence, Poisson right-hand side (Sec. 3.1) -------------------------

__global__ __launch_bounds__(256) void k_div(Geo g, int kchunk, const double* __restrict__ u,
                                             const double* __restrict__ v, const double* __restrict__ w,
                                             double* __restrict__ b, double inv_dt, double* __restrict__ part)
{
    __shared__ double lds[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double acc = 0.0;
    if (i < g.nx && j < g.ny) {
        const int ip = wp(i, g.nx), jp = wp(j, g.ny);
        const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
        for (int k = k0; k < k1; ++k) {
            const long long c = at(g, i, j, k);
            const double d = (u[at(g, ip, j, k)] - u[c]) * g.idx + (v[at(g, i, jp, k)] - v[c]) * g.idy +
                             (w[c + g.plane] - w[c]) * g.idz;
            const double val = d * inv_dt;
            b[c] = val;
            acc += val;
        }
    }
    const double r = block_reduce<false>(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = r;
}

// r = b - L_p p in FP64 with partial sums of r^2; optional FP32 copy of r.
__global__ __launch_bounds__(256) void k_residual(Geo g, int kchunk, const double* __restrict__ b,
                                                  const double* __restrict__ p, float* __restrict__ r32,
                                                  double r32_scale, double* __restrict__ part)
{
    __shared__ double lds[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double acc = 0.0;
    if (i < g.nx && j < g.ny) {
        const int im = wm(i, g.nx), ip = wp(i, g.nx), jm = wm(j, g.ny), jp = wp(j, g.ny);
        const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
        double pc = p[at(g, i, j, k0)];
        double pb = k0 > 0 ? p[at(g, i, j, k0 - 1)] : pc;
        for (int k = k0; k < k1; ++k) {
            const long long c = at(g, i, j, k);
            const double pt = k + 1 < g.nz ? p[c + g.plane] : pc;
            const double lap = (p[at(g, im, j, k)] + p[at(g, ip, j, k)] - 2.0 * pc) * g.idx2 +
                               (p[at(g, i, jm, k)] + p[at(g, i, jp, k)] - 2.0 * pc) * g.idy2 +
                               ((pt - pc) + (pb - pc)) * g.idz2;
            const double r = b[c] - lap;
            if (r32) r32[c] = (float)(r32_scale * r);
            acc += r * r;
            pb = pc;
            pc = pt;
        }
    }
    const double r = block_reduce<false>(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = r;
}

// ---- projection correction (Sec. 3.1) ---------------------------------------

__global__ __launch_bounds__(256) void k_project(Geo g, int kchunk, const double* __restrict__ p,
                                                 double* __restrict__ u, double* __restrict__ v,
                                                 double* __restrict__ w, double dt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int im = wm(i, g.nx), jm = wm(j, g.ny);
    const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
    for (int k = k0; k < k1; ++k) {
        const long long c = at(g, i, j, k);
        const double pc = p[c];
        u[c] -= dt * (pc - p[at(g, im, j, k)]) * g.idx;
        v[c] -= dt * (pc - p[at(g, i, jm, k)]) * g.idy;
        if (k > 0) w[c] -= dt * (pc - p[c - g.plane]) * g.idz;
    }
}

// ---- diagnostics: max|div u|, sum u, max|u|, CFL, centreline sum -------------

__global__ __launch_bounds__(256) void k_diag(Geo g, int kchunk, const double* __restrict__ u,
                                              const double* __restrict__ v, const double* __restrict__ w, double dt,
                                              double* __restrict__ part)
{
    __shared__ double lds[16];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double mdiv = 0.0, su = 0.0, mu = 0.0, cfl = 0.0, sc = 0.0;
    if (i < g.nx && j < g.ny) {
        const int ip = wp(i, g.nx), jp = wp(j, g.ny);
        const int k0 = blockIdx.z * kchunk, k1 = min(g.nz, k0 + kchunk);
        const int kc0 = g.nz % 2 == 0 ? g.nz / 2 - 1 : g.nz / 2;
        const int kc1 = g.nz / 2;
        for (int k = k0; k < k1; ++k) {
            const long long c = at(g, i, j, k);
            const double uc = u[c];
            const double d = (u[at(g, ip, j, k)] - uc) * g.idx + (v[at(g, i, jp, k)] - v[c]) * g.idy +
                             (w[c + g.plane] - w[c]) * g.idz;
            mdiv = fmax(mdiv, fabs(d));
            su += uc;
            mu = fmax(mu, fabs(uc));
            cfl = fmax(cfl, fmax(fabs(uc) * dt * g.idx, fabs(v[c]) * dt * g.idy));
            cfl = fmax(cfl, fabs(w[c]) * dt * g.idz);
            if (k == g.nz - 1) cfl = fmax(cfl, fabs(w[c + g.plane]) * dt * g.idz);
            if (k == kc0) sc += kc0 == kc1 ? uc : 0.5 * uc;
            else if (k == kc1) sc += 0.5 * uc;
        }
    }
    const int b = block_id(), nb = block_count();
    double r;
    r = block_reduce<true>(mdiv, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[0 * nb + b] = r;
    r = block_reduce<false>(su, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[1 * nb + b] = r;
    r = block_reduce<true>(mu, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[2 * nb + b] = r;
    r = block_reduce<true>(cfl, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[3 * nb + b] = r;
    r = block_reduce<false>(sc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[4 * nb + b] = r;
}

// ---- plane statistics (Sec. 6: averages over x and y at each height) -------

// One workgroup per height k = 0..nz; sums over the plane in a fixed order,
// written as plane means to out[q (nz+1) + k]:
//   q = 0 u, 1 v, 2 u^2, 3 v^2, 4 nu_T on the cell planes k < nz (0 at k = nz);
//   q = 5 w, 6 w^2 on the face planes k = 0..nz;
//   q = 7 u w on the x-z edges (i dx, k dz): u averaged over the planes k-1
//   and k (odd ghosts beyond the walls), w over the columns i-1 and i.
template <typename TN>
__global__ __launch_bounds__(256) void k_plane_stats(Geo g, const double* __restrict__ u, const double* __restrict__ v,
                                                     const double* __restrict__ w, const TN* __restrict__ nut,
                                                     double* __restrict__ out)
{
    __shared__ double lds[16];
    const int k = blockIdx.x;
    const long long pl = g.plane;
    double acc[kPlaneStats] = {};
    for (long long c = threadIdx.x; c < pl; c += blockDim.x) {
        const int i = (int)(c % g.nx);
        const long long cw = k * pl + c;  // face plane k
        const long long iw = cw - i + wm(i, g.nx);
        const double wc = w[cw];
        acc[5] += wc;
        acc[6] += wc * wc;
        if (k < g.nz) {
            const double uc = u[cw], vc = v[cw];
            acc[0] += uc;
            acc[1] += vc;
            acc[2] += uc * uc;
            acc[3] += vc * vc;
            acc[4] += (double)nut[cw];
        }
        const double ulo = k > 0 ? u[cw - pl] : -u[cw];
        const double uhi = k < g.nz ? u[cw] : -u[cw - pl];
        acc[7] += (0.5 * (ulo + uhi)) * (0.5 * (w[iw] + wc));
    }
    const double inv = 1.0 / (double)pl;
#pragma unroll
    for (int q = 0; q < kPlaneStats; ++q) {
        const double r = block_reduce<false>(acc[q], lds);
        if (threadIdx.x == 0) out[(long long)q * (g.nz + 1) + k] = r * inv;
    }
}

}  // namespace

// ============================================================================
// launchers

March march_shape(const Geo& g, int min_blocks)
{
    March m;
    int bx = 64;
    while (bx > 8 && bx / 2 >= g.nx) bx /= 2;
    const int by = 256 / bx;
    const int gx = (g.nx + bx - 1) / bx, gy = (g.ny + by - 1) / by;
    const long long cols = (long long)gx * gy;
    int gz = (int)std::min<long long>(g.nz, std::max<long long>(1, (min_blocks + cols - 1) / cols));
    // keep the partial-sum buffer large enough
    while ((long long)gz * cols > kMaxPartBlocks && gz > 1) --gz;
    m.kchunk = (g.nz + gz - 1) / gz;
    gz = (g.nz + m.kchunk - 1) / m.kchunk;
    m.grid = dim3(gx, gy, gz);
    m.block = dim3(bx, by, 1);
    return m;
}

hipError_t fill(double* a, double v, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill<double>, dim3(grid1d(n)), dim3(kBlock1d), 0, s, a, v, n);
    return hipGetLastError();
}
hipError_t fill(float* a, float v, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill<float>, dim3(grid1d(n)), dim3(kBlock1d), 0, s, a, v, n);
    return hipGetLastError();
}
hipError_t copy(double* dst, const double* src, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy, dim3(grid1d(n)), dim3(kBlock1d), 0, s, dst, src, n);
    return hipGetLastError();
}
hipError_t extrapolate(const double* p, const double* p1, const double* p2, int order, double* out, long long n,
                       hipStream_t s)
{
    if (order != 1 && order != 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_extrapolate, dim3(grid1d(n)), dim3(kBlock1d), 0, s, p, p1, p2, order, out, n);
    return hipGetLastError();
}
hipError_t copy(float* dst, const float* src, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy32, dim3(grid1d(n)), dim3(kBlock1d), 0, s, dst, src, n);
    return hipGetLastError();
}
hipError_t proj_gram(int k, const double* const* y, const double* b, long long n, double* part, double* res,
                     int slot, hipStream_t s)
{
    if (k < 1 || k > kMaxProj) return hipErrorInvalidValue;
    HistPtrs h{};
    for (int j = 0; j < k; ++j) h.a[j] = y[j];
    const int nb = grid1d(n, 1024);
    const int nq = k * (k + 1) / 2 + k;
    switch (k) {
    case 1: hipLaunchKernelGGL(k_proj_gram<1>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    case 2: hipLaunchKernelGGL(k_proj_gram<2>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    case 3: hipLaunchKernelGGL(k_proj_gram<3>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    case 4: hipLaunchKernelGGL(k_proj_gram<4>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    case 5: hipLaunchKernelGGL(k_proj_gram<5>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    case 6: hipLaunchKernelGGL(k_proj_gram<6>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    case 7: hipLaunchKernelGGL(k_proj_gram<7>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    default: hipLaunchKernelGGL(k_proj_gram<8>, dim3(nb), dim3(kBlock1d), 0, s, h, b, n, part); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalize_each, dim3(nq), dim3(256), 0, s, part, nb, res, slot);
    return hipGetLastError();
}
hipError_t proj_combine(int k, const double* const* x, const double* a, double* out, long long n, hipStream_t s)
{
    if (k < 1 || k > kMaxProj) return hipErrorInvalidValue;
    HistPtrs h{};
    ProjCoef c{};
    for (int j = 0; j < k; ++j) {
        h.a[j] = x[j];
        c.a[j] = a[j];
    }
    const dim3 grid(grid1d(n)), block(kBlock1d);
    switch (k) {
    case 1: hipLaunchKernelGGL(k_proj_combine<1>, grid, block, 0, s, h, c, out, n); break;
    case 2: hipLaunchKernelGGL(k_proj_combine<2>, grid, block, 0, s, h, c, out, n); break;
    case 3: hipLaunchKernelGGL(k_proj_combine<3>, grid, block, 0, s, h, c, out, n); break;
    case 4: hipLaunchKernelGGL(k_proj_combine<4>, grid, block, 0, s, h, c, out, n); break;
    case 5: hipLaunchKernelGGL(k_proj_combine<5>, grid, block, 0, s, h, c, out, n); break;
    case 6: hipLaunchKernelGGL(k_proj_combine<6>, grid, block, 0, s, h, c, out, n); break;
    case 7: hipLaunchKernelGGL(k_proj_combine<7>, grid, block, 0, s, h, c, out, n); break;
    default: hipLaunchKernelGGL(k_proj_combine<8>, grid, block, 0, s, h, c, out, n); break;
    }
    return hipGetLastError();
}
hipError_t sumsq_into(const double* a, long long n, double* part, double* res, int slot, hipStream_t s)
{
    const int nb = grid1d(n, 2048);
    hipLaunchKernelGGL(k_sumsq, dim3(nb), dim3(kBlock1d), 0, s, a, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(part, nb, 1, 0u, res, slot, s);
}
hipError_t zero_walls(const Geo& g, double* w, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_walls, dim3(grid1d(g.plane, 1024)), dim3(kBlock1d), 0, s, g, w);
    return hipGetLastError();
}

template <typename T>
hipError_t nut_smagorinsky(const Geo& g, const T* u, const T* v, const T* w, T* nut, double nu, double cs_delta,
                           double inv_wall_unit, double lz, const double* ub, double* part, double* res,
                           hipStream_t s)
{
    const March m = march_shape(g, 2048);
    hipLaunchKernelGGL(k_nut<T>, m.grid, m.block, 0, s, g, m.kchunk, u, v, w, nut, nu, cs_delta, inv_wall_unit, lz,
                       ub, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(part, m.nblocks(), 1, 1u, res, RES_NUT_MAX, s);
}
template hipError_t nut_smagorinsky<double>(const Geo&, const double*, const double*, const double*, double*, double,
                                            double, double, double, const double*, double*, double*, hipStream_t);
template hipError_t nut_smagorinsky<float>(const Geo&, const float*, const float*, const float*, float*, double,
                                           double, double, double, const double*, double*, double*, hipStream_t);

template <typename T>
hipError_t momentum_rhs(const Geo& g, int comp, const MomArgsT<T>& a, hipStream_t s)
{
    Geo gw = g;
    if (comp == 2) gw.nz = g.nz + 1;  // march over all nz+1 z-face planes
    const March m = march_shape(gw, 2048);
    if (comp == 0) hipLaunchKernelGGL(k_mom_u<T>, m.grid, m.block, 0, s, g, m.kchunk, a);
    else if (comp == 1) hipLaunchKernelGGL(k_mom_v<T>, m.grid, m.block, 0, s, g, m.kchunk, a);
    else hipLaunchKernelGGL(k_mom_w<T>, m.grid, m.block, 0, s, g, m.kchunk, a);
    return hipGetLastError();
}
template hipError_t momentum_rhs<double>(const Geo&, int, const MomArgsT<double>&, hipStream_t);
template hipError_t momentum_rhs<float>(const Geo&, int, const MomArgsT<float>&, hipStream_t);

hipError_t cn_iterate(const Geo& g, int comp, const double* nut, double nu, const double* rhs, const double* x,
                      double* xout, double half_dt, double inv_shift, hipStream_t s)
{
    Geo gw = g;
    if (comp == 2) gw.nz = g.nz + 1;
    const March m = march_shape(gw, 2048);
    if (comp == 0)
        hipLaunchKernelGGL(k_cn<0>, m.grid, m.block, 0, s, g, m.kchunk, nut, nu, rhs, x, xout, half_dt, inv_shift);
    else if (comp == 1)
        hipLaunchKernelGGL(k_cn<1>, m.grid, m.block, 0, s, g, m.kchunk, nut, nu, rhs, x, xout, half_dt, inv_shift);
    else
        hipLaunchKernelGGL(k_cn<2>, m.grid, m.block, 0, s, g, m.kchunk, nut, nu, rhs, x, xout, half_dt, inv_shift);
    return hipGetLastError();
}

hipError_t cn_defect(const Geo& g, int comp, int phase, const float* nut32, double nu, const double* rhs,
                     const float* d0in, float* d0out, const float* x, float* xo, double* uo, double half_dt,
                     double inv_shift, hipStream_t s)
{
    Geo gw = g;  // w has nz + 1 planes
    if (comp == 2) gw.nz = g.nz + 1;
    const March m = march_shape(gw, 2048);
#define STP_CND(C, P)                                                                                             \
    hipLaunchKernelGGL((k_cn_defect<C, P>), m.grid, m.block, 0, s, g, m.kchunk, nut32, nu, rhs, d0in, d0out, x, xo, \
                       uo, half_dt, inv_shift)
    if (comp < 0 || comp > 2 || phase < 0 || phase > 2) return hipErrorInvalidValue;
    if (comp == 0) { if (phase == 0) STP_CND(0, 0); else if (phase == 1) STP_CND(0, 1); else STP_CND(0, 2); }
    if (comp == 1) { if (phase == 0) STP_CND(1, 0); else if (phase == 1) STP_CND(1, 1); else STP_CND(1, 2); }
    if (comp == 2) { if (phase == 0) STP_CND(2, 0); else if (phase == 1) STP_CND(2, 1); else STP_CND(2, 2); }
#undef STP_CND
    return hipGetLastError();
}

hipError_t round_to_f32(float* dst, const double* src, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_round32, dim3(grid1d(n)), dim3(kBlock1d), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t round_departure_f32(const Geo& g, float* dst, const double* src, double* ub, hipStream_t s)
{
    hipLaunchKernelGGL(k_plane_mean, dim3(g.nz), dim3(256), 0, s, src, g.plane, ub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bx = (int)std::max<long long>(1, std::min<long long>((g.plane + kBlock1d - 1) / kBlock1d, 64));
    hipLaunchKernelGGL(k_round32_sub, dim3(bx, g.nz), dim3(kBlock1d), 0, s, dst, src, ub, g.plane);
    return hipGetLastError();
}

hipError_t divergence_rhs(const Geo& g, const double* u, const double* v, const double* w, double* b, double inv_dt,
                          double* part, double* res, hipStream_t s)
{
    const March m = march_shape(g, 2048);
    hipLaunchKernelGGL(k_div, m.grid, m.block, 0, s, g, m.kchunk, u, v, w, b, inv_dt, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(part, m.nblocks(), 1, 0u, res, RES_SUM_B, s);
}

hipError_t remove_mean(double* a, long long n, const double* res_sum, int res_out_sq, double* part, double* res,
                       hipStream_t s)
{
    const int nb = grid1d(n, 2048);
    hipLaunchKernelGGL(k_remove_mean, dim3(nb), dim3(kBlock1d), 0, s, a, n, res_sum, part, res_out_sq >= 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || res_out_sq < 0) return e;
    return finalize(part, nb, 1, 0u, res, res_out_sq, s);
}

hipError_t sum_into(const double* a, long long n, double* part, double* res, int slot, hipStream_t s)
{
    const int nb = grid1d(n, 2048);
    hipLaunchKernelGGL(k_sum, dim3(nb), dim3(kBlock1d), 0, s, a, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(part, nb, 1, 0u, res, slot, s);
}

hipError_t residual(const Geo& g, const double* b, const double* p, float* r32, double* part, double* res,
                    hipStream_t s, double r32_scale)
{
    const March m = march_shape(g, 2048);
    hipLaunchKernelGGL(k_residual, m.grid, m.block, 0, s, g, m.kchunk, b, p, r32, r32_scale, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(part, m.nblocks(), 1, 0u, res, RES_R2, s);
}

__global__ void k_sqrt_into(const double* __restrict__ x, double* __restrict__ out) { out[0] = sqrt(x[0]); }

hipError_t residual_norm_into(const Geo& g, const double* b, const double* p, double* part, double* norm,
                              hipStream_t s)
{
    const March m = march_shape(g, 2048);
    const int nb = m.nblocks();
    hipLaunchKernelGGL(k_residual, m.grid, m.block, 0, s, g, m.kchunk, b, p, (float*)nullptr, 1.0, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = finalize(part, nb, 1, 0u, part + nb, 0, s);  // sum r^2 into part[nb]
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sqrt_into, dim3(1), dim3(1), 0, s, part + nb, norm);
    return hipGetLastError();
}

hipError_t add_correction(double* p, const float* e, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_correction, dim3(grid1d(n)), dim3(kBlock1d), 0, s, p, e, n);
    return hipGetLastError();
}
hipError_t add_correction_scaled(double* p, const float* e, long long n, double inv_scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_correction_scaled, dim3(grid1d(n)), dim3(kBlock1d), 0, s, p, e, n, inv_scale);
    return hipGetLastError();
}
hipError_t half_scaled(_Float16* dst, const float* r, long long n, float scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_half_scaled, dim3(grid1d(n)), dim3(kBlock1d), 0, s, dst, r, n, scale);
    return hipGetLastError();
}

hipError_t project(const Geo& g, const double* p, double* u, double* v, double* w, double dt, hipStream_t s)
{
    const March m = march_shape(g, 2048);
    hipLaunchKernelGGL(k_project, m.grid, m.block, 0, s, g, m.kchunk, p, u, v, w, dt);
    return hipGetLastError();
}

template <typename TN>
hipError_t plane_stats(const Geo& g, const double* u, const double* v, const double* w, const TN* nut, double* out,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_plane_stats<TN>, dim3(g.nz + 1), dim3(256), 0, s, g, u, v, w, nut, out);
    return hipGetLastError();
}
template hipError_t plane_stats<double>(const Geo&, const double*, const double*, const double*, const double*,
                                        double*, hipStream_t);
template hipError_t plane_stats<float>(const Geo&, const double*, const double*, const double*, const float*,
                                       double*, hipStream_t);

hipError_t diagnostics(const Geo& g, const double* u, const double* v, const double* w, double dt, double* part,
                       double* res, hipStream_t s)
{
    const March m = march_shape(g, 2048);
    hipLaunchKernelGGL(k_diag, m.grid, m.block, 0, s, g, m.kchunk, u, v, w, dt, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return finalize(part, m.nblocks(), 5, 0b01101u, res, RES_DIAG, s);
}

}  // namespace stp
