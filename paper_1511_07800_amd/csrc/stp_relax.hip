// Temporally blocked Jacobi-SOR sweeps for gfx950 (Sec. 3.4: the SRJ cycle
// is a sequence of weighted Jacobi sweeps p <- p + (omega_s/D)(L_p p - b)).
//
// NT consecutive sweeps of the cycle are fused into one launch: every
// workgroup owns a 64 x 32 column tile of the x-y plane (periodic wrap
// computed in-kernel) and marches along z.  At each z step it loads one plane
// of p and b, then advances every stage s = 1..NT of the pipeline by one
// plane: stage s produces plane t - s from stage s-1's planes t-s-1, t-s,
// t-s+1.  The vertical neighbours live in per-thread register rings, the x-y
// neighbours in one LDS plane per stage.  Stage s is exact on points at least
// s away from the tile edge, so a tile writes its central (64 - 2NT) x
// (32 - 2NT) columns; a z-chunk is extended by NT planes on each side
// (clipped at the walls).  Each point evaluates exactly the unblocked formula
// (sweep_point) in the same order, so NT fused sweeps equal NT single sweeps
// bit for bit.
//
// With HBM traffic cut by NT, the kernel is bound by vector-ALU issue and by
// load latency along the march, which shape the code: the point update is
// eight instructions, a stage skips (per wavefront) the rows and planes that
// no later stage reads, the wall ghosts are stored in the rings instead of
// selected per point, loads are addressed as a 32-bit lane offset on a
// uniform plane base, and the next plane is requested one step ahead.
#include "stp_internal.h"

#include <algorithm>

namespace stp {

namespace {

constexpr int kTileX = 64;  // one wavefront across x
constexpr int kTileY = 32;
static int kMinChunk = 48;       // planes per z-chunk, at least (measured best at 512x256x192)
static int kTargetBlocks = 2048;  // workgroups to aim for
#ifndef STP_RELAX_WAVES
#define STP_RELAX_WAVES 8      // wavefronts per workgroup; kTileY / waves rows per thread
#endif
#ifndef STP_RELAX_PF
#define STP_RELAX_PF 1         // planes of p and b requested ahead of the one processed
#endif
constexpr int PF = STP_RELAX_PF;

// Coefficients of one weighted Jacobi sweep, from omega and D = 2/dx^2 +
// 2/dy^2 + 2/dz^2:  p + (omega/D)(L_p p - b)
//   = (1 - omega) p + kx (pw + pe) + ky (ps + pn) + kz (pt + pb) - kb b,
// kx = omega/(D dx^2), ky = omega/(D dy^2), kz = omega/(D dz^2), kb = omega/D:
// the relaxation (1 - omega) p + omega J(p) of the plain Jacobi update J.
struct StageCoefs {
    double k0[kMaxFused], kx[kMaxFused], ky[kMaxFused], kz[kMaxFused], kb[kMaxFused];
};

StageCoefs stage_coefs(const Geo& g, const Weights& w, int n)
{
    const double D = 2.0 * (g.idx2 + g.idy2 + g.idz2);
    StageCoefs k{};
    for (int s = 0; s < n; ++s) {
        const double kb = w.omega[s] / D;
        k.k0[s] = 1.0 - w.omega[s];
        k.kx[s] = kb * g.idx2;
        k.ky[s] = kb * g.idy2;
        k.kz[s] = kb * g.idz2;
        k.kb[s] = kb;
    }
    return k;
}

template <typename T>
struct Coef {
    T k0, kx, ky, kz, kb;
};

template <typename T>
__device__ __forceinline__ T fma_(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One weighted Jacobi update of a cell from its six neighbours (zero-gradient
// ghosts already substituted), with explicit fused multiply-adds in a fixed
// order so the single-sweep and the fused kernels round identically: three
// adds, one multiply, four fused multiply-adds.
template <typename T>
__device__ __forceinline__ T sweep_point(const Coef<T>& k, T pw, T pe, T ps, T pn, T pt, T pb, T pc, T bb)
{
    T acc = fma_(-k.kb, bb, k.k0 * pc);
    acc = fma_(k.kx, pw + pe, acc);
    acc = fma_(k.ky, ps + pn, acc);
    return fma_(k.kz, pt + pb, acc);
}

// Buffer-resource access: a uniform plane base in scalar registers, a 32-bit
// per-lane byte offset, and the plane size as the range (out-of-range loads
// return zero, stores are dropped).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

template <typename T, int NT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_relax_fused(int nx, int ny, int nz, int zchunk,
                                                            const T* __restrict__ b, const T* __restrict__ p,
                                                            T* __restrict__ out, StageCoefs kc)
{
    constexpr int PTS = kTileY / WAVES;  // rows per thread
    constexpr int OX = kTileX - 2 * NT, OY = kTileY - 2 * NT;
    __shared__ T lds[NT][kTileY][kTileX];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int x0 = blockIdx.x * OX - NT;  // tile origin (may be negative: wrapped)
    const int y0 = blockIdx.y * OY - NT;
    const int z0 = blockIdx.z * zchunk, z1 = min(nz, z0 + zchunk);
    const long long plane = (long long)nx * ny;
    const unsigned pbytes = (unsigned)(plane * (long long)sizeof(T));

    // global offsets of this thread's columns (periodic wrap)
    const int gx = ((x0 + lane) % nx + nx) % nx;
    // byte offset of this thread's column within a plane: a 32-bit vector
    // offset on a uniform plane address (planes below 4 GiB)
    unsigned col[PTS];
    int row[PTS];
#pragma unroll
    for (int m = 0; m < PTS; ++m) {
        row[m] = wave + WAVES * m;
        const int gy = ((y0 + row[m]) % ny + ny) % ny;
        col[m] = (unsigned)(gy * nx + gx) * (unsigned)sizeof(T);
    }
    const int xm = max(lane - 1, 0), xp = min(lane + 1, kTileX - 1);
    const bool out_x = lane >= NT && lane < kTileX - NT && x0 + lane < nx;

    Coef<T> c[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) c[s] = Coef<T>{(T)kc.k0[s], (T)kc.kx[s], (T)kc.ky[s], (T)kc.kz[s], (T)kc.kb[s]};

    // rings: R[s][0] newest plane of stage s, R[s][1] the one before, R[s][2] before that
    T R[NT][3][PTS];
    T B[NT + 1][PTS];
#pragma unroll
    for (int s = 0; s < NT; ++s)
#pragma unroll
        for (int m = 0; m < PTS; ++m) R[s][0][m] = R[s][1][m] = R[s][2][m] = T(0);
#pragma unroll
    for (int s = 0; s <= NT; ++s)
#pragma unroll
        for (int m = 0; m < PTS; ++m) B[s][m] = T(0);

    // Plane t + PF is requested while plane t is processed, into a register
    // slot chosen statically (the loop is unrolled by PF), so PF planes of
    // loads stay in flight across the barriers instead of one load latency
    // being exposed per z step.  Planes past the top wall are clamped to
    // nz - 1, which is the zero-gradient ghost plane of stage 0.
    T Pq[PF][PTS], Bq[PF][PTS];
    const int t_begin = max(0, z0 - NT);
    const int t_end = z1 - 1 + NT;  // the final stage reaches plane z1 - 1
#pragma unroll
    for (int d = 0; d < PF; ++d) {
        const long long o = plane * min(t_begin + d, nz - 1);
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(p + o, pbytes), rb = plane_rsrc(b + o, pbytes);
#pragma unroll
        for (int m = 0; m < PTS; ++m) {
            Pq[d][m] = buf_load<T>(rp, col[m]);
            Bq[d][m] = buf_load<T>(rb, col[m]);
        }
    }
    for (int tb = t_begin; tb <= t_end; tb += PF) {
#pragma unroll
        for (int d = 0; d < PF; ++d) {
            const int t = tb + d;
            if (t > t_end) break;
            // stage 0: plane t from its slot, which then requests plane t + PF
            const long long o = plane * min(t + PF, nz - 1);
            const __amdgpu_buffer_rsrc_t rp = plane_rsrc(p + o, pbytes), rb = plane_rsrc(b + o, pbytes);
#pragma unroll
            for (int m = 0; m < PTS; ++m) {
                R[0][2][m] = R[0][1][m];
                R[0][1][m] = R[0][0][m];
                R[0][0][m] = Pq[d][m];
#pragma unroll
                for (int s = NT; s > 0; --s) B[s][m] = B[s - 1][m];
                B[0][m] = Bq[d][m];
                Pq[d][m] = buf_load<T>(rp, col[m]);
                Bq[d][m] = buf_load<T>(rb, col[m]);
            }
            // Zero-gradient walls: every ring holds, in place of plane -1 and
            // plane nz, a copy of plane 0 and plane nz - 1 of its stage, so
            // the point update needs no select.  Stage 0 gets plane nz - 1
            // again from the clamped loads, plane -1 here.
            if (t == 0) {
#pragma unroll
                for (int m = 0; m < PTS; ++m) R[0][1][m] = R[0][0][m];
            }
            // stages 1..NT: stage s produces plane q = t - s.  Stage s is
            // needed only on rows [s, 32 - s) and planes [z0 - (NT - s),
            // z1 + (NT - s)) inside the walls; both tests are uniform per
            // wavefront, so skipped rows and planes cost no issue slots.
#pragma unroll
            for (int s = 1; s <= NT; ++s) {
                const int q = t - s;
                T res[PTS];
                if (q >= max(0, z0 - (NT - s)) && q <= min(nz - 1, z1 - 1 + (NT - s))) {
#pragma unroll
                    for (int m = 0; m < PTS; ++m) {
                        const int r = row[m];
                        res[m] = R[s - 1][1][m];
                        if (r < s || r >= kTileY - s) continue;
                        res[m] = sweep_point<T>(c[s - 1], lds[s - 1][r][xm], lds[s - 1][r][xp],
                                                lds[s - 1][r - 1][lane], lds[s - 1][r + 1][lane], R[s - 1][0][m],
                                                R[s - 1][2][m], R[s - 1][1][m], B[s][m]);
                    }
                } else if (s < NT) {
                    // not needed; past the top wall this is the ghost plane nz
#pragma unroll
                    for (int m = 0; m < PTS; ++m) res[m] = R[s][0][m];
                }
                if (s < NT) {
#pragma unroll
                    for (int m = 0; m < PTS; ++m) {
                        R[s][2][m] = R[s][1][m];
                        R[s][1][m] = R[s][0][m];
                        R[s][0][m] = res[m];
                    }
                    if (q == 0) {
#pragma unroll
                        for (int m = 0; m < PTS; ++m) R[s][1][m] = res[m];  // ghost plane -1
                    }
                } else if (q >= z0 && q < z1 && out_x) {
                    const __amdgpu_buffer_rsrc_t ro = plane_rsrc(out + plane * q, pbytes);
#pragma unroll
                    for (int m = 0; m < PTS; ++m) {
                        const int r = row[m];
                        if (r >= NT && r < kTileY - NT && y0 + r < ny) buf_store(res[m], ro, col[m]);
                    }
                }
            }
            __syncthreads();  // every read of this iteration's LDS planes is done
#pragma unroll
            for (int s = 0; s < NT; ++s)
#pragma unroll
                for (int m = 0; m < PTS; ++m) lds[s][row[m]][lane] = R[s][0][m];
            __syncthreads();
        }
    }
}

template <typename T, int NT, int WAVES>
hipError_t launch_fused(const Geo& g, const T* b, const T* p, T* out, const Weights& wts, hipStream_t s)
{
    constexpr int OX = kTileX - 2 * NT, OY = kTileY - 2 * NT;
    const int tx = (g.nx + OX - 1) / OX, ty = (g.ny + OY - 1) / OY;
    // enough workgroups to fill the 256 CUs, z-chunks of at least
    // kMinChunk planes (each chunk recomputes NT planes at both ends)
    const long long tiles = (long long)tx * ty;
    int nzc = (int)std::max<long long>(
        1, std::min<long long>(g.nz / kMinChunk, (kTargetBlocks + tiles - 1) / tiles));
    const int zchunk = (g.nz + nzc - 1) / nzc;
    nzc = (g.nz + zchunk - 1) / zchunk;
    hipLaunchKernelGGL((k_relax_fused<T, NT, WAVES>), dim3(tx, ty, nzc), dim3(64 * WAVES), 0, s, g.nx, g.ny, g.nz,
                       zchunk, b, p, out, stage_coefs(g, wts, NT));
    return hipGetLastError();
}

// One sweep per launch, one thread per (i, j) column marching along z with the
// vertical neighbours in registers; used for grids narrower than a tile.
template <typename T>
__global__ __launch_bounds__(256) void k_relax(int nx, int ny, int nz, int kchunk, const T* __restrict__ b,
                                               const T* __restrict__ p, T* __restrict__ out, StageCoefs kc)
{
    const Coef<T> c{(T)kc.k0[0], (T)kc.kx[0], (T)kc.ky[0], (T)kc.kz[0], (T)kc.kb[0]};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const long long plane = (long long)nx * ny;
    const int im = i == 0 ? nx - 1 : i - 1, ip = i == nx - 1 ? 0 : i + 1;
    const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
    const long long row = (long long)nx * j, rowm = (long long)nx * jm, rowp = (long long)nx * jp;
    const int k0 = blockIdx.z * kchunk, k1 = min(nz, k0 + kchunk);
    long long o = plane * k0;
    T pc = p[o + row + i];
    T pb = k0 > 0 ? p[o - plane + row + i] : pc;
    for (int k = k0; k < k1; ++k, o += plane) {
        const T pt = k + 1 < nz ? p[o + plane + row + i] : pc;
        out[o + row + i] =
            sweep_point<T>(c, p[o + row + im], p[o + row + ip], p[o + rowm + i], p[o + rowp + i], pt, pb, pc, b[o + row + i]);
        pb = pc;
        pc = pt;
    }
}

}  // namespace

bool relax_fusable(const Geo& g)
{
    return g.nx >= kTileX && g.ny >= kTileY && (long long)g.nx * g.ny < (1LL << 29);
}

template <typename T>
hipError_t relax(const Geo& g, const T* b, const T* p, T* out, const Weights& wts, int nfused, hipStream_t s)
{
    if (nfused == 1 || !relax_fusable(g)) {
        if (nfused != 1) return hipErrorInvalidValue;
        const March m = march_shape(g, 2048);
        hipLaunchKernelGGL(k_relax<T>, m.grid, m.block, 0, s, g.nx, g.ny, g.nz, m.kchunk, b, p, out,
                           stage_coefs(g, wts, 1));
        return hipGetLastError();
    }
    if (nfused == 2) return launch_fused<T, 2, STP_RELAX_WAVES>(g, b, p, out, wts, s);
    if (nfused == 4) return launch_fused<T, 4, STP_RELAX_WAVES>(g, b, p, out, wts, s);
    return hipErrorInvalidValue;
}
template hipError_t relax<double>(const Geo&, const double*, const double*, double*, const Weights&, int, hipStream_t);
template hipError_t relax<float>(const Geo&, const float*, const float*, float*, const Weights&, int, hipStream_t);

}  // namespace stp
