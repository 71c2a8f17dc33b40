// Temporally blocked Jacobi-SOR sweeps for gfx950 (Sec. 3.4: the SRJ cycle
// is a sequence of weighted Jacobi sweeps p <- p + (omega_s/D)(L_p p - b)).
//
// The sweep is HBM-bound (about one flop per byte), so NT consecutive sweeps
// of the cycle are fused into one launch: every workgroup owns a 64 x 32
// column tile of the x-y plane (periodic wrap computed in-kernel) and marches
// along z.  At each z step it loads one plane of p and b, then advances every
// stage s = 1..NT of the pipeline by one plane: stage s produces plane t - s
// from stage s-1's planes t-s-1, t-s, t-s+1.  The vertical neighbours live in
// per-thread register rings, the x-y neighbours in one LDS plane per stage.
// Stage s is exact on points at least s away from the tile edge, so a tile
// writes its central (64 - 2NT) x (32 - 2NT) columns; a z-chunk is extended
// by NT planes on each side (clipped at the walls, where the zero-gradient
// ghost equals the centre value).  Each point evaluates exactly the unblocked
// formula in the same order, so NT fused sweeps equal NT single sweeps bit
// for bit.
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

template <typename T, int NT, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_relax_fused(int nx, int ny, int nz, int zchunk,
                                                            const T* __restrict__ b, const T* __restrict__ p,
                                                            T* __restrict__ out, Weights wts, T idx2, T idy2,
                                                            T idz2)
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

    // global offsets of this thread's columns (periodic wrap)
    const int gx = ((x0 + lane) % nx + nx) % nx;
    int col[PTS];  // offset within a plane (nx*ny < 2^31)
    int row[PTS];
#pragma unroll
    for (int m = 0; m < PTS; ++m) {
        row[m] = wave + WAVES * m;
        const int gy = ((y0 + row[m]) % ny + ny) % ny;
        col[m] = gy * nx + gx;
    }
    const int xm = max(lane - 1, 0), xp = min(lane + 1, kTileX - 1);
    const bool out_x = lane >= NT && lane < kTileX - NT && x0 + lane < nx;

    T c[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) c[s] = (T)wts.c[s];

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

    const int t_begin = max(0, z0 - NT);
    const int t_end = z1 - 1 + NT;  // the final stage reaches plane z1 - 1
    for (int t = t_begin; t <= t_end; ++t) {
        // stage 0: load plane t of p and b
        const T* __restrict__ pt_plane = p + plane * t;
        const T* __restrict__ bt_plane = b + plane * t;
#pragma unroll
        for (int m = 0; m < PTS; ++m) {
            R[0][2][m] = R[0][1][m];
            R[0][1][m] = R[0][0][m];
#pragma unroll
            for (int s = NT; s > 0; --s) B[s][m] = B[s - 1][m];
            if (t < nz) {
                R[0][0][m] = pt_plane[col[m]];
                B[0][m] = bt_plane[col[m]];
            }
        }
        // stages 1..NT: stage s produces plane q = t - s
#pragma unroll
        for (int s = 1; s <= NT; ++s) {
            const int q = t - s;
            T res[PTS];
#pragma unroll
            for (int m = 0; m < PTS; ++m) {
                const T pc = R[s - 1][1][m];
                const T pt = q + 1 < nz ? R[s - 1][0][m] : pc;
                const T pb = q > 0 ? R[s - 1][2][m] : pc;
                const int r = row[m];
                const int ym = max(r - 1, 0), yp = min(r + 1, kTileY - 1);
                const T lap = (lds[s - 1][r][xm] + lds[s - 1][r][xp] - T(2) * pc) * idx2 +
                              (lds[s - 1][ym][lane] + lds[s - 1][yp][lane] - T(2) * pc) * idy2 +
                              ((pt - pc) + (pb - pc)) * idz2;
                res[m] = pc + c[s - 1] * (lap - B[s][m]);
            }
            if (s < NT) {
#pragma unroll
                for (int m = 0; m < PTS; ++m) {
                    R[s][2][m] = R[s][1][m];
                    R[s][1][m] = R[s][0][m];
                    R[s][0][m] = res[m];
                }
            } else if (q >= z0 && q < z1 && out_x) {
                T* __restrict__ oq = out + plane * q;
#pragma unroll
                for (int m = 0; m < PTS; ++m) {
                    const int r = row[m];
                    if (r >= NT && r < kTileY - NT && y0 + r < ny) oq[col[m]] = res[m];
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
                       zchunk, b, p, out, wts, (T)g.idx2, (T)g.idy2, (T)g.idz2);
    return hipGetLastError();
}

// One sweep per launch, one thread per (i, j) column marching along z with the
// vertical neighbours in registers; used for grids narrower than a tile.
template <typename T>
__global__ __launch_bounds__(256) void k_relax(int nx, int ny, int nz, int kchunk, const T* __restrict__ b,
                                               const T* __restrict__ p, T* __restrict__ out, T c, T idx2, T idy2,
                                               T idz2)
{
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
        const T lap = (p[o + row + im] + p[o + row + ip] - T(2) * pc) * idx2 +
                      (p[o + rowm + i] + p[o + rowp + i] - T(2) * pc) * idy2 + ((pt - pc) + (pb - pc)) * idz2;
        out[o + row + i] = pc + c * (lap - b[o + row + i]);
        pb = pc;
        pc = pt;
    }
}

}  // namespace

bool relax_fusable(const Geo& g) { return g.nx >= kTileX && g.ny >= kTileY; }

template <typename T>
hipError_t relax(const Geo& g, const T* b, const T* p, T* out, const Weights& wts, int nfused, hipStream_t s)
{
    if (nfused == 1 || !relax_fusable(g)) {
        if (nfused != 1) return hipErrorInvalidValue;
        const March m = march_shape(g, 2048);
        hipLaunchKernelGGL(k_relax<T>, m.grid, m.block, 0, s, g.nx, g.ny, g.nz, m.kchunk, b, p, out, (T)wts.c[0],
                           (T)g.idx2, (T)g.idy2, (T)g.idz2);
        return hipGetLastError();
    }
    if (nfused == 2) return launch_fused<T, 2, STP_RELAX_WAVES>(g, b, p, out, wts, s);
    if (nfused == 4) return launch_fused<T, 4, STP_RELAX_WAVES>(g, b, p, out, wts, s);
    return hipErrorInvalidValue;
}
template hipError_t relax<double>(const Geo&, const double*, const double*, double*, const Weights&, int, hipStream_t);
template hipError_t relax<float>(const Geo&, const float*, const float*, float*, const Weights&, int, hipStream_t);

}  // namespace stp
