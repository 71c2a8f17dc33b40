// Temporally blocked Jacobi-SOR sweeps for gfx950 (Sec. 3.4: the SRJ cycle
// is a sequence of weighted Jacobi sweeps p <- p + (omega_s/D)(L_p p - b)).
//
// NT consecutive sweeps of the cycle are fused into one launch.  A workgroup
// owns a 64 x 34 column tile of the x-y plane (periodic wrap computed
// in-kernel; rows 1..32 are updated, rows 0 and 33 are only loaded) and
// marches along z.  At each z step it takes in one plane of p and b, then
// advances every stage s = 1..NT of the pipeline by one plane: stage s
// produces plane t - s from stage s-1's planes t-s-1, t-s, t-s+1.  A
// wavefront owns 32/waves contiguous rows: z neighbours live in per-thread
// register rings, x neighbours in the next lanes' registers (DPP wave
// shifts), y neighbours in the thread's own adjacent rows, except across
// wavefronts, where the boundary rows go through LDS planes (double-buffered:
// one barrier per z step).  Stage s is exact on points at
// least s away from the tile edge, so a tile writes its central
// (64 - 2NT) x (34 - 2NT) columns; a z-chunk is extended by NT planes on each
// side (clipped at the walls).  Each point evaluates exactly the unblocked
// formula (sweep_point) in the same order, so NT fused sweeps equal NT single
// sweeps bit for bit.
//
// With HBM traffic cut by NT, the kernel is bound by vector-ALU issue and by
// latency along the march, which shape the code: the point update is eight
// instructions with the walls folded into per-plane coefficients (no ghost
// values, no per-point selects); the march is unrolled so that ring slots are
// static registers; the next plane is requested one step ahead; loads and
// stores are a 32-bit lane offset on a uniform plane base; coefficients
// arrive rounded to the element type so they stay in scalar registers; every
// stage updates all 32 rows (straight-line code; rows a later stage does not
// read are discarded); the tile order is XCD-aware (see k_relax_fused).
#include "stp_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace stp {

namespace {

constexpr int kTileX = 64;  // one wavefront across x
constexpr int kTileY = 32;  // rows updated by a workgroup; two more halo rows are only loaded
constexpr int kMinChunk = 8;  // planes per z-chunk, at least
constexpr int kXcds = 8;          // accelerator complex dies of an MI355X, each with its own L2
// wavefronts per workgroup (kTileY / waves rows per thread): measured best
// 8 for FP32 (two workgroups per CU under the 128-VGPR cap) and 16 for FP64
template <typename T>
constexpr int kWaves = sizeof(T) == 4 ? 8 : 16;
// Five FP32 sweeps per launch run on taller tiles: 16 wavefronts of 4 rows
// (64 updated rows, one workgroup per CU), whose halo is a smaller share of
// the tile than with 8 wavefronts (64x66 loaded for 54x56 written, against
// 64x34 for 54x24).
constexpr bool kWide5 = true;
constexpr int kWide5Rows = 64;

// Coefficients of one weighted Jacobi sweep, from omega and D = 2/dx^2 +
// 2/dy^2 + 2/dz^2:  p + (omega/D)(L_p p - b)
//   = (1 - omega) p + kx (pw + pe) + ky (ps + pn) + kz (pt + pb) - kb b,
// kx = omega/(D dx^2), ky = omega/(D dy^2), kz = omega/(D dz^2), kb = omega/D:
// the relaxation (1 - omega) p + omega J(p) of the plain Jacobi update J.
// On a wall plane the zero-gradient ghost equals the centre value, so the
// missing neighbour's kz moves onto the centre coefficient (k0w: one wall,
// k0ww: both walls, nz = 1) and that neighbour gets coefficient 0.
// Computed in double on the host and rounded once to the kernel's type, so
// the kernel holds them in scalar registers as they arrive.
template <typename T>
struct StageCoefs {
    T k0[kMaxFused], k0w[kMaxFused], k0ww[kMaxFused], kx[kMaxFused], ky[kMaxFused], kz[kMaxFused], kb[kMaxFused];
};

template <typename T>
StageCoefs<T> stage_coefs(const Geo& g, const Weights& w, int n)
{
    const double D = 2.0 * (g.idx2 + g.idy2 + g.idz2);
    StageCoefs<T> k{};
    for (int s = 0; s < n; ++s) {
        const double kb = w.omega[s] / D, kz = kb * g.idz2, k0 = 1.0 - w.omega[s];
        k.kx[s] = (T)(kb * g.idx2);
        k.ky[s] = (T)(kb * g.idy2);
        k.kz[s] = (T)kz;
        k.kb[s] = (T)kb;
        k.k0[s] = (T)k0;
        k.k0w[s] = (T)(k0 + kz);
        k.k0ww[s] = (T)(k0 + 2.0 * kz);
    }
    return k;
}

template <typename T>
struct Coef {
    T k0, k0w, k0ww, kx, ky, kz, kb;
};

template <typename T>
__device__ __forceinline__ Coef<T> coef_of(const StageCoefs<T>& kc, int s)
{
    return Coef<T>{kc.k0[s], kc.k0w[s], kc.k0ww[s], kc.kx[s], kc.ky[s], kc.kz[s], kc.kb[s]};
}

// the coefficients of plane q (uniform): centre, top and bottom neighbour
template <typename T>
struct PlaneCoef {
    T k0, kzt, kzb;
};
template <typename T>
__device__ __forceinline__ PlaneCoef<T> plane_coef(const Coef<T>& k, int q, int nz)
{
    // The selects act on the bit patterns: integer selects of uniform values
    // stay in scalar registers (floating-point ones become per-lane
    // v_cndmask), and values rather than references avoid selecting between
    // two fields' addresses, which would keep the coefficients in memory.
    using U = std::conditional_t<sizeof(T) == 4, unsigned, unsigned long long>;
    const U k0 = __builtin_bit_cast(U, k.k0), k0w = __builtin_bit_cast(U, k.k0w), k0ww = __builtin_bit_cast(U, k.k0ww),
            kz = __builtin_bit_cast(U, k.kz);
    const bool top = q == nz - 1, bottom = q == 0;
    // centre coefficient by the number of walls (0, 1, 2) with masks
    const int walls = (int)top + (int)bottom;
    const U m0 = (U)(long long)((walls - 1) >> 31), m2 = (U)(long long)(-(walls >> 1));
    const U c0 = (k0 & m0) | (k0w & ~(m0 | m2)) | (k0ww & m2);
    return PlaneCoef<T>{__builtin_bit_cast(T, c0), __builtin_bit_cast(T, top ? U(0) : kz),
                        __builtin_bit_cast(T, bottom ? U(0) : kz)};
}

template <typename T>
__device__ __forceinline__ T fma_(T a, T b, T c);
template <>
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One weighted Jacobi update of a cell from its six neighbours, with explicit
// fused multiply-adds in a fixed order so the single-sweep and the fused
// kernels round identically: two adds, one multiply, five fused
// multiply-adds.  A wall neighbour has coefficient 0 (its value, any finite
// number, drops out exactly).
template <typename T>
__device__ __forceinline__ T sweep_point(const Coef<T>& k, const PlaneCoef<T>& kq, T pw, T pe, T ps, T pn, T pt, T pb,
                                         T pc, T bb)
{
    T acc = fma_(-k.kb, bb, kq.k0 * pc);
    acc = fma_(k.kx, pw + pe, acc);
    acc = fma_(k.ky, ps + pn, acc);
    acc = fma_(kq.kzt, pt, acc);
    return fma_(kq.kzb, pb, acc);
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
// a right-hand-side value stored as TB (T itself, or a scaled FP16 copy of
// an FP32 residual) widened to T exactly
template <typename T, typename TB>
__device__ __forceinline__ T buf_load_rhs(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(TB) == 2) {
        return (T)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
    } else {
        return buf_load<T>(r, off);
    }
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

// value of the lane below / above in the wavefront (DPP wave shifts); the
// end lanes get 0, as they lie in the tile's halo
__device__ __forceinline__ float lane_from_below(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_above(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_below(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_from_above(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// f(t0 + U, U) for U = 0, 1, ..., in order, with U a compile-time constant
template <typename F, int... U>
__device__ __forceinline__ void unrolled(int t0, F& f, std::integer_sequence<int, U...>)
{
    (f(t0 + U, std::integral_constant<int, U>{}), ...);
}

// FP32 is capped at 128 VGPRs so two workgroups share a CU; FP64 needs about
// 200 VGPRs, one workgroup per CU.
template <typename T>
constexpr int kMinWavesPerSimd = sizeof(T) == 4 ? 4 : 1;

// TY: rows a workgroup updates (two more halo rows are only loaded)
template <typename T, typename TB, int NT, int WAVES, int TY>
__global__ __launch_bounds__(64 * WAVES, kMinWavesPerSimd<T>) void k_relax_fused(int nx, int ny, int nz, int zchunk,
                                                            int tx, int ty, int ntiles,
                                                            const TB* __restrict__ b, const T* __restrict__ p,
                                                            T* __restrict__ out, StageCoefs<T> kc)
{
    constexpr int kTileY = TY, kRows = TY + 2;
    // Workgroups are dealt to the 8 XCDs round-robin (workgroup w runs on XCD
    // w mod 8).  Tile L = (w mod 8) * (grid / 8) + w / 8 gives every XCD a
    // contiguous run of tiles (x fastest, then y, then z-chunk), so the halo
    // a tile shares with its neighbours is read through the same L2.
    const int per_xcd = gridDim.x / kXcds;
    const int tile = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    if (tile >= ntiles) return;
    const int bx = tile % tx, by = (tile / tx) % ty, bz = tile / (tx * ty);
    constexpr int PTS = kTileY / WAVES;  // rows per thread
    constexpr int OX = kTileX - 2 * NT, OY = kRows - 2 * NT;
    // LDS holds, per stage, only the rows read across wavefronts: slot 2w + 1
    // is wavefront w's first row, 2w + 2 its last, 0 and 2 WAVES + 1 the halo
    // rows 0 and kRows - 1.  Wavefront w then reads the row above its first
    // from slot 2w and the row below its last from slot 2w + 3.
    constexpr int kSlots = 2 * WAVES + 2;
    __shared__ T lds[2][NT][kSlots][kTileX];  // step t reads buffer (t-1) & 1, writes t & 1

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int x0 = bx * OX - NT;  // tile origin (may be negative: wrapped)
    const int y0 = by * OY - NT;
    const int z0 = bz * zchunk, z1 = min(nz, z0 + zchunk);
    const long long plane = (long long)nx * ny;
    const unsigned pbytes = (unsigned)(plane * (long long)sizeof(T));
    const unsigned bbytes = (unsigned)(plane * (long long)sizeof(TB));
    // b offsets: this thread's p offsets scaled to TB's size
    constexpr int kBShift = sizeof(T) / sizeof(TB) == 2 ? 1 : 0;

    // global offsets of this thread's columns (periodic wrap)
    const int gx = ((x0 + lane) % nx + nx) % nx;
    // byte offset of this thread's column within a plane: a 32-bit vector
    // offset on a uniform plane address (planes below 4 GiB)
    // Tile rows 1..kTileY are updated (row[m] = 1 + wave PTS + m); rows 0
    // and kRows - 1 are the y halo of the first stage, loaded by the first
    // and the last wavefront and never updated.
    unsigned col[PTS];
    int row[PTS];
#pragma unroll
    for (int m = 0; m < PTS; ++m) {
        row[m] = 1 + wave * PTS + m;
        const int gy = ((y0 + row[m]) % ny + ny) % ny;
        col[m] = (unsigned)(gy * nx + gx) * (unsigned)sizeof(T);
    }
    const int hrow = wave == 0 ? 0 : (wave == WAVES - 1 ? kRows - 1 : -1);  // uniform per wavefront
    const unsigned hcol = (unsigned)(((((y0 + max(hrow, 0)) % ny + ny) % ny) * nx + gx)) * (unsigned)sizeof(T);
    const bool out_x = lane >= NT && lane < kTileX - NT && x0 + lane < nx;

    Coef<T> c[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) c[s] = coef_of<T>(kc, s);

    // The march is unrolled by kUnroll steps so that every register slot is
    // fixed at compile time and no value moves between registers: stage s
    // keeps its last three planes in V[s][(q - t_begin) mod 3], b of the last
    // kRing planes sits in Bz[(q - t_begin) mod kRing], and the LDS buffers
    // alternate with the step's parity.  Plane t + 1 of p and b is requested
    // while plane t is processed (p into Pn, b straight into its slot, which
    // therefore must not hold plane t - NT, still read by the last stage:
    // kRing >= NT + 2, a multiple of 3).  Loads past the top wall are clamped
    // to plane nz - 1; ring slots of planes -1 and nz hold finite stale values
    // that the wall coefficients zero out.
    constexpr int kRing = (NT + 2 + 2) / 3 * 3;
    constexpr int kUnroll = kRing % 2 == 0 ? kRing : 2 * kRing;
    T V[NT][3][PTS];
    T Bz[kRing][PTS];
    T Pn[PTS];
#pragma unroll
    for (int s = 0; s < NT; ++s)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int m = 0; m < PTS; ++m) V[s][k][m] = T(0);
#pragma unroll
    for (int k = 0; k < kRing; ++k)
#pragma unroll
        for (int m = 0; m < PTS; ++m) Bz[k][m] = T(0);

    const int t_begin = max(0, z0 - NT);
    const int t_end = z1 - 1 + NT;  // the final stage reaches plane z1 - 1
    {
        const long long o = plane * t_begin;
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(p + o, pbytes), rb = plane_rsrc(b + o, bbytes);
#pragma unroll
        for (int m = 0; m < PTS; ++m) {
            Pn[m] = buf_load<T>(rp, col[m]);
            Bz[0][m] = buf_load_rhs<T, TB>(rb, col[m] >> kBShift);
        }
    }
    // halo row of the first stage: plane t + 1 is requested (Ph) when plane
    // t arrives (Vh), and Vh goes to LDS at the end of step t
    T Ph = T(0), Vh = T(0);
    if (hrow >= 0) Ph = buf_load<T>(plane_rsrc(p + plane * t_begin, pbytes), hcol);

    // z step t at unroll position U = (t - t_begin) mod kUnroll
    auto step = [&](const int t, auto U) {
        constexpr int u = decltype(U)::value;
        // slot of plane t - k in the stage rings and in the b ring
        auto vs = [](int k) { return ((u - k) % 3 + 3) % 3; };
        auto bs = [](int k) { return ((u - k) % kRing + kRing) % kRing; };
        if (t > t_end) return;
        auto& rd = lds[(u + 1) & 1];  // planes written by the previous step
        auto& wr = lds[u & 1];
        // stage 0: plane t arrives; plane t + 1 is requested (the halo row's
        // first: loads complete in order)
        {
            const long long o = plane * min(t + 1, nz - 1);
            const __amdgpu_buffer_rsrc_t rp = plane_rsrc(p + o, pbytes), rb = plane_rsrc(b + o, bbytes);
            if (hrow >= 0) {
                Vh = Ph;
                Ph = buf_load<T>(rp, hcol);
            }
#pragma unroll
            for (int m = 0; m < PTS; ++m) {
                V[0][vs(0)][m] = Pn[m];
                Pn[m] = buf_load<T>(rp, col[m]);
                Bz[bs(-1)][m] = buf_load_rhs<T, TB>(rb, col[m] >> kBShift);
            }
        }
        // stages 1..NT: stage s produces plane q = t - s from stage s-1's
        // planes q + 1, q, q - 1.  Stage s is needed only on tile rows
        // [s, 34 - s) and on planes [z0 - (NT - s), z1 + (NT - s)) inside the
        // walls; planes outside are skipped (a uniform test), rows outside are
        // computed from neighbours that are not valid and never read.
#pragma unroll
        for (int s = 1; s <= NT; ++s) {
            const int q = t - s;
            if (q < max(0, z0 - (NT - s)) || q > min(nz - 1, z1 - 1 + (NT - s))) continue;
            const PlaneCoef<T> kq = plane_coef(c[s - 1], q, nz);
            T res[PTS];
#pragma unroll
            for (int m = 0; m < PTS; ++m) {
                // x neighbours: the centre register of the neighbouring lanes
                const T pcm = V[s - 1][vs(s)][m];
                // y neighbours: this thread's adjacent rows, or (at the
                // wavefront's first and last row) the neighbouring wavefront's
                // row through LDS
                const T ps = m > 0 ? V[s - 1][vs(s)][m > 0 ? m - 1 : 0] : rd[s - 1][2 * wave][lane];
                const T pn = m + 1 < PTS ? V[s - 1][vs(s)][m + 1 < PTS ? m + 1 : 0] : rd[s - 1][2 * wave + 3][lane];
                res[m] = sweep_point<T>(c[s - 1], kq, lane_from_below(pcm), lane_from_above(pcm), ps, pn,
                                        V[s - 1][vs(s - 1)][m], V[s - 1][vs(s + 1)][m], pcm, Bz[bs(s)][m]);
                if (s < NT) V[s][vs(s)][m] = res[m];
            }
            if (s == NT && q >= z0 && out_x) {
                const __amdgpu_buffer_rsrc_t ro = plane_rsrc(out + plane * q, pbytes);
#pragma unroll
                for (int m = 0; m < PTS; ++m) {
                    const int r = row[m];
                    if (r >= NT && r < kRows - NT && y0 + r < ny) buf_store(res[m], ro, col[m]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NT; ++s)
#pragma unroll
            for (int m = 0; m < PTS; ++m)
            {  // rows other wavefronts read
                if (m == 0) wr[s][2 * wave + 1][lane] = V[s][vs(s)][m];
                if (m == PTS - 1) wr[s][2 * wave + 2][lane] = V[s][vs(s)][m];
            }
        if (hrow >= 0) wr[0][hrow == 0 ? 0 : kSlots - 1][lane] = Vh;
        __syncthreads();  // one barrier: double-buffered planes
    };

    for (int tb = t_begin; tb <= t_end; tb += kUnroll) unrolled(tb, step, std::make_integer_sequence<int, kUnroll>{});
}

// Workgroups of k_relax_fused<T, TB, NT, WAVES, TY> resident on the device at once.
template <typename T, typename TB, int NT, int WAVES, int TY>
int resident_workgroups()
{
    static int cached = 0;  // per kernel instance; one device model per process
    if (cached == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_relax_fused<T, TB, NT, WAVES, TY>, 64 * WAVES,
                                                         0) != hipSuccess)
            return 0;
        cached = std::max(1, cus * per_cu);
    }
    return cached;
}

// Column tiles of a launch fusing NT sweeps over tiles of TY + 2 rows
template <int NT, int TY = kTileY>
long long tile_count(const Geo& g, int* tx = nullptr, int* ty = nullptr)
{
    constexpr int OX = kTileX - 2 * NT, OY = TY + 2 - 2 * NT;
    const int x = (g.nx + OX - 1) / OX, y = (g.ny + OY - 1) / OY;
    if (tx) *tx = x;
    if (ty) *ty = y;
    return (long long)x * y;
}

// Planes per z-chunk: the fewest rounds of resident workgroups times steps
// per chunk (a chunk of zc planes takes zc + 2 NT steps).
int zchunk_planes(long long tiles, int nz, int resident, int nt)
{
    int nzc = 1;
    long long best = -1;
    for (int k = 1; k <= std::max(1, nz / kMinChunk); ++k) {
        const long long zc = (nz + k - 1) / k;
        const long long cost = (tiles * k + resident - 1) / resident * (zc + 2 * nt);
        if (best < 0 || cost < best) {
            best = cost;
            nzc = k;
        }
    }
    return (nz + nzc - 1) / nzc;
}

template <typename T, typename TB, int NT, int WAVES, int TY = kTileY>
hipError_t launch_fused(const Geo& g, const TB* b, const T* p, T* out, const Weights& wts, hipStream_t s)
{
    int tx = 0, ty = 0;
    const long long tiles = tile_count<NT, TY>(g, &tx, &ty);
    const int resident = resident_workgroups<T, TB, NT, WAVES, TY>();
    if (resident == 0) return hipErrorInvalidDevice;
    const int zchunk = zchunk_planes(tiles, g.nz, resident, NT);
    const int nzc = (g.nz + zchunk - 1) / zchunk;
    const int ntiles = (int)(tiles * nzc);
    const int grid = (ntiles + kXcds - 1) / kXcds * kXcds;  // whole rounds over the XCDs
    hipLaunchKernelGGL((k_relax_fused<T, TB, NT, WAVES, TY>), dim3(grid), dim3(64 * WAVES), 0, s, g.nx, g.ny, g.nz,
                       zchunk, tx, ty, ntiles, b, p, out, stage_coefs<T>(g, wts, NT));
    return hipGetLastError();
}

// One sweep per launch, one thread per (i, j) column marching along z with the
// vertical neighbours in registers; used for grids narrower than a tile.
template <typename T, typename TB>
__global__ __launch_bounds__(256) void k_relax(int nx, int ny, int nz, int kchunk, const TB* __restrict__ b,
                                               const T* __restrict__ p, T* __restrict__ out, StageCoefs<T> kc)
{
    const Coef<T> c = coef_of<T>(kc, 0);
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
        out[o + row + i] = sweep_point<T>(c, plane_coef(c, k, nz), p[o + row + im], p[o + row + ip], p[o + rowm + i],
                                          p[o + rowp + i], pt, pb, pc, (T)b[o + row + i]);
        pb = pc;
        pc = pt;
    }
}

}  // namespace

bool relax_fusable(const Geo& g)
{
    return g.nx >= kTileX && g.ny >= kTileY && (long long)g.nx * g.ny < (1LL << 29);
}

// The fusion depth for FP32 sweeps.  Five sweeps per launch on the tall
// 16-wavefront tiles are the fastest wherever those tiles fit the grid
// (measured in the step: 512x256x192, 18.3 us per sweep against 19.2 with
// four per launch on 8-wavefront tiles, 17.3 against 17.8 with the FP16
// right-hand side; 1024x512x384, 139 us per sweep against 164, and 118
// against 137 on 8-wavefront five-sweep tiles with the FP16 right-hand
// side).  On grids too narrow for them: when every workgroup of a four-sweep
// launch is resident at once, the tiles march in z-step and read the halo
// rows they share through L2, and four sweeps per launch do the least vector
// work per update; when the launch needs several rounds of workgroups, the
// halos are fetched once per tile and five sweeps per launch spread that
// traffic over one more sweep.
int relax_auto_depth(const Geo& g)
{
    if (!relax_fusable(g)) return 1;
    if (kWide5 && g.ny >= kWide5Rows + 2) return 5;
    const long long tiles = tile_count<4>(g);
    const int resident = resident_workgroups<float, float, 4, kWaves<float>, kTileY>();
    if (resident == 0) return 4;
    const int zchunk = zchunk_planes(tiles, g.nz, resident, 4);
    const long long launched = tiles * ((g.nz + zchunk - 1) / zchunk);
    return launched > resident ? 5 : 4;
}

template <typename T, typename TB>
hipError_t relax_impl(const Geo& g, const TB* b, const T* p, T* out, const Weights& wts, int nfused, hipStream_t s)
{
    if (nfused == 1 || !relax_fusable(g)) {
        if (nfused != 1) return hipErrorInvalidValue;
        const March m = march_shape(g, 2048);
        hipLaunchKernelGGL((k_relax<T, TB>), m.grid, m.block, 0, s, g.nx, g.ny, g.nz, m.kchunk, b, p, out,
                           stage_coefs<T>(g, wts, 1));
        return hipGetLastError();
    }
    switch (nfused) {
    case 2: return launch_fused<T, TB, 2, kWaves<T>>(g, b, p, out, wts, s);
    case 3: return launch_fused<T, TB, 3, kWaves<T>>(g, b, p, out, wts, s);
    case 4: return launch_fused<T, TB, 4, kWaves<T>>(g, b, p, out, wts, s);
    }
    if constexpr (sizeof(T) == 4) {  // FP64 rings do not fit deeper pipelines in registers
        if (nfused == 5) {
            if (kWide5 && g.ny >= kWide5Rows + 2) return launch_fused<T, TB, 5, 16, kWide5Rows>(g, b, p, out, wts, s);
            return launch_fused<T, TB, 5, kWaves<T>>(g, b, p, out, wts, s);
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t relax(const Geo& g, const T* b, const T* p, T* out, const Weights& wts, int nfused, hipStream_t s)
{
    return relax_impl<T, T>(g, b, p, out, wts, nfused, s);
}
template hipError_t relax<double>(const Geo&, const double*, const double*, double*, const Weights&, int, hipStream_t);
template hipError_t relax<float>(const Geo&, const float*, const float*, float*, const Weights&, int, hipStream_t);

hipError_t relax(const Geo& g, const _Float16* b, const float* p, float* out, const Weights& wts, int nfused,
                 hipStream_t s)
{
    return relax_impl<float, _Float16>(g, b, p, out, wts, nfused, s);
}

}  // namespace stp
