// Learned warm start: 3-level 3-D convolutional network with BF16 MFMA
// forward and backward kernels for gfx950, FP32 accumulation.
//
// Tensors are channels-last BF16, channel counts padded to multiples of 16
// (the 2 input channels and the 1 output channel are padded with zero
// weights, which stay zero under training because their gradients vanish).
// A 3x3x3 convolution is an implicit GEMM: M = cells, N = output channels,
// K = 27 taps x input channels, computed 16 x 16 x 16 at a time by
// v_mfma_f32_16x16x16_bf16; every wavefront owns 16 consecutive cells and all
// output channels, so an A fragment (8 bytes per lane, contiguous channels of
// the neighbour cell, periodic in x and y, zero beyond the walls) is reused
// across the output-channel tiles.  The input gradient is the same kernel
// with flipped, transposed weights; the weight gradient is a GEMM over cells
// (M = output channels, N = input channels, K = cells) staged through LDS,
// one tap per workgroup, reduced over cell chunks in a fixed order.
#include "stp_net.h"

#include <algorithm>
#include <type_traits>
#include <cmath>

namespace stp {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct Lvl {
    int nx, ny, nz;
    long long n;
};

// round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ void cell_xyz(const Lvl& L, long long v, int& x, int& y, int& z)
{
    x = (int)(v % L.nx);
    const long long r = v / L.nx;
    y = (int)(r % L.ny);
    z = (int)(r / L.ny);
}

// ---- reductions (fixed order) --------------------------------------------------

__device__ double block_sum(double v, double* lds)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) r += lds[w];
    return r;
}

constexpr int kRedBlocks = 2048;  // 8 workgroups per CU keep enough loads in flight

// part[q * kRedBlocks + block] for q < 2: sums of f0(v), f1(v)
__global__ __launch_bounds__(256) void k_sum_p(const double* __restrict__ p, long long n, double* __restrict__ part)
{
    __shared__ double lds[8];
    double a = 0.0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
        a += p[v];
    a = block_sum(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void k_mean_from(const double* __restrict__ part, long long n, double* __restrict__ sc)
{
    __shared__ double lds[8];
    double a = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) a += part[b];
    a = block_sum(a, lds);
    if (threadIdx.x == 0) sc[0] = a / (double)n;
}

// L p at cell v (periodic in x, y; zero normal gradient at the walls)
struct LapGeo {
    int nx, ny, nz;
    double idx2, idy2, idz2;
};
// Cell coordinates along a grid-stride loop: divisions once per thread,
// then the stride is added with carries (x fastest).
struct CellIter {
    long long v;
    int x, y, z;
    int sx, sy;
    long long sz;
    __device__ CellIter(const LapGeo& G, long long v0, long long stride) : v(v0)
    {
        const long long plane = (long long)G.nx * G.ny;
        x = (int)(v0 % G.nx);
        y = (int)((v0 / G.nx) % G.ny);
        z = (int)(v0 / plane);
        sx = (int)(stride % G.nx);
        sy = (int)((stride / G.nx) % G.ny);
        sz = stride / plane;
    }
    __device__ void advance(const LapGeo& G, long long stride)
    {
        v += stride;
        x += sx;
        int carry = 0;
        if (x >= G.nx) {
            x -= G.nx;
            carry = 1;
        }
        y += sy + carry;
        carry = 0;
        if (y >= G.ny) {
            y -= G.ny;
            carry = 1;
        }
        z += (int)sz + carry;
    }
};

__device__ __forceinline__ double lap_at(const LapGeo& G, const double* __restrict__ p, long long v, int x, int y, int z)
{
    const long long plane = (long long)G.nx * G.ny;
    const long long row = v - x, pl = v - (long long)y * G.nx - x;
    const double pc = p[v];
    const double pe = p[row + (x == G.nx - 1 ? 0 : x + 1)], pw = p[row + (x == 0 ? G.nx - 1 : x - 1)];
    const double pn = p[pl + (long long)(y == G.ny - 1 ? 0 : y + 1) * G.nx + x];
    const double ps = p[pl + (long long)(y == 0 ? G.ny - 1 : y - 1) * G.nx + x];
    const double pt = z + 1 < G.nz ? p[v + plane] : pc;
    const double pb = z > 0 ? p[v - plane] : pc;
    return (pw + pe - 2.0 * pc) * G.idx2 + (ps + pn - 2.0 * pc) * G.idy2 + ((pt - pc) + (pb - pc)) * G.idz2;
}

// partial sums of (p - mean)^2 and (r / D)^2 with r = b - L p
__global__ __launch_bounds__(256) void k_sumsq_pr(LapGeo G, const double* __restrict__ p, const double* __restrict__ b,
                                                  long long n, double invD, const double* __restrict__ sc,
                                                  double* __restrict__ part)
{
    __shared__ double lds[8];
    const double m = sc[0];
    double a = 0.0, c = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (CellIter it(G, blockIdx.x * (long long)blockDim.x + threadIdx.x, stride); it.v < n; it.advance(G, stride)) {
        const long long v = it.v;
        const double d = p[v] - m;
        a += d * d;
        const double e = (b[v] - lap_at(G, p, v, it.x, it.y, it.z)) * invD;
        c += e * e;
    }
    a = block_sum(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
    c = block_sum(c, lds);
    if (threadIdx.x == 0) part[kRedBlocks + blockIdx.x] = c;
}

// sc[1] = s_r = rms(r / D), sc[3] = s_p = rms(p - mean); 1 where zero
__global__ __launch_bounds__(256) void k_scale_from(const double* __restrict__ part, long long n, double* __restrict__ sc)
{
    __shared__ double lds[8];
    double a = 0.0, c = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) {
        a += part[b];
        c += part[kRedBlocks + b];
    }
    a = block_sum(a, lds);
    c = block_sum(c, lds);
    if (threadIdx.x == 0) {
        double sp = sqrt(a / (double)n), sr = sqrt(c / (double)n);
        sc[1] = sr == 0.0 ? 1.0 : sr;
        sc[3] = sp == 0.0 ? 1.0 : sp;
    }
}

// X[v] = (r/(D s_r), (p - mean)/s_p, 0 ...) in BF16, xstride (8 or 16) channels per cell
__global__ void k_normalise(LapGeo G, const double* __restrict__ b, const double* __restrict__ p, long long n,
                            double invD, const double* __restrict__ sc, uint16_t* __restrict__ X, int xstride)
{
    const double m = sc[0], sr = sc[1], sp = sc[3];
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (CellIter it(G, blockIdx.x * (long long)blockDim.x + threadIdx.x, stride); it.v < n; it.advance(G, stride)) {
        const long long v = it.v;
        const unsigned c01 = f2bf((float)((b[v] - lap_at(G, p, v, it.x, it.y, it.z)) * invD / sr)) |
                             ((unsigned)f2bf((float)((p[v] - m) / sp)) << 16);
        u32x4* o = reinterpret_cast<u32x4*>(X + v * xstride);
        o[0] = u32x4{c01, 0u, 0u, 0u};
        if (xstride == 16) o[1] = u32x4{0u, 0u, 0u, 0u};
    }
}

// ---- convolution forward / input gradient --------------------------------------

enum { OUT_BF16 = 0, OUT_F32 = 1, OUT_HEAD = 2, OUT_POOL = 3 };

// out[v][co] = act(bias[co] + sum_{tap, ci} in[nbr(v, tap)][ci] w[tap][co][ci])
// MODE OUT_BF16: BF16 into a channel slice (ostride, ooff) with bias and
// optional ReLU; OUT_F32: FP32 contiguous, no bias; OUT_HEAD: FP32 channel 0
// with bias.
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(Lvl L, const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                              const float* __restrict__ bias, void* __restrict__ out, int ostride,
                                              int ooff, int relu)
{
    constexpr int NT = COUT / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const long long v0 = ((long long)blockIdx.x * 4 + wave) * 16;
    const long long va = v0 + m;
    const bool valid = va < L.n;
    int x = 0, y = 0, z = 0;
    if (valid) cell_xyz(L, va, x, y, z);
    floatx4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bf16x4 zero4 = bf16x4{0, 0, 0, 0};
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const int zz = z + dz;
        const bool ok = valid && zz >= 0 && zz < L.nz;
        int yy = y + dy, xx = x + dx;
        yy = yy < 0 ? yy + L.ny : (yy >= L.ny ? yy - L.ny : yy);
        xx = xx < 0 ? xx + L.nx : (xx >= L.nx ? xx - L.nx : xx);
        const long long nb = ok ? (((long long)zz * L.ny + yy) * L.nx + xx) : 0;
        const uint16_t* src = in + nb * CIN + 4 * kq;
        const uint16_t* wt = w + (long long)t * COUT * CIN + (long long)m * CIN + 4 * kq;
#pragma unroll
        for (int c0 = 0; c0 < CIN; c0 += 16) {
            const bf16x4 a = ok ? *reinterpret_cast<const bf16x4*>(src + c0) : zero4;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const bf16x4 bb = *reinterpret_cast<const bf16x4*>(wt + (long long)16 * j * CIN + c0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[j], 0, 0, 0);
            }
        }
    }
    // acc[j][r] = D[cell 4 kq + r][channel m] of tile j
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = 16 * j + m;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long long v = v0 + 4 * kq + r;
            if (v >= L.n) continue;
            float val = acc[j][r];
            if (MODE == OUT_BF16) {
                val += bias[co];
                if (relu) val = fmaxf(val, 0.f);
                static_cast<uint16_t*>(out)[v * ostride + ooff + co] = f2bf(val);
            } else if (MODE == OUT_F32) {
                static_cast<float*>(out)[v * COUT + co] = val;
            } else if (co == 0) {
                static_cast<float*>(out)[v] = val + bias[0];
            }
        }
    }
}

template <int CIN, int COUT, int MODE>
hipError_t conv(const Lvl& L, const uint16_t* in, const uint16_t* w, const float* bias, void* out, int ostride, int ooff,
                int relu, hipStream_t s)
{
    const long long blocks = (L.n + 63) / 64;
    hipLaunchKernelGGL((k_conv<CIN, COUT, MODE>), dim3((unsigned)blocks), dim3(256), 0, s, L, in, w, bias, out, ostride,
                       ooff, relu);
    return hipGetLastError();
}

// ---- plane-marching convolution (forward) ----------------------------------------
//
// The same operator as k_conv for one 16-channel output tile per workgroup,
// computed as D^T = W X^T with v_mfma_f32_16x16x32_bf16 (A: 16 output channels
// x 32 of K, B: 32 of K x 16 cells).  Within one dz slice K is ordered
// (dy, dx, ci): K9 = 9 CIN, padded to whole 32-chunks with zero weights.  The
// workgroup owns a 32 x (2 WAVES) tile of an x-y plane and marches along z one
// INPUT plane at a time: the plane, with a one-cell halo (periodic in x and y),
// sits in LDS, and every B fragment read from it feeds the three dz weight
// slices, accumulating into output planes j + 1, j and j - 1; plane j - 1 is
// then complete and stored.  Input fragments are thus read from LDS once per
// plane instead of 27 times from cache, the weights of the tile sit in LDS in
// fragment order (one 16-byte read per lane), and the next input plane is
// loaded into registers while the current one is computed.  The input may be
// the concatenation of two tensors, the first optionally at half resolution
// (nearest upsampling folded into the load).

struct SrcView {  // channels-last BF16 slice: element (cell, c) at p[cell * stride + off + c]
    const uint16_t* p;
    int stride, off;
    int nx, ny, nz;  // its own grid (the coarse grid when upsampled)
};

template <int CIN, int WAVES>
struct PlaneTile {
    static constexpr int TX = 32, TY = 2 * WAVES, HX = TX + 2, HY = TY + 2;
    static constexpr int CU = CIN / 8;  // 16-byte channel groups per cell
    // LDS bytes per cell: an odd number of 16-byte units, so the 16 cells of a
    // fragment fall on distinct banks
    static constexpr int CSTR = (CU % 2 == 1 ? CU : CU + 1) * 16;
    static constexpr int PLANE = HX * HY * CSTR;
    static constexpr int KC = (9 * CIN + 31) / 32;  // K chunks per dz slice
    static constexpr int WBYTES = 3 * KC * 64 * 16;  // fragment-ordered weights of one output tile
    static constexpr int NCHUNK = HX * HY * CU;      // 16-byte loads per plane
};

// 16-byte load slots per thread of a halo plane whose first CA channels come
// from one source and the rest from another: each slot reads one source only
template <int CIN, int CA, int WAVES>
struct PlaneSlots {
    static constexpr int T = 64 * WAVES, HXY = PlaneTile<CIN, WAVES>::HX * PlaneTile<CIN, WAVES>::HY;
    static constexpr int NA = HXY * (CA / 8), NB = HXY * ((CIN - CA) / 8);
    static constexpr int SA = (NA + T - 1) / T, SB = (NB + T - 1) / T, S = SA + SB;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// The first layer (8 input channels) and the head fit in 128 VGPRs and keep
// four waves per SIMD (two workgroups per CU), which hide the LDS latency
// between K chunks; there the chunks are kept apart in the schedule, so that
// the compiler does not hoist all fragment reads.  Wider layers are limited by
// LDS to one workgroup per CU and rely on the compiler's interleaving.
template <int CIN, int MODE>
constexpr int kConvMinWaves = CIN <= 8 || MODE == 2 ? 4 : 1;

template <int CIN, int CA, bool UPA, int WAVES, int MODE>
__global__ __launch_bounds__(64 * WAVES, (kConvMinWaves<CIN, MODE>)) void k_conv_march(Lvl L, SrcView A, SrcView B, const u32x4* __restrict__ wf,
                                                           const float* __restrict__ bias, void* __restrict__ out,
                                                           int ostride, int ooff, int relu, int zchunk, int ncot,
                                                           uint16_t* __restrict__ pool, int pstride)
{
    using PT = PlaneTile<CIN, WAVES>;
    static_assert(CIN % 8 == 0 && CA % 8 == 0 && CA <= CIN, "channel groups of 8");
    __shared__ __align__(16) unsigned char sx[PT::PLANE + 16];  // plane + sink
    __shared__ u32x4 sw[PT::WBYTES / 16];
    __shared__ float sbias[16];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int jc = lane & 15, g = lane >> 4;
    const int cot = blockIdx.z % ncot;
    const int z0 = (blockIdx.z / ncot) * zchunk, z1 = min(L.nz, z0 + zchunk);
    const int x0 = blockIdx.x * PT::TX, y0 = blockIdx.y * PT::TY;

    // weights and bias of this output tile into LDS
    for (int e = tid; e < PT::WBYTES / 16; e += 64 * WAVES) sw[e] = wf[(long long)cot * (PT::WBYTES / 16) + e];
    if (tid < 16) sbias[tid] = bias ? bias[16 * cot + tid] : 0.f;

    // This thread's 16-byte slots of the halo plane: SA slots over the CA / 8
    // channel groups of A of every halo cell, then SB slots over those of B,
    // each slot reading one source with 32-bit offsets into a buffer resource
    // of one source plane.  Lanes past the end of a source load nothing (an
    // offset beyond the plane) and store into a 16-byte sink behind the plane.
    using SL = PlaneSlots<CIN, CA, WAVES>;
    constexpr int CUA = CA / 8, CUB = PT::CU - CUA;
    constexpr unsigned kPast = 0x80000000u;
    const unsigned bytesA = (unsigned)A.nx * (unsigned)A.ny * (unsigned)A.stride * 2u;
    const unsigned bytesB = (unsigned)B.nx * (unsigned)B.ny * (unsigned)B.stride * 2u;
    unsigned soff[SL::S];
    int loff[SL::S];
#pragma unroll
    for (int s = 0; s < SL::S; ++s) {
        const bool inA = s < SL::SA;
        const int e = tid + (inA ? s : s - SL::SA) * SL::T;
        const int cpc = inA ? CUA : (CUB > 0 ? CUB : 1);  // groups per cell in this source
        const int h = e / cpc, cu = e - h * cpc;
        const int hx = h % PT::HX, hy = h / PT::HX;
        int gx = (x0 - 1 + hx) % L.nx, gy = (y0 - 1 + hy) % L.ny;
        gx = gx < 0 ? gx + L.nx : gx;
        gy = gy < 0 ? gy + L.ny : gy;
        const int ax = UPA ? gx / 2 : gx, ay = UPA ? gy / 2 : gy;
        if (inA) {
            const bool live = e < SL::NA;
            soff[s] = live ? (unsigned)(((ay * A.nx + ax) * A.stride + A.off + 8 * cu) * 2) : kPast;
            loff[s] = live ? h * PT::CSTR + 16 * cu : PT::PLANE;
        } else {
            const bool live = e < SL::NB;
            soff[s] = live ? (unsigned)(((gy * B.nx + gx) * B.stride + B.off + 8 * cu) * 2) : kPast;
            loff[s] = live ? h * PT::CSTR + 16 * (CUA + cu) : PT::PLANE;
        }
    }
    u32x4 pre[SL::S];
    auto load_plane = [&](int j) {
        const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(A.p) + (long long)(UPA ? j / 2 : j) * (bytesA / 2), (short)0, (int)bytesA, 0x00020000);
        const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint16_t*>(B.p) + (long long)j * (bytesB / 2), (short)0, (int)bytesB, 0x00020000);
#pragma unroll
        for (int s = 0; s < SL::S; ++s)
            pre[s] = __builtin_amdgcn_raw_buffer_load_b128(s < SL::SA ? rA : rB, soff[s], 0, 0);
    };
    auto store_plane = [&]() {
#pragma unroll
        for (int s = 0; s < SL::S; ++s) *reinterpret_cast<u32x4*>(sx + loff[s]) = pre[s];
    };

    // B fragments: chunk q, lane group g covers k = 32 q + 8 g .. + 7, i.e.
    // tap9 = k / CIN (dy + 1 = tap9 / 3, dx + 1 = tap9 % 3), channels c.  The
    // weights of k >= 9 CIN are zero, so those lanes read any finite operand
    // (tap 0).  kb[q] addresses the lane's cell in the wave's first 16-cell
    // tile; the four tiles (rows 2 wave + (n >> 1), x halves n & 1) sit at
    // fixed distances from it.
    int kb[PT::KC];
#pragma unroll
    for (int q = 0; q < PT::KC; ++q) {
        const int k = 32 * q + 8 * g < 9 * CIN ? 32 * q + 8 * g : 0;
        const int tap = k / CIN, c = k - tap * CIN;
        kb[q] = ((2 * wave + tap / 3) * PT::HX + jc + tap % 3) * PT::CSTR + 2 * c;
    }
    constexpr int kTileOff[4] = {0, 16 * PT::CSTR, PT::HX * PT::CSTR, (PT::HX + 16) * PT::CSTR};

    // Output plane t accumulates in acc[(t - z0 + 1) mod 3]; the z loop is
    // unrolled by three so that the slots are static.
    floatx4 acc[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[d][n] = floatx4{0.f, 0.f, 0.f, 0.f};

    // Output plane z through a buffer resource: lanes outside the grid (and,
    // for the head, lanes of channels other than 0) get an offset beyond the
    // plane, which the buffer range check drops.  No branch, so the wait for
    // the next plane's loads does not also wait for these stores.
    //
    // OUT_POOL also writes the 2 x 2 x 2 mean of the stored (BF16) output at
    // half resolution into pool (pstride channels, this tile's 16 from
    // 16 cot), summed in the order x, then y, then z fastest-first: the
    // x pair sits in lanes jc, jc + 1, the y pair in tiles n, n + 2 of the
    // same lane, and the z pair in consecutive planes, carried in psum.
    constexpr unsigned ESZ = MODE == OUT_HEAD ? 4u : 2u;
    const unsigned pbytes = (unsigned)L.nx * (unsigned)L.ny * (unsigned)ostride * ESZ;
    const unsigned qbytes = (unsigned)(L.nx / 2) * (unsigned)(L.ny / 2) * (unsigned)pstride * 2u;
    float psum[2][4] = {};
    float bv[4];  // from LDS once the weights are staged
    auto store_out = [&](int z, const floatx4* o, bool live) {
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            static_cast<char*>(out) + (long long)max(z, 0) * pbytes, (short)0, (int)pbytes, 0x00020000);
        unsigned h[4][2];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int x = x0 + 16 * (n & 1) + jc, y = y0 + 2 * wave + (n >> 1);
            const bool in = live && x < L.nx && y < L.ny;
            const unsigned v = (unsigned)y * (unsigned)L.nx + (unsigned)x;
            if (MODE == OUT_HEAD) {  // channel 0 only
                const unsigned off = in && g == 0 ? v * ESZ : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, o[n][0] + bv[0]), r, off, 0, 0);
            } else {
                float val[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) val[q] = relu ? fmaxf(o[n][q] + bv[q], 0.f) : o[n][q] + bv[q];
                h[n][0] = f2bf(val[0]) | ((unsigned)f2bf(val[1]) << 16);
                h[n][1] = f2bf(val[2]) | ((unsigned)f2bf(val[3]) << 16);
                const unsigned off = in ? (v * ostride + ooff + 16 * cot + 4 * g) * ESZ : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{h[n][0], h[n][1]}, r, off, 0, 0);
            }
        }
        if (MODE == OUT_POOL) {
            const bool odd = z & 1;
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const unsigned sh = 16 * (q & 1);
                    const float f0 = __uint_as_float((h[m][q >> 1] >> sh) << 16);
                    const float f2 = __uint_as_float((h[m + 2][q >> 1] >> sh) << 16);
                    // quad_perm [1, 1, 3, 3]: the even lane of each pair gets its odd neighbour
                    const float f0n = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, f0), 0xF5, 0xf, 0xf, false));
                    const float f2n = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, f2), 0xF5, 0xf, 0xf, false));
                    float a = odd ? psum[m][q] : 0.f;
                    a += f0;
                    a += f0n;
                    a += f2;
                    a += f2n;
                    psum[m][q] = a;
                }
            {  // written on odd planes only, but issued on every plane (see above)
                const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(
                    pool + (long long)max(z >> 1, 0) * (qbytes / 2), (short)0, (int)qbytes, 0x00020000);
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int x = x0 + 16 * m + jc, y = y0 + 2 * wave;
                    const bool in = live && odd && x < L.nx && y < L.ny && (jc & 1) == 0;
                    const unsigned v = (unsigned)(y >> 1) * (unsigned)(L.nx >> 1) + (unsigned)(x >> 1);
                    const unsigned off = in ? (v * pstride + 16 * cot + 4 * g) * 2u : 0x80000000u;
                    __builtin_amdgcn_raw_buffer_store_b64(
                        u32x2{f2bf(psum[m][0] * 0.125f) | ((unsigned)f2bf(psum[m][1] * 0.125f) << 16),
                              f2bf(psum[m][2] * 0.125f) | ((unsigned)f2bf(psum[m][3] * 0.125f) << 16)},
                        rq, off, 0, 0);
                }
            }
        }
    };

    __syncthreads();  // weights and bias in LDS
#pragma unroll
    for (int r = 0; r < 4; ++r) bv[r] = sbias[4 * g + r];
    if (z0 - 1 >= 0) {
        load_plane(z0 - 1);
        store_plane();
    }
    __syncthreads();
    // step with input plane j (in LDS), U = (j - z0 + 1) mod 3: the dz slices
    // d = 0, 1, 2 add to output planes j + 1, j, j - 1; plane j - 1 is then
    // complete, stored, and its slot cleared for plane j + 2
    auto step = [&](const int j, auto U) {
        constexpr int u = decltype(U)::value;
        constexpr int slot[3] = {(u + 1) % 3, u, (u + 2) % 3};
        const bool next = j + 1 <= z1 && j + 1 < L.nz;  // uniform
        if (next) load_plane(j + 1);
        if (j >= 0 && j < L.nz) {
#pragma unroll
            for (int q = 0; q < PT::KC; ++q) {
                bf16x8 bx[4];
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    bx[n] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(sx + kb[q] + kTileOff[n]));
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const bf16x8 aw = __builtin_bit_cast(bf16x8, sw[(d * PT::KC + q) * 64 + lane]);
#pragma unroll
                    for (int n = 0; n < 4; ++n)
                        acc[slot[d]][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx[n], acc[slot[d]][n], 0, 0, 0);
                }
                if (kConvMinWaves<CIN, MODE> > 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
        // unconditional, so that the stores are the same on every path and
        // the wait for the next plane's loads need not cover them
        store_out(j - 1, acc[slot[2]], j - 1 >= z0);
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[slot[2]][n] = floatx4{0.f, 0.f, 0.f, 0.f};
        __syncthreads();  // all reads of plane j done
        if (next) store_plane();
        __syncthreads();
    };
    for (int j = z0 - 1; j <= z1; j += 3) {
        step(j, std::integral_constant<int, 0>{});
        if (j + 1 > z1) break;
        step(j + 1, std::integral_constant<int, 1>{});
        if (j + 2 > z1) break;
        step(j + 2, std::integral_constant<int, 2>{});
    }
}

template <int CIN, int CA, bool UPA, int WAVES, int MODE>
hipError_t conv_march(const Lvl& L, const SrcView& A, const SrcView& B, const uint16_t* wf, int ncot,
                      const float* bias, void* out, int ostride, int ooff, int relu, hipStream_t s,
                      uint16_t* pool = nullptr, int pstride = 0)
{
    using PT = PlaneTile<CIN, WAVES>;
    // planes of the output and of both sources stay below 2^31 bytes (32-bit
    // buffer offsets, with 2^31 as the out-of-range marker)
    if ((long long)L.nx * L.ny * ostride * (MODE == OUT_BF16 ? 2 : 4) >= (1ll << 31) ||
        (long long)A.nx * A.ny * A.stride * 2 >= (1ll << 31) || (long long)B.nx * B.ny * B.stride * 2 >= (1ll << 31))
        return hipErrorInvalidValue;
    const int tx = (L.nx + PT::TX - 1) / PT::TX, ty = (L.ny + PT::TY - 1) / PT::TY;
    // z chunks: about 2048 workgroups, at least 8 output planes each
    const long long tiles = (long long)tx * ty * ncot;
    int nzc = (int)std::max<long long>(1, std::min<long long>(L.nz / 8, (2048 + tiles - 1) / tiles));
    int zchunk = (L.nz + nzc - 1) / nzc;
    if (MODE == OUT_POOL) {  // whole z pairs per workgroup, even extents
        if (L.nx % 2 || L.ny % 2 || L.nz % 2 || pool == nullptr || pstride < 16 * ncot ||
            (long long)(L.nx / 2) * (L.ny / 2) * pstride * 2 >= (1ll << 31))
            return hipErrorInvalidValue;
        zchunk += zchunk & 1;
    }
    nzc = (L.nz + zchunk - 1) / zchunk;
    hipLaunchKernelGGL((k_conv_march<CIN, CA, UPA, WAVES, MODE>), dim3(tx, ty, nzc * ncot), dim3(64 * WAVES), 0, s, L, A,
                       B, reinterpret_cast<const u32x4*>(wf), bias, out, ostride, ooff, relu, zchunk, ncot, pool,
                       pstride);
    return hipGetLastError();
}

// Wf[cot][dz][q][lane][e] = Wb[dz 9 + tap9][16 cot + (lane & 15)][c + e] with
// k = 32 q + 8 (lane >> 4) + e, tap9 = k / cin_eff, c = k % cin_eff (zero for
// k >= 9 cin_eff): the A fragments of k_conv_march in reading order.
__global__ void k_pack_frag(const uint16_t* __restrict__ Wb, int cout, int cin_mem, int cin_eff, int kc,
                            uint16_t* __restrict__ Wf)
{
    const long long total = (long long)(cout / 16) * 3 * kc * 64 * 8;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int el = (int)(e % 8), lane = (int)((e / 8) % 64), q = (int)((e / 512) % kc);
        const int dz = (int)((e / (512LL * kc)) % 3), cot = (int)(e / (1536LL * kc));
        const int k = 32 * q + 8 * (lane >> 4) + el;
        uint16_t h = 0;
        if (k < 9 * cin_eff) {
            const int tap = k / cin_eff, c = k % cin_eff;
            h = Wb[((long long)(dz * 9 + tap) * cout + 16 * cot + (lane & 15)) * cin_mem + c];
        }
        Wf[e] = h;
    }
}

// ---- weight gradient ----------------------------------------------------------------

// part[chunk][tap][co][ci] = sum over the chunk's cells v of
// dout[v][co] * in[nbr(v, tap)][ci]; one tap per workgroup (blockIdx.y).
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(Lvl L, const uint16_t* __restrict__ in, const uint16_t* __restrict__ dout,
                                               float* __restrict__ part, long long vchunk)
{
    constexpr int TM = COUT / 16, TN = CIN / 16, TT = TM * TN, TPW = (TT + 3) / 4;
    __shared__ uint16_t sA[64][COUT + 4];
    __shared__ uint16_t sB[64][CIN + 4];
    const int t = blockIdx.y;
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const long long vbeg = (long long)blockIdx.x * vchunk;
    const long long vend = min(L.n, vbeg + vchunk);
    floatx4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (long long vb = vbeg; vb < vend; vb += 64) {
        // stage 64 cells of dout and the tap-shifted input
        for (int e = threadIdx.x; e < 64 * COUT; e += blockDim.x) {
            const int c = e / COUT, ch = e % COUT;
            const long long v = vb + c;
            sA[c][ch] = v < vend ? dout[v * COUT + ch] : (uint16_t)0;
        }
        for (int e = threadIdx.x; e < 64 * CIN; e += blockDim.x) {
            const int c = e / CIN, ch = e % CIN;
            const long long v = vb + c;
            uint16_t val = 0;
            if (v < vend) {
                int x, y, z;
                cell_xyz(L, v, x, y, z);
                const int zz = z + dz;
                if (zz >= 0 && zz < L.nz) {
                    int yy = y + dy, xx = x + dx;
                    yy = yy < 0 ? yy + L.ny : (yy >= L.ny ? yy - L.ny : yy);
                    xx = xx < 0 ? xx + L.nx : (xx >= L.nx ? xx - L.nx : xx);
                    val = in[(((long long)zz * L.ny + yy) * L.nx + xx) * CIN + ch];
                }
            }
            sB[c][ch] = val;
        }
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                const int tile = wave + 4 * q;
                if (tile >= TT) break;
                const int tm = tile / TN, tn = tile % TN;
                bf16x4 a, bb;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    a[r] = (short)sA[16 * kc + 4 * kq + r][16 * tm + m];
                    bb[r] = (short)sB[16 * kc + 4 * kq + r][16 * tn + m];
                }
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    float* o = part + ((long long)blockIdx.x * 27 + t) * COUT * CIN;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile >= TT) break;
        const int tm = tile / TN, tn = tile % TN;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[(16 * tm + 4 * kq + r) * CIN + 16 * tn + m] = acc[q][r];
    }
}

// g[i] = sum over chunks of part[chunk][i], i < 27*COUT*CIN
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nchunk, long long per, float* __restrict__ g)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < per; i += (long long)gridDim.x * blockDim.x) {
        float a = 0.f;
        for (int c = 0; c < nchunk; ++c) a += part[(long long)c * per + i];
        g[i] = a;
    }
}

template <int CIN, int COUT>
hipError_t wgrad(const Lvl& L, const uint16_t* in, const uint16_t* dout, float* part, long long part_floats, float* g,
                 hipStream_t s)
{
    const long long per = 27LL * COUT * CIN;
    long long nchunk = std::min<long long>((L.n + 4095) / 4096, std::max<long long>(1, part_floats / per));
    nchunk = std::max<long long>(1, std::min<long long>(nchunk, 65535));
    long long vchunk = (L.n + nchunk - 1) / nchunk;
    vchunk = (vchunk + 63) / 64 * 64;
    nchunk = (L.n + vchunk - 1) / vchunk;
    hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3((unsigned)nchunk, 27), dim3(256), 0, s, L, in, dout, part, vchunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)std::min<long long>(1024, (per + 255) / 256)), dim3(256), 0, s, part,
                       (int)nchunk, per, g);
    return hipGetLastError();
}

// bias gradient: g[co] = sum_v dout[v][co]; partials per block then a fixed-order sum
__global__ __launch_bounds__(256) void k_bgrad_part(const uint16_t* __restrict__ dout, long long n, int C,
                                                    float* __restrict__ part)
{
    // thread handles channel (threadIdx.x % C) for cells strided by blockDim.x / C
    const int ch = threadIdx.x % C, lane_cells = blockDim.x / C, cell0 = threadIdx.x / C;
    float a = 0.f;
    if (cell0 < lane_cells)
        for (long long v = (long long)blockIdx.x * lane_cells + cell0; v < n; v += (long long)gridDim.x * lane_cells)
            a += bf2f(dout[v * C + ch]);
    __shared__ float s[256];
    s[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x < C) {
        float t = 0.f;
        for (int c = 0; c < lane_cells; ++c) t += s[c * C + threadIdx.x];
        part[(long long)blockIdx.x * C + threadIdx.x] = t;
    }
}

__global__ void k_bgrad_reduce(const float* __restrict__ part, int nblk, int C, float* __restrict__ g)
{
    const int ch = threadIdx.x;
    if (ch >= C) return;
    float a = 0.f;
    for (int b = 0; b < nblk; ++b) a += part[(long long)b * C + ch];
    g[ch] = a;
}

// ---- pooling, upsampling, concatenation and their adjoints ---------------------------

// dst[v][doff + c] (stride dstride) = src[parent(v)][c]; Lf: fine level
__global__ void k_up(Lvl Lf, const uint16_t* __restrict__ src, int C, uint16_t* __restrict__ dst, int dstride, int doff)
{
    const long long total = Lf.n * C;
    const int cnx = Lf.nx / 2, cny = Lf.ny / 2;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long v = e / C;
        const int c = (int)(e % C);
        int x, y, z;
        cell_xyz(Lf, v, x, y, z);
        const long long pv = ((long long)(z / 2) * cny + y / 2) * cnx + x / 2;
        dst[v * dstride + doff + c] = src[pv * C + c];
    }
}

// dst[v][c] = bf16(src[v][c] * (act[v * astride + aoff + c] > 0))
__global__ void k_mask_round(long long n, int C, const float* __restrict__ src, const uint16_t* __restrict__ act,
                             int astride, int aoff, uint16_t* __restrict__ dst)
{
    const long long total = n * C;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long v = e / C;
        const int c = (int)(e % C);
        const bool on = bf2f(act[v * astride + aoff + c]) > 0.f;
        dst[e] = f2bf(on ? src[e] : 0.f);
    }
}

// adjoint of upsampling then mask: dst[v'][c] = bf16(sum_8 src[child][soff + c] * (act[v'] > 0)); Lc: coarse level
__global__ void k_upbwd_mask(Lvl Lc, const float* __restrict__ src, int sstride, int soff, int C,
                             const uint16_t* __restrict__ act, int astride, int aoff, uint16_t* __restrict__ dst)
{
    const long long total = Lc.n * C;
    const int fnx = 2 * Lc.nx, fny = 2 * Lc.ny;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long v = e / C;
        const int c = (int)(e % C);
        int x, y, z;
        cell_xyz(Lc, v, x, y, z);
        float a = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const long long f = ((long long)(2 * z + (q >> 2)) * fny + (2 * y + ((q >> 1) & 1))) * fnx + (2 * x + (q & 1));
            a += src[f * sstride + soff + c];
        }
        const bool on = bf2f(act[v * astride + aoff + c]) > 0.f;
        dst[e] = f2bf(on ? a : 0.f);
    }
}

// skip path plus adjoint of pooling, then mask:
// dst[v][c] = bf16((src[v][soff + c] + dq[parent(v)][c] / 8) * (act > 0)); Lf: fine level
__global__ void k_skip_pool_mask(Lvl Lf, const float* __restrict__ src, int sstride, int soff, const float* __restrict__ dq,
                                 int C, const uint16_t* __restrict__ act, int astride, int aoff, uint16_t* __restrict__ dst)
{
    const long long total = Lf.n * C;
    const int cnx = Lf.nx / 2, cny = Lf.ny / 2;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long v = e / C;
        const int c = (int)(e % C);
        int x, y, z;
        cell_xyz(Lf, v, x, y, z);
        const long long pv = ((long long)(z / 2) * cny + y / 2) * cnx + x / 2;
        const float g = src[v * sstride + soff + c] + dq[pv * C + c] * 0.125f;
        const bool on = bf2f(act[v * astride + aoff + c]) > 0.f;
        dst[e] = f2bf(on ? g : 0.f);
    }
}

// ---- output, loss, optimiser -------------------------------------------------------------

__global__ void k_guess(const double* __restrict__ p_prev, const float* __restrict__ y, long long n,
                        const double* __restrict__ sc, double* __restrict__ out)
{
    const double s = sc[1];
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x)
        out[v] = p_prev[v] + s * (double)y[v];
}

// target t = (p_next - p_prev)/s; gY[v] = (bf16(2 (y - t)/n), 0 x 15); partial sums of (y - t)^2
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const double* __restrict__ p_prev,
                                              const double* __restrict__ p_next, long long n,
                                              const double* __restrict__ sc, uint16_t* __restrict__ gY,
                                              double* __restrict__ part)
{
    __shared__ double lds[8];
    const double s = sc[1];
    double a = 0.0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < n; v += (long long)gridDim.x * blockDim.x) {
        const double t = (p_next[v] - p_prev[v]) / s;
        const double d = (double)y[v] - t;
        a += d * d;
        uint16_t* o = gY + v * 16;
        o[0] = f2bf((float)(2.0 * d / (double)n));
#pragma unroll
        for (int c = 1; c < 16; ++c) o[c] = 0;
    }
    a = block_sum(a, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, long long n, double* __restrict__ sc)
{
    __shared__ double lds[8];
    double a = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) a += part[b];
    a = block_sum(a, lds);
    if (threadIdx.x == 0) sc[2] = a / (double)n;
}

// Adam (Kingma and Ba) with bias correction folded into lr_t and eps_t
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long long n, float lr_t, float eps_t, float b1, float b2)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr_t * mi / (sqrtf(vi) + eps_t);
    }
}

// Wb[t][co][ci] = bf16(W[t][co][ci]);  Wt[t][ci][co] = bf16(W[26 - t][co][ci])
__global__ void k_convert(const float* __restrict__ W, int cout, int cin, uint16_t* __restrict__ Wb, uint16_t* __restrict__ Wt)
{
    const long long total = 27LL * cout * cin;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int t = (int)(e / ((long long)cout * cin));
        const int co = (int)((e / cin) % cout), ci = (int)(e % cin);
        const uint16_t h = f2bf(W[e]);
        Wb[e] = h;
        Wt[((long long)(26 - t) * cin + ci) * cout + co] = h;
    }
}

// counter-based uniform in [-lim, lim] for logical entries, 0 for padding
__global__ void k_init(float* __restrict__ W, int cout, int cin, int cout_l, int cin_l, float lim, unsigned long long seed)
{
    const long long total = 27LL * cout * cin;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int co = (int)((e / cin) % cout), ci = (int)(e % cin);
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(e + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const float u = (float)((z >> 40) * (1.0 / 16777216.0));  // [0, 1)
        W[e] = (co < cout_l && ci < cin_l) ? lim * (2.f * u - 1.f) : 0.f;
    }
}

int g1(long long n) { return (int)std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256)); }

}  // namespace

// =====================================================================================

bool NetModel::grid_ok(int nx, int ny, int nz)
{
    return nx % 4 == 0 && ny % 4 == 0 && nz % 4 == 0 && nx >= 4 && ny >= 4 && nz >= 4;
}

namespace {
struct Sizes {
    long long v1, v2, v4, nparam, nwb, nwf;
    size_t off[40];
    size_t total;
};

const int kCin[6] = {16, 16, 32, 96, 48, 16};
const int kCout[6] = {16, 32, 64, 32, 16, 16};
const int kCinL[6] = {2, 16, 32, 96, 48, 16};
const int kCoutL[6] = {16, 32, 64, 32, 16, 1};
const int kLevel[6] = {0, 1, 2, 1, 0, 0};
// input channels the plane-marching kernel reads (the first layer's two
// logical channels sit in a group of 8)
const int kCinEff[6] = {8, 16, 32, 96, 48, 16};
int frag_chunks(int l) { return (9 * kCinEff[l] + 31) / 32; }
long long frag_elems(int l) { return (long long)(kCout[l] / 16) * 3 * frag_chunks(l) * 64 * 8; }
constexpr long long kWpartFloats = 16LL * 1024 * 1024;  // weight-gradient partial sums (64 MiB)

Sizes sizes(int nx, int ny, int nz, bool training)
{
    Sizes S{};
    S.v1 = (long long)nx * ny * nz;
    S.v2 = S.v1 / 8;
    S.v4 = S.v1 / 64;
    S.nparam = 0;
    S.nwb = 0;
    S.nwf = 0;
    for (int l = 0; l < 6; ++l) {
        S.nparam += 27LL * kCin[l] * kCout[l] + kCout[l];
        S.nwb += 27LL * kCin[l] * kCout[l];
        S.nwf += frag_elems(l);
    }
    size_t o = 0;
    int k = 0;
    auto take = [&](size_t bytes) {
        S.off[k++] = o;
        o = (o + bytes + 255) / 256 * 256;
    };
    take(S.nparam * 4);  // 0 P
    take(S.nparam * 4);  // 1 G
    take(S.nparam * 4);  // 2 M
    take(S.nparam * 4);  // 3 V
    take(S.nwb * 2);     // 4 Wb
    take(S.nwb * 2);     // 5 Wt
    take(S.v1 * 16 * 2); // 6 X
    take(S.v1 * 48 * 2); // 7 C1
    take(S.v1 * 16 * 2); // 8 D1
    take(S.v2 * 16 * 2); // 9 Q1
    take(S.v2 * 96 * 2); // 10 C2
    take(S.v2 * 32 * 2); // 11 D2
    take(S.v4 * 32 * 2); // 12 Q2
    take(S.v4 * 64 * 2); // 13 E3
    take(S.v1 * 4);      // 14 Y
    take(2 * kRedBlocks * 8);  // 15 reduction partials
    take(64 * 8);        // 16 scalars
    take(S.nwf * 2);     // 17 fragment-ordered BF16 weights
    if (training) {
        take(S.v1 * 16 * 2);  // 18 gY
        take(S.v1 * 16 * 4);  // 19 dD1
        take(S.v1 * 16 * 2);  // 20 gD1
        take(S.v1 * 48 * 4);  // 21 dC1
        take(S.v2 * 32 * 2);  // 22 gD2
        take(S.v2 * 96 * 4);  // 23 dC2
        take(S.v4 * 64 * 2);  // 24 gE3
        take(S.v4 * 32 * 4);  // 25 dQ2
        take(S.v2 * 32 * 2);  // 26 gE2
        take(S.v2 * 16 * 4);  // 27 dQ1
        take(S.v1 * 16 * 2);  // 28 gE1
        take(kWpartFloats * 4);  // 29 weight partials
    }
    S.total = o;
    return S;
}
}  // namespace

size_t NetModel::workspace_bytes(int nx, int ny, int nz, bool training)
{
    if (!grid_ok(nx, ny, nz)) return 0;
    return sizes(nx, ny, nz, training).total;
}

NetModel::NetModel(int nx, int ny, int nz, double idx2, double idy2, double idz2, bool training, void* ws,
                   hipStream_t s)
    : D_(2.0 * (idx2 + idy2 + idz2)), idx2_(idx2), idy2_(idy2), idz2_(idz2), training_(training), s_(s)
{
    const Sizes S = sizes(nx, ny, nz, training);
    for (int l = 0; l < 3; ++l) {
        nx_[l] = nx >> l;
        ny_[l] = ny >> l;
        nz_[l] = nz >> l;
        nv_[l] = (long long)nx_[l] * ny_[l] * nz_[l];
    }
    long long wo = 0, bo = 0;
    for (int l = 0; l < kLayers; ++l) {
        L_[l].cin = kCin[l];
        L_[l].cout = kCout[l];
        L_[l].cin_logical = kCinL[l];
        L_[l].cout_logical = kCoutL[l];
        L_[l].level = kLevel[l];
        L_[l].w_off = wo;
        wo += 27LL * kCin[l] * kCout[l];
        L_[l].b_off = wo;
        wo += kCout[l];
        L_[l].wb_off = bo;
        bo += 27LL * kCin[l] * kCout[l];
    }
    nparam_ = S.nparam;
    nwb_ = S.nwb;
    char* b = static_cast<char*>(ws);
    P_ = (float*)(b + S.off[0]);
    G_ = (float*)(b + S.off[1]);
    M_ = (float*)(b + S.off[2]);
    V_ = (float*)(b + S.off[3]);
    Wb_ = (uint16_t*)(b + S.off[4]);
    Wt_ = (uint16_t*)(b + S.off[5]);
    X_ = (uint16_t*)(b + S.off[6]);
    C1_ = (uint16_t*)(b + S.off[7]);
    D1_ = (uint16_t*)(b + S.off[8]);
    Q1_ = (uint16_t*)(b + S.off[9]);
    C2_ = (uint16_t*)(b + S.off[10]);
    D2_ = (uint16_t*)(b + S.off[11]);
    Q2_ = (uint16_t*)(b + S.off[12]);
    E3_ = (uint16_t*)(b + S.off[13]);
    Y_ = (float*)(b + S.off[14]);
    red_ = (double*)(b + S.off[15]);
    sc_ = (double*)(b + S.off[16]);
    Wf_ = (uint16_t*)(b + S.off[17]);
    {
        long long fo = 0;
        for (int l = 0; l < kLayers; ++l) {
            wf_off_[l] = fo;
            fo += frag_elems(l);
        }
    }
    if (training) {
        gY_ = (uint16_t*)(b + S.off[18]);
        dD1_ = (float*)(b + S.off[19]);
        gD1_ = (uint16_t*)(b + S.off[20]);
        dC1_ = (float*)(b + S.off[21]);
        gD2_ = (uint16_t*)(b + S.off[22]);
        dC2_ = (float*)(b + S.off[23]);
        gE3_ = (uint16_t*)(b + S.off[24]);
        dQ2_ = (float*)(b + S.off[25]);
        gE2_ = (uint16_t*)(b + S.off[26]);
        dQ1_ = (float*)(b + S.off[27]);
        gE1_ = (uint16_t*)(b + S.off[28]);
        wpart_ = (float*)(b + S.off[29]);
        wpart_floats_ = kWpartFloats;
    }
}

hipError_t NetModel::init_params(uint64_t seed)
{
    for (int l = 0; l < kLayers; ++l) {
        const NetLayer& ly = L_[l];
        const float lim = (float)std::sqrt(6.0 / (27.0 * ly.cin_logical));
        hipLaunchKernelGGL(k_init, dim3(g1(27LL * ly.cin * ly.cout)), dim3(256), 0, s_, P_ + ly.w_off, ly.cout, ly.cin,
                           ly.cout_logical, ly.cin_logical, lim, (unsigned long long)(seed * 1000003ull + l));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = hipMemsetAsync(P_ + ly.b_off, 0, ly.cout * sizeof(float), s_);
        if (e != hipSuccess) return e;
    }
    return sync();
}

hipError_t NetModel::convert_weights()
{
    for (int l = 0; l < kLayers; ++l) {
        const NetLayer& ly = L_[l];
        hipLaunchKernelGGL(k_convert, dim3(g1(27LL * ly.cin * ly.cout)), dim3(256), 0, s_, P_ + ly.w_off, ly.cout, ly.cin,
                           Wb_ + ly.wb_off, Wt_ + ly.wb_off);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_pack_frag, dim3(g1(frag_elems(l))), dim3(256), 0, s_, Wb_ + ly.wb_off, ly.cout, ly.cin,
                           kCinEff[l], frag_chunks(l), Wf_ + wf_off_[l]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t NetModel::sync()
{
    adam_t_ = 0;
    hipError_t e;
    if (training_) {
        if ((e = hipMemsetAsync(M_, 0, nparam_ * sizeof(float), s_)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(V_, 0, nparam_ * sizeof(float), s_)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(G_, 0, nparam_ * sizeof(float), s_)) != hipSuccess) return e;
    }
    return convert_weights();
}

hipError_t NetModel::normalise(const double* b, const double* p_prev)
{
    const long long n = nv_[0];
    const LapGeo G{nx_[0], ny_[0], nz_[0], idx2_, idy2_, idz2_};
    hipLaunchKernelGGL(k_sum_p, dim3(kRedBlocks), dim3(256), 0, s_, p_prev, n, red_);
    hipLaunchKernelGGL(k_mean_from, dim3(1), dim3(256), 0, s_, red_, n, sc_);
    hipLaunchKernelGGL(k_sumsq_pr, dim3(kRedBlocks), dim3(256), 0, s_, G, p_prev, b, n, 1.0 / D_, sc_, red_);
    hipLaunchKernelGGL(k_scale_from, dim3(1), dim3(256), 0, s_, red_, n, sc_);
    hipLaunchKernelGGL(k_normalise, dim3(g1(n)), dim3(256), 0, s_, G, b, p_prev, n, 1.0 / D_, sc_, X_, xstride());
    return hipGetLastError();
}

#define NCHK(x)                              \
    do {                                     \
        hipError_t e_ = (x);                 \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

hipError_t NetModel::forward()
{
    const Lvl l0{nx_[0], ny_[0], nz_[0], nv_[0]}, l1{nx_[1], ny_[1], nz_[1], nv_[1]}, l2{nx_[2], ny_[2], nz_[2], nv_[2]};
    const float* P = P_;
    auto view = [&](const uint16_t* p, int stride, int off, int lvl) {
        return SrcView{p, stride, off, nx_[lvl], ny_[lvl], nz_[lvl]};
    };
    const SrcView none{};
    // Training keeps the skip tensors e1, e2 inside the concatenated inputs of
    // conv5 and conv4 (C1 = [up d2 | e1], C2 = [up e3 | e2]) for the weight
    // gradients; inference stores them densely, so that their rows are whole
    // cache lines.
    const int c1s = training_ ? 48 : 16, c1o = training_ ? 32 : 0;
    const int c2s = training_ ? 96 : 32, c2o = training_ ? 64 : 0;
    // e1 = relu(conv1(x)) and its 2 x 2 x 2 mean into Q1
    NCHK((conv_march<8, 8, false, 8, OUT_POOL>(l0, view(X_, xstride(), 0, 0), none, Wf_ + wf_off_[0], 1,
                                                 P + L_[0].b_off, C1_, c1s, c1o, 1, s_, Q1_, 16)));
    // e2 = relu(conv2(pool e1)) and its mean into Q2
    NCHK((conv_march<16, 16, false, 8, OUT_POOL>(l1, view(Q1_, 16, 0, 1), none, Wf_ + wf_off_[1], 2, P + L_[1].b_off,
                                                   C2_, c2s, c2o, 1, s_, Q2_, 32)));
    // e3 = relu(conv3(pool e2))
    NCHK((conv_march<32, 32, false, 8, OUT_BF16>(l2, view(Q2_, 32, 0, 2), none, Wf_ + wf_off_[2], 4, P + L_[2].b_off,
                                                   E3_, 64, 0, 1, s_)));
    // d2 = relu(conv4([up e3, e2])); the upsampling is read directly from e3.
    // Training keeps the concatenated tensor for the weight gradient.
    if (training_) {
        hipLaunchKernelGGL(k_up, dim3(g1(l1.n * 64)), dim3(256), 0, s_, l1, E3_, 64, C2_, 96, 0);
        NCHK(hipGetLastError());
    }
    NCHK((conv_march<96, 64, true, 4, OUT_BF16>(l1, view(E3_, 64, 0, 2), view(C2_, c2s, c2o, 1), Wf_ + wf_off_[3], 2,
                                                  P + L_[3].b_off, D2_, 32, 0, 1, s_)));
    // d1 = relu(conv5([up d2, e1]))
    if (training_) {
        hipLaunchKernelGGL(k_up, dim3(g1(l0.n * 32)), dim3(256), 0, s_, l0, D2_, 32, C1_, 48, 0);
        NCHK(hipGetLastError());
    }
    NCHK((conv_march<48, 32, true, 8, OUT_BF16>(l0, view(D2_, 32, 0, 1), view(C1_, c1s, c1o, 0), Wf_ + wf_off_[4], 1,
                                                  P + L_[4].b_off, D1_, 16, 0, 1, s_)));
    // y = conv6(d1)
    NCHK((conv_march<16, 16, false, 8, OUT_HEAD>(l0, view(D1_, 16, 0, 0), none, Wf_ + wf_off_[5], 1, P + L_[5].b_off,
                                                   Y_, 1, 0, 0, s_)));
    return hipSuccess;
}

hipError_t NetModel::predict(const double* b, const double* p_prev, double* p_guess)
{
    NCHK(normalise(b, p_prev));
    NCHK(forward());
    hipLaunchKernelGGL(k_guess, dim3(g1(nv_[0])), dim3(256), 0, s_, p_prev, Y_, nv_[0], sc_, p_guess);
    return hipGetLastError();
}

hipError_t NetModel::backward()
{
    const Lvl l0{nx_[0], ny_[0], nz_[0], nv_[0]}, l1{nx_[1], ny_[1], nz_[1], nv_[1]}, l2{nx_[2], ny_[2], nz_[2], nv_[2]};
    float* part = wpart_;
    const long long pf = wpart_floats_;
    auto bgrad = [&](const uint16_t* dout, long long n, int C, float* g) -> hipError_t {
        const int nblk = (int)std::min<long long>(1024, std::max<long long>(1, n / 256));
        hipLaunchKernelGGL(k_bgrad_part, dim3(nblk), dim3(256), 0, s_, dout, n, C, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bgrad_reduce, dim3(1), dim3(128), 0, s_, part, nblk, C, g);
        return hipGetLastError();
    };
    // head
    NCHK((conv<16, 16, OUT_F32>(l0, gY_, Wt_ + L_[5].wb_off, nullptr, dD1_, 16, 0, 0, s_)));
    NCHK((wgrad<16, 16>(l0, D1_, gY_, part, pf, G_ + L_[5].w_off, s_)));
    NCHK(bgrad(gY_, l0.n, 16, G_ + L_[5].b_off));
    hipLaunchKernelGGL(k_mask_round, dim3(g1(l0.n * 16)), dim3(256), 0, s_, l0.n, 16, dD1_, D1_, 16, 0, gD1_);
    NCHK(hipGetLastError());
    // conv5: input C1 (48), dout gD1 (16)
    NCHK((conv<16, 48, OUT_F32>(l0, gD1_, Wt_ + L_[4].wb_off, nullptr, dC1_, 48, 0, 0, s_)));
    NCHK((wgrad<48, 16>(l0, C1_, gD1_, part, pf, G_ + L_[4].w_off, s_)));
    NCHK(bgrad(gD1_, l0.n, 16, G_ + L_[4].b_off));
    hipLaunchKernelGGL(k_upbwd_mask, dim3(g1(l1.n * 32)), dim3(256), 0, s_, l1, dC1_, 48, 0, 32, D2_, 32, 0, gD2_);
    NCHK(hipGetLastError());
    // conv4: input C2 (96), dout gD2 (32)
    NCHK((conv<32, 96, OUT_F32>(l1, gD2_, Wt_ + L_[3].wb_off, nullptr, dC2_, 96, 0, 0, s_)));
    NCHK((wgrad<96, 32>(l1, C2_, gD2_, part, pf, G_ + L_[3].w_off, s_)));
    NCHK(bgrad(gD2_, l1.n, 32, G_ + L_[3].b_off));
    hipLaunchKernelGGL(k_upbwd_mask, dim3(g1(l2.n * 64)), dim3(256), 0, s_, l2, dC2_, 96, 0, 64, E3_, 64, 0, gE3_);
    NCHK(hipGetLastError());
    // conv3: input Q2 (32), dout gE3 (64)
    NCHK((conv<64, 32, OUT_F32>(l2, gE3_, Wt_ + L_[2].wb_off, nullptr, dQ2_, 32, 0, 0, s_)));
    NCHK((wgrad<32, 64>(l2, Q2_, gE3_, part, pf, G_ + L_[2].w_off, s_)));
    NCHK(bgrad(gE3_, l2.n, 64, G_ + L_[2].b_off));
    hipLaunchKernelGGL(k_skip_pool_mask, dim3(g1(l1.n * 32)), dim3(256), 0, s_, l1, dC2_, 96, 64, dQ2_, 32, C2_, 96, 64,
                       gE2_);
    NCHK(hipGetLastError());
    // conv2: input Q1 (16), dout gE2 (32)
    NCHK((conv<32, 16, OUT_F32>(l1, gE2_, Wt_ + L_[1].wb_off, nullptr, dQ1_, 16, 0, 0, s_)));
    NCHK((wgrad<16, 32>(l1, Q1_, gE2_, part, pf, G_ + L_[1].w_off, s_)));
    NCHK(bgrad(gE2_, l1.n, 32, G_ + L_[1].b_off));
    hipLaunchKernelGGL(k_skip_pool_mask, dim3(g1(l0.n * 16)), dim3(256), 0, s_, l0, dC1_, 48, 32, dQ1_, 16, C1_, 48, 32,
                       gE1_);
    NCHK(hipGetLastError());
    // conv1: input X (16), dout gE1 (16); no input gradient needed
    NCHK((wgrad<16, 16>(l0, X_, gE1_, part, pf, G_ + L_[0].w_off, s_)));
    NCHK(bgrad(gE1_, l0.n, 16, G_ + L_[0].b_off));
    return hipSuccess;
}

hipError_t NetModel::train_step(const double* b, const double* p_prev, const double* p_next, float lr, double* loss_dev)
{
    if (!training_) return hipErrorInvalidValue;
    NCHK(normalise(b, p_prev));
    NCHK(forward());
    hipLaunchKernelGGL(k_loss, dim3(kRedBlocks), dim3(256), 0, s_, Y_, p_prev, p_next, nv_[0], sc_, gY_, red_);
    NCHK(hipGetLastError());
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s_, red_, nv_[0], sc_);
    NCHK(hipGetLastError());
    NCHK(backward());
    if (lr > 0.f) {
        ++adam_t_;
        const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
        const double c1 = 1.0 - std::pow(b1, adam_t_), c2 = 1.0 - std::pow(b2, adam_t_);
        // lr * (m/c1) / (sqrt(v/c2) + eps) = (lr sqrt(c2)/c1) m / (sqrt(v) + eps sqrt(c2))
        const float lr_t = (float)(lr * std::sqrt(c2) / c1), eps_t = (float)(eps * std::sqrt(c2));
        hipLaunchKernelGGL(k_adam, dim3(g1(nparam_)), dim3(256), 0, s_, P_, G_, M_, V_, nparam_, lr_t, eps_t, (float)b1,
                           (float)b2);
        NCHK(hipGetLastError());
        NCHK(convert_weights());
    }
    if (loss_dev) NCHK(hipMemcpyAsync(loss_dev, sc_ + 2, sizeof(double), hipMemcpyDeviceToDevice, s_));
    return hipSuccess;
}

}  // namespace stp
