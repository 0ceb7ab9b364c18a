// Learned warm start: the encoder-decoder network of ep_net.h, its forward
// and backward passes and Adam, all in HIP kernels on the gfx950 matrix
// cores (bfloat16 operands, FP32 accumulation).
//
// Tensors of the network are channel-last over the network volume with a
// one-voxel zero border (the padding of the 3x3x3 'same' convolutions):
// voxel (z, y, x) of a D x H x W level is stored at ((z+1)(H+2) + y+1)(W+2)
// + x+1, times the channel count.  Borders are zeroed once and never written.
//
// Convolution = implicit GEMM: rows are voxels, columns output channels,
// the reduction runs over 27 taps x input channels.  One wave computes 64
// voxels (4 MFMA row blocks of 16) x all output channels with
// v_mfma_f32_16x16x32_bf16: the A operand of a lane is 8 consecutive input
// channels of one voxel (read from an LDS copy of the block's input with
// halo), the B operand 8 consecutive input channels of one output channel's
// weights (the 16-channel input layer uses the K = 16 form).  The gradient with respect to
// the input is the same kernel on the output gradient with the weights
// transposed (input <-> output channels) and the taps mirrored.  The weight
// gradient reduces over voxels: a workgroup stages 64 voxels of the output
// gradient and of the tap-shifted input in LDS and accumulates 16 x 16
// blocks with the voxels as the MFMA reduction dimension, then adds its
// partial sums to the FP32 gradient with atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "ep.h"
#include "ep_handle.h"
#include "ep_internal.h"
#include "ep_net.h"

using namespace ep;

namespace {

typedef unsigned short bf16_t;
typedef __attribute__((ext_vector_type(4))) short s4;
typedef __attribute__((ext_vector_type(8))) __bf16 b8;
typedef __attribute__((ext_vector_type(4))) float f4;

// 8 bfloat16 values (16 bytes) as the operand of a K = 32 MFMA
__device__ __forceinline__ b8 ld_b8(const bf16_t* p) { return __builtin_bit_cast(b8, *(const uint4*)p); }

constexpr int NL = 11;      // convolutions
constexpr int CIN0 = 16;    // input channels (11 used)
constexpr int COUT = 16;    // output channels (3 used)
constexpr long PART_FLOATS = 1L << 23;   // partial-sum buffer of the parameter gradients (32 MiB)

// ------------------------------------------------------------ bfloat16
__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float((unsigned)b << 16); }
// round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ bf16_t f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
bf16_t host_f2bf(float f)
{
    unsigned u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
float host_bf2f(bf16_t b)
{
    unsigned u = (unsigned)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// ------------------------------------------------------------ geometry
struct Vol {
    int D, H, W;      // interior
    int Hp, Wp;       // padded
    long V;           // interior voxels
    long Vp;          // padded voxels
};

Vol make_vol(int D, int H, int W)
{
    Vol g;
    g.D = D; g.H = H; g.W = W;
    g.Hp = H + 2; g.Wp = W + 2;
    g.V = (long)D * H * W;
    g.Vp = (long)(D + 2) * (H + 2) * (W + 2);
    return g;
}

__device__ __forceinline__ long pidx(const Vol& g, long v)
{
    const int x = (int)(v % g.W);
    const long r = v / g.W;
    const int y = (int)(r % g.H);
    const int z = (int)(r / g.H);
    return ((long)(z + 1) * g.Hp + (y + 1)) * g.Wp + (x + 1);
}

__device__ __forceinline__ long tap_off(const Vol& g, int t)
{
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    return ((long)dz * g.Hp + dy) * g.Wp + dx;
}

// ------------------------------------------------------------ convolution
enum { EPI_RELU = 0, EPI_LIN = 1, EPI_MASK = 2, EPI_F32 = 3 };

// Y[v][c] = epilogue(b[c] + sum_t sum_i X[v + off_t][i] W[c][t][i]) for the
// NB*16 output channels.  EPI_F32 writes an unpadded FP32 [V][16] array.
// A workgroup computes a 4 (z) x 4 (y) x 16 (x) block of output voxels; wave w
// takes the z-slice w, its 4 MFMA row blocks are the 4 y-rows of 16 voxels.
// The input block with its one-voxel halo (6 x 6 x 18 voxels) is staged in
// LDS 32 input channels at a time (rows of 40 bf16: 16-byte aligned, and 16
// lanes reading 16 consecutive voxels hit distinct banks) and serves all 27
// taps; the weights come through the L1/L2 caches.
constexpr int CB_X = 16, CB_Y = 4, CB_Z = 4;
constexpr int CT_X = CB_X + 2, CT_Y = CB_Y + 2, CT_Z = CB_Z + 2, CT_N = CT_X * CT_Y * CT_Z;
constexpr int CT_ROW = 40;

template <int NB, int EPI>
__global__ __launch_bounds__(256) void k_conv(const bf16_t* __restrict__ X, int cin, const bf16_t* __restrict__ Wt,
                                              const float* __restrict__ bias, void* __restrict__ Y,
                                              const bf16_t* __restrict__ M, Vol g)
{
    constexpr int CO = NB * 16;
    __shared__ __attribute__((aligned(16))) bf16_t tile[CT_N * CT_ROW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int x0 = blockIdx.x * CB_X, y0 = blockIdx.y * CB_Y, z0 = blockIdx.z * CB_Z;
    f4 acc[4][NB];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < cin; c0 += 32) {
        const int kc = cin - c0 < 32 ? cin - c0 : 32;    // 16 or 32 channels in this chunk
        const int nq = kc / 8;                            // 16-byte pieces per voxel
        __syncthreads();
        for (int e = threadIdx.x; e < CT_N * nq; e += 256) {
            const int tv = e / nq, q = e % nq;
            const int tx = tv % CT_X, ty = (tv / CT_X) % CT_Y, tz = tv / (CT_X * CT_Y);
            // padded coordinates of the tile voxel (the halo starts at the border)
            const int px = x0 + tx, py = y0 + ty, pz = z0 + tz;
            uint4 val = {0u, 0u, 0u, 0u};
            if (px < g.Wp && py < g.Hp && pz < g.D + 2)
                val = *(const uint4*)(X + (((long)pz * g.Hp + py) * g.Wp + px) * cin + c0 + q * 8);
            *(uint4*)(tile + tv * CT_ROW + q * 8) = val;
        }
        __syncthreads();
        if (kc == 32) {
            // K = 32: lane (r, kq) holds channels kq*8 .. kq*8+7 of voxel row r
            // (A) and of output channel r (B); A and B share the lane-to-
            // channel map, so the reduction covers the 32 channels whatever
            // order the matrix core takes them in
            // the weights of tap t+1 are loaded while tap t computes
            const bf16_t* wl = Wt + (long)r * 27 * cin + c0 + kq * 8;
            const long wstep = 16L * 27 * cin;                   // next output-channel block
            b8 bw[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bw[nb] = ld_b8(wl + nb * wstep);
            for (int t = 0; t < 27; ++t) {
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;     // 0..2: tap offset + 1
                b8 bn[NB];
                const int tn = t + 1 < 27 ? t + 1 : t;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) bn[nb] = ld_b8(wl + nb * wstep + (long)tn * cin);
                b8 a[4];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) {
                    const int tv = ((wave + dz) * CT_Y + (mb + dy)) * CT_X + (r + dx);
                    a[mb] = ld_b8(tile + tv * CT_ROW + kq * 8);
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], bw[nb], acc[mb][nb], 0, 0, 0);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) bw[nb] = bn[nb];
            }
        } else {
            // a 16-channel chunk (the 16-channel input layer): K = 16
            for (int t = 0; t < 27; ++t) {
                const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
                s4 a[4];
#pragma unroll
                for (int mb = 0; mb < 4; ++mb) {
                    const int tv = ((wave + dz) * CT_Y + (mb + dy)) * CT_X + (r + dx);
                    a[mb] = *(const s4*)(tile + tv * CT_ROW + kq * 4);
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const s4 bw = *(const s4*)(Wt + ((long)(nb * 16 + r) * 27 + t) * cin + c0 + kq * 4);
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mb], bw, acc[mb][nb], 0, 0, 0);
                }
            }
        }
    }
    // lane holds rows kq*4 + i (x within the row block) of column r (output channel)
    const int z = z0 + wave;
    if (z >= g.D) return;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        const int y = y0 + mb;
        if (y >= g.H) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = x0 + kq * 4 + i;
            if (x >= g.W) continue;
            const long v = ((long)z * g.H + y) * g.W + x;
            const long p = ((long)(z + 1) * g.Hp + (y + 1)) * g.Wp + (x + 1);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int c = nb * 16 + r;
                float zz = acc[mb][nb][i] + (bias ? bias[c] : 0.f);
                if (EPI == EPI_F32) {
                    ((float*)Y)[v * CO + c] = zz;
                } else {
                    if (EPI == EPI_RELU) zz = fmaxf(zz, 0.f);
                    if (EPI == EPI_MASK) zz = bf2f(M[p * CO + c]) > 0.f ? zz : 0.f;
                    ((bf16_t*)Y)[p * CO + c] = f2bf(zz);
                }
            }
        }
    }
}

// Block index -> logical index so that consecutive logical indices run on
// the same XCD (workgroups are dispatched round-robin over the 8 XCDs).
// Bijective for any nb.
__device__ __forceinline__ int xcd_order(int b, int nb)
{
    const int q = nb / 8, r = nb % 8;
    const int x = b % 8, s = b / 8;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// Channels 0..7 of voxels v (a) and v + 1 (b) to eight channel rows of a
// channel-major LDS stage: row k gets the dword (a_k, b_k) at d + k * rw
// (d at an even voxel index, so every dword is aligned).
__device__ __forceinline__ void stage_pair(bf16_t* d, int rw, const uint4& a, const uint4& b)
{
    const unsigned aw[4] = {a.x, a.y, a.z, a.w}, bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // channel 2k: low halves of a and b; channel 2k + 1: high halves
        *(unsigned*)(d + (2 * k) * rw) = (aw[k] & 0xffffu) | (bw[k] << 16);
        *(unsigned*)(d + (2 * k + 1) * rw) = (aw[k] >> 16) | (bw[k] & 0xffff0000u);
    }
}

// part[chunk][o][t][i] = sum over the chunk's voxels v of G[v][o] X[v + off_t][i],
// one workgroup per (voxel chunk, tap); k_wsum adds the chunks up in a fixed
// order, so a gradient does not depend on the order the workgroups run in.
// The 27 taps of a chunk are consecutive logical workgroups on one XCD, so
// that the chunk's output gradient and the overlapping input windows of its
// taps can be served from that XCD's L2 (no change in time measured: the
// kernel is bound by its LDS staging).
template <int NBO, int NBI, int SL>
__global__ __launch_bounds__(256) void k_wgrad(const bf16_t* __restrict__ X, const bf16_t* __restrict__ G,
                                               float* __restrict__ part, Vol g, long vchunk)
{
    constexpr int CO = NBO * 16, CI = NBI * 16;
    constexpr long E = 27L * CO * CI;                  // entries of one chunk's partial gradient
    constexpr int RW = SL + 8;                         // SL voxels + 8: rows of 144 or 272 bytes
    constexpr int NP = NBO * NBI, PW = (NP + 3) / 4;   // block pairs, per wave
    // channel-major (transposed) stage: a lane's 8 voxels of one channel are
    // one 16-byte LDS read
    __shared__ __attribute__((aligned(16))) bf16_t sG[CO * RW], sX[CI * RW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kq = lane >> 4;
    const int lb = xcd_order(blockIdx.x, gridDim.x);
    const int t = lb % 27, chunk = lb / 27;
    const long off = tap_off(g, t);
    const long v0 = (long)chunk * vchunk;
    const long v1 = v0 + vchunk < g.V ? v0 + vchunk : g.V;
    f4 acc[PW];
#pragma unroll
    for (int q = 0; q < PW; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
    // stage SL voxels: a pair of voxels x 8 channels (two 16-byte loads) per
    // thread and task, loaded into registers one slab ahead and written
    // transposed as 8 dwords (channel k of both voxels); the SL / 2 lanes of
    // a channel group take consecutive pairs, so that a wave's dword writes
    // fall in distinct LDS banks
    constexpr int NPR = SL / 2;                        // voxel pairs per slab
    constexpr int NGT = NPR * (CO / 8), NXT = NPR * (CI / 8);
    constexpr int NGL = (NGT + 255) / 256, NXL = (NXT + 255) / 256;
    uint4 ga[NGL], gb[NGL], xa[NXL], xb[NXL];
    auto load = [&](long vs) {
#pragma unroll
        for (int u = 0; u < NGL; ++u) {
            const int e = threadIdx.x + 256 * u, row = 2 * (e % NPR), q = e / NPR;
            const long v = vs + row;
            ga[u] = uint4{0u, 0u, 0u, 0u};
            gb[u] = uint4{0u, 0u, 0u, 0u};
            if (e < NGT && v < v1) ga[u] = *(const uint4*)(G + pidx(g, v) * CO + q * 8);
            if (e < NGT && v + 1 < v1) gb[u] = *(const uint4*)(G + pidx(g, v + 1) * CO + q * 8);
        }
#pragma unroll
        for (int u = 0; u < NXL; ++u) {
            const int e = threadIdx.x + 256 * u, row = 2 * (e % NPR), q = e / NPR;
            const long v = vs + row;
            xa[u] = uint4{0u, 0u, 0u, 0u};
            xb[u] = uint4{0u, 0u, 0u, 0u};
            if (e < NXT && v < v1) xa[u] = *(const uint4*)(X + (pidx(g, v) + off) * CI + q * 8);
            if (e < NXT && v + 1 < v1) xb[u] = *(const uint4*)(X + (pidx(g, v + 1) + off) * CI + q * 8);
        }
    };
    if (v0 < v1) load(v0);
    for (long vs = v0; vs < v1; vs += SL) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NGL; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < NGT) stage_pair(sG + (e / NPR) * 8 * RW + 2 * (e % NPR), RW, ga[u], gb[u]);
        }
#pragma unroll
        for (int u = 0; u < NXL; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < NXT) stage_pair(sX + (e / NPR) * 8 * RW + 2 * (e % NPR), RW, xa[u], xb[u]);
        }
        __syncthreads();
        if (vs + SL < v1) load(vs + SL);
#pragma unroll
        for (int q = 0; q < PW; ++q) {
            const int pr = wave + 4 * q;
            if (pr >= NP) break;
            const int ob = pr / NBI, ib = pr % NBI;
#pragma unroll
            for (int ks = 0; ks < SL / 32; ++ks) {
                // K = 32 voxels: lane (r, kq) holds voxels ks*32 + kq*8 .. +7 of
                // output channel ob*16 + r (A) and input channel ib*16 + r (B)
                const b8 a = ld_b8(sG + (ob * 16 + r) * RW + ks * 32 + kq * 8);
                const b8 b = ld_b8(sX + (ib * 16 + r) * RW + ks * 32 + kq * 8);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PW; ++q) {
        const int pr = wave + 4 * q;
        if (pr >= NP) break;
        const int ob = pr / NBI, ib = pr % NBI;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = ob * 16 + kq * 4 + i, c = ib * 16 + r;
            part[chunk * E + ((long)o * 27 + t) * CI + c] = acc[q][i];
        }
    }
}

// dW[e] += sum over chunks of part[chunk][e], in chunk order: thread (j, e)
// of a 256-thread block (32 entries x 8) sums chunks j, j + 8, ..., then the
// eight sums are added in j order.
__global__ __launch_bounds__(256) void k_wsum(const float* __restrict__ part, long nch, long E, float* __restrict__ dW)
{
    __shared__ float s[8][32];
    const int el = threadIdx.x & 31, jl = threadIdx.x >> 5;
    const long e = (long)blockIdx.x * 32 + el;
    float acc = 0.f;
    if (e < E)
        for (long c = jl; c < nch; c += 8) acc += part[c * E + e];
    s[jl][el] = acc;
    __syncthreads();
    if (jl == 0 && e < E) {
        float sum = s[0][el];
        for (int j = 1; j < 8; ++j) sum += s[j][el];
        dW[e] += sum;
    }
}

// part[block][c] = sum over the block's voxels of G[v][c] (k_bsum adds the
// blocks up in a fixed order)
__global__ void k_bias_grad(const bf16_t* __restrict__ G, int C, float* __restrict__ part, Vol g)
{
    // thread = (voxel slot, group of 8 channels): 16-byte loads, a block
    // covers 256 / (C / 8) voxels per step (C in {16, 32, 64, 128})
    __shared__ float s[256 * 8];
    const int ng = C / 8, grp = threadIdx.x % ng, vq = threadIdx.x / ng, nv = 256 / ng;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (long v = (long)blockIdx.x * nv + vq; v < g.V; v += (long)gridDim.x * nv) {
        const uint4 val = *(const uint4*)(G + pidx(g, v) * C + grp * 8);
        const bf16_t* h = (const bf16_t*)&val;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] += bf2f(h[k]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) s[threadIdx.x * 8 + k] = acc[k];
    __syncthreads();
    if (threadIdx.x < C) {
        const int gq = threadIdx.x / 8, k = threadIdx.x % 8;
        float sum = 0.f;
        for (int q = 0; q < nv; ++q) sum += s[(q * ng + gq) * 8 + k];
        part[(long)blockIdx.x * C + threadIdx.x] = sum;
    }
}

// db[c] += sum over blocks of part[block][c], one workgroup per channel:
// thread j sums blocks j, j + 256, ..., then a tree of fixed shape adds the
// 256 sums.
__global__ __launch_bounds__(256) void k_bsum(const float* __restrict__ part, int nb, int C, float* __restrict__ db)
{
    __shared__ float s[256];
    const int c = blockIdx.x;
    float acc = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) acc += part[(long)b * C + c];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] += s[0];
}

// ------------------------------------------------------------ elementwise
// pool: out (level g2) = mean of the 8 children in level g
__global__ void k_pool(const bf16_t* __restrict__ in, bf16_t* __restrict__ out, int C, Vol g, Vol g2)
{
    // grid-stride: the element count can exceed 2^32 work-items
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g2.V * C; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long v = e / C;
        const int x = (int)(v % g2.W), y = (int)((v / g2.W) % g2.H), z = (int)(v / ((long)g2.W * g2.H));
        float s = 0.f;
        for (int q = 0; q < 8; ++q) {
            const int zz = 2 * z + (q >> 2), yy = 2 * y + ((q >> 1) & 1), xx = 2 * x + (q & 1);
            s += bf2f(in[(((long)(zz + 1) * g.Hp + yy + 1) * g.Wp + xx + 1) * C + c]);
        }
        out[pidx(g2, v) * C + c] = f2bf(s * 0.125f);
    }
}

// up: out (level g) = parent value (level g2)
__global__ void k_up(const bf16_t* __restrict__ in, bf16_t* __restrict__ out, int C, Vol g, Vol g2)
{
    // grid-stride: the element count can exceed 2^32 work-items
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g.V * C; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long v = e / C;
        const int x = (int)(v % g.W), y = (int)((v / g.W) % g.H), z = (int)(v / ((long)g.W * g.H));
        out[pidx(g, v) * C + c] = in[(((long)(z / 2 + 1) * g2.Hp + y / 2 + 1) * g2.Wp + x / 2 + 1) * C + c];
    }
}

// gradient of up: out (level g2) = sum of the 8 children (level g)
__global__ void k_up_dx(const bf16_t* __restrict__ in, bf16_t* __restrict__ out, int C, Vol g, Vol g2)
{
    // grid-stride: the element count can exceed 2^32 work-items
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g2.V * C; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long v = e / C;
        const int x = (int)(v % g2.W), y = (int)((v / g2.W) % g2.H), z = (int)(v / ((long)g2.W * g2.H));
        float s = 0.f;
        for (int q = 0; q < 8; ++q) {
            const int zz = 2 * z + (q >> 2), yy = 2 * y + ((q >> 1) & 1), xx = 2 * x + (q & 1);
            s += bf2f(in[(((long)(zz + 1) * g.Hp + yy + 1) * g.Wp + xx + 1) * C + c]);
        }
        out[pidx(g2, v) * C + c] = f2bf(s);
    }
}

// out (level g) = a + pool gradient of t (level g2): a + t(parent) / 8
__global__ void k_add_pool_dx(const bf16_t* __restrict__ a, const bf16_t* __restrict__ t, bf16_t* __restrict__ out,
                              int C, Vol g, Vol g2)
{
    // grid-stride: the element count can exceed 2^32 work-items
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g.V * C; e += (long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        const long v = e / C;
        const int x = (int)(v % g.W), y = (int)((v / g.W) % g.H), z = (int)(v / ((long)g.W * g.H));
        const long p = pidx(g, v) * C + c;
        const float tv = bf2f(t[(((long)(z / 2 + 1) * g2.Hp + y / 2 + 1) * g2.Wp + x / 2 + 1) * C + c]);
        out[p] = f2bf(bf2f(a[p]) + tv * 0.125f);
    }
}

// out = a + b
__global__ void k_add(const bf16_t* __restrict__ a, const bf16_t* __restrict__ b, bf16_t* __restrict__ out, int C,
                      Vol g)
{
    // grid-stride: the element count can exceed 2^32 work-items
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g.V * C; e += (long)gridDim.x * blockDim.x) {
        const long p = pidx(g, e / C) * C + e % C;
        out[p] = f2bf(bf2f(a[p]) + bf2f(b[p]));
    }
}

// out = a where m > 0, else 0
__global__ void k_mask(const bf16_t* __restrict__ a, const bf16_t* __restrict__ m, bf16_t* __restrict__ out, int C,
                       Vol g)
{
    // grid-stride: the element count can exceed 2^32 work-items
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < g.V * C; e += (long)gridDim.x * blockDim.x) {
        const long p = pidx(g, e / C) * C + e % C;
        out[p] = bf2f(m[p]) > 0.f ? a[p] : (bf16_t)0;
    }
}

// Loss: mean squared error over the interior faces; gy = its gradient.
// Output channel d of voxel (x, y, z) is the lower d-face of that cell; the
// face is interior when its index along d is in 1 .. n_d - 1.
// Output gradient of the loss, and part[block] = the block's share of the
// loss (k_lsum adds the blocks up in a fixed order).
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ tg, bf16_t* __restrict__ gy, Vol g,
                       int nx, int ny, int nz, float inv_n, double* __restrict__ part)
{
    __shared__ float s[256];
    float acc = 0.f;
    for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < g.V; v += (long)gridDim.x * blockDim.x) {
        const int x = (int)(v % g.W), yy = (int)((v / g.W) % g.H), z = (int)(v / ((long)g.W * g.H));
        const bool in = x < nx && yy < ny && z < nz;
        const long p = pidx(g, v);
        for (int c = 0; c < COUT; ++c) {
            bool ok = false;
            if (c == 0) ok = in && x >= 1;
            if (c == 1) ok = in && yy >= 1;
            if (c == 2) ok = in && z >= 1;
            float d = ok ? y[v * COUT + c] - tg[v * 4 + c] : 0.f;
            acc += d * d;
            gy[p * COUT + c] = f2bf(2.f * d * inv_n);
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = (double)s[0] * inv_n;
}

// loss = sum of the nb block shares, thread j taking blocks j, j + 256, ...,
// then a tree of fixed shape (one workgroup of 256 threads)
__global__ __launch_bounds__(256) void k_lsum(const double* __restrict__ part, int nb, double* __restrict__ loss)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0];
}

__global__ void k_fill_f(float* p, float v, long n)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// Adam step on the master parameters; bias corrections c1 = 1 - b1^t,
// c2 = 1 - b2^t.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ vv, long n, float lr, float c1, float c2)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gg = gr[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float v2 = b2 * vv[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    vv[e] = v2;
    w[e] -= lr * (mm / c1) / (sqrtf(v2 / c2) + eps);
}

// bfloat16 copies of one layer's weights: Wb[o][t][i] and the transposed,
// tap-mirrored Wtb[i][26 - t][o] of the input-gradient convolution.
__global__ void k_wcopy(const float* __restrict__ w, bf16_t* __restrict__ wb, bf16_t* __restrict__ wtb, int co, int ci)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)co * 27 * ci) return;
    const int i = (int)(e % ci), t = (int)((e / ci) % 27), o = (int)(e / ((long)ci * 27));
    const bf16_t b = f2bf(w[e]);
    wb[e] = b;
    wtb[((long)i * 27 + (26 - t)) * co + o] = b;
}

// ------------------------------------------------------------ solver side
struct SolverView {
    const double *txx, *tyy, *txy, *txz, *tyz, *p, *epsp;
    const double *vx, *vy, *vz;
    int nx, ny, nz, sy;
    long sz;
};

// Features of the solver state into a padded input tensor (16 channels).
__global__ void k_features(SolverView s, const float* __restrict__ dvp, bf16_t* __restrict__ x, Vol g, float iss,
                           float ise, float isv)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.V) return;
    const int i = (int)(v % g.W), j = (int)((v / g.W) % g.H), k = (int)(v / ((long)g.W * g.H));
    float f[16];
    for (int c = 0; c < 16; ++c) f[c] = 0.f;
    if (i < s.nx && j < s.ny && k < s.nz) {
        const long sy = s.sy, sz = s.sz;
        const long e = i + sy * j + sz * k;
        const double txx = s.txx[e], tyy = s.tyy[e];
        f[0] = (float)(txx * iss);
        f[1] = (float)(tyy * iss);
        f[2] = (float)(-(txx + tyy) * iss);
        f[3] = (float)(0.25 * (s.txy[e] + s.txy[e + 1] + s.txy[e + sy] + s.txy[e + sy + 1]) * iss);
        f[4] = (float)(0.25 * (s.txz[e] + s.txz[e + 1] + s.txz[e + sz] + s.txz[e + sz + 1]) * iss);
        f[5] = (float)(0.25 * (s.tyz[e] + s.tyz[e + sy] + s.tyz[e + sz] + s.tyz[e + sy + sz]) * iss);
        f[6] = (float)(s.p[e] * iss);
        f[7] = (float)(s.epsp[e] * ise);
        f[8] = dvp[v * 4 + 0] * isv;
        f[9] = dvp[v * 4 + 1] * isv;
        f[10] = dvp[v * 4 + 2] * isv;
    }
    const long p = pidx(g, v) * 16;
    for (int c = 0; c < 16; ++c) x[p + c] = f2bf(f[c]);
}

// After an increment: velocity change at the lower faces since the last
// call -> tracked previous change (and a target when tg != null).
__global__ void k_observe(SolverView s, double* __restrict__ vlast, float* __restrict__ dvp, float* __restrict__ tg,
                          Vol g, int first, float iso)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.V) return;
    const int i = (int)(v % g.W), j = (int)((v / g.W) % g.H), k = (int)(v / ((long)g.W * g.H));
    for (int d = 0; d < 3; ++d) {
        float dv = 0.f;
        if (i < s.nx && j < s.ny && k < s.nz) {
            const long e = i + (long)s.sy * j + s.sz * k;
            const double cur = d == 0 ? s.vx[e] : d == 1 ? s.vy[e] : s.vz[e];
            if (!first) dv = (float)(cur - vlast[v * 3 + d]);
            vlast[v * 3 + d] = cur;
        }
        dvp[v * 4 + d] = dv;
        if (tg) tg[v * 4 + d] = dv * iso;
    }
    dvp[v * 4 + 3] = 0.f;
    if (tg) tg[v * 4 + 3] = 0.f;
}

// Guess velocities: current + scale * y at interior faces, current elsewhere.
__global__ void k_apply_guess(SolverView s, const float* __restrict__ y, double* __restrict__ gx,
                              double* __restrict__ gyv, double* __restrict__ gz, Vol g, float so)
{
    const long n = (long)(s.nx + 1) * (s.ny + 1) * (s.nz + 1);
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int i = (int)(q % (s.nx + 1)), j = (int)((q / (s.nx + 1)) % (s.ny + 1)),
              k = (int)(q / ((long)(s.nx + 1) * (s.ny + 1)));
    const long e = i + (long)s.sy * j + s.sz * k;
    auto yv = [&](int c) { return y[(((long)k * g.H + j) * g.W + i) * COUT + c]; };
    if (j < s.ny && k < s.nz) gx[e] = s.vx[e] + ((i >= 1 && i < s.nx) ? (double)(so * yv(0)) : 0.0);
    if (i < s.nx && k < s.nz) gyv[e] = s.vy[e] + ((j >= 1 && j < s.ny) ? (double)(so * yv(1)) : 0.0);
    if (i < s.nx && j < s.ny) gz[e] = s.vz[e] + ((k >= 1 && k < s.nz) ? (double)(so * yv(2)) : 0.0);
}

// blocks for n elements, capped at 2^22 (2^30 work-items, below the 2^32
// limit of a dispatch); kernels whose n can exceed that loop grid-stride
inline unsigned nblk(long n, int t = 256) { return (unsigned)std::min<long>((n + t - 1) / t, 1L << 22); }

}  // namespace

// =========================================================================
struct ep_net {
    ep_net_config cfg;
    hipStream_t st;
    Vol g[3];
    int ch[NL][2];             // (Cin, Cout)
    long woff[NL], boff[NL];   // offsets in the parameter vector
    long wboff[NL];            // offsets in the bf16 weight arrays
    long np, nwb;
    float *w, *gr, *m, *v;     // FP32 masters, gradient, moments
    bf16_t *wb, *wtb;          // bf16 weights and transposed copies
    // activations
    bf16_t *xin, *a0, *s0, *p0, *a1, *s1, *p1, *a2, *b2, *u1, *r6, *c1, *d1, *u0, *r8, *c0, *d0;
    float* y;
    // gradients
    bf16_t *gy, *z9, *gc0, *z8, *t0, *gd1, *z7, *gc1, *z6, *t1, *gb2, *z5, *z4, *t2, *gs1, *z3, *z2, *t3, *gs0, *z1,
        *z0;
    // samples and tracking
    bf16_t* sx;                // max_samples x Vp0 x 16
    float* stg;                // max_samples x V0 x 4
    double* vlast;             // V0 x 3
    float* dvp;                // V0 x 4
    double* loss;
    float* part;               // per-chunk partial sums of the weight and bias gradients (training only)
    bool have_last;
    long adam_t;
    char err[512];
};

namespace {

int nerr(ep_net* n, int code, const char* fmt, ...)
{
    if (n) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(n->err, sizeof(n->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define NCHK(n, x)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess)                                                               \
            return nerr((n), EP_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
    } while (0)

int validate_cfg(const ep_net_config* c)
{
    if (!c) return EP_EINVAL;
    if (c->nx < 4 || c->ny < 4 || c->nz < 4) return EP_EINVAL;
    if (c->base != 16 && c->base != 32) return EP_EINVAL;
    if (c->max_samples < 0) return EP_EINVAL;
    for (int q = 0; q < 4; ++q)
        if (!(c->scale[q] > 0)) return EP_EINVAL;
    return EP_OK;
}

void layer_channels(int base, int ch[NL][2])
{
    const int c = base, c2 = 2 * base, c4 = 4 * base;
    const int t[NL][2] = {{CIN0, c}, {c, c}, {c, c2}, {c2, c2}, {c2, c4}, {c4, c4},
                          {c4, c2}, {c2, c2}, {c2, c}, {c, c}, {c, COUT}};
    std::memcpy(ch, t, sizeof(t));
}

// Walk the workspace layout (assign pointers when n->... base != null).
size_t net_carve(const ep_net_config* c, ep_net* n, char* base)
{
    int ch[NL][2];
    layer_channels(c->base, ch);
    const int D0 = (c->nz + 3) / 4 * 4, H0 = (c->ny + 3) / 4 * 4, W0 = (c->nx + 3) / 4 * 4;
    Vol g0 = make_vol(D0, H0, W0), g1 = make_vol(D0 / 2, H0 / 2, W0 / 2), g2 = make_vol(D0 / 4, H0 / 4, W0 / 4);
    long np = 0, nwb = 0;
    long woff[NL], boff[NL], wboff[NL];
    for (int l = 0; l < NL; ++l) {
        woff[l] = np;
        np += (long)ch[l][1] * 27 * ch[l][0];
        boff[l] = np;
        np += ch[l][1];
        wboff[l] = nwb;
        nwb += (long)ch[l][1] * 27 * ch[l][0];
    }
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) / 256 * 256;
        char* r = base ? base + off : nullptr;
        off += bytes;
        return r;
    };
    auto act = [&](const Vol& g, int C) { return (bf16_t*)take((size_t)g.Vp * C * sizeof(bf16_t)); };
    const int C = c->base, C2 = 2 * C, C4 = 4 * C;
    float* w = (float*)take(np * 4);
    float* gr = (float*)take(np * 4);
    float* m = (float*)take(np * 4);
    float* v = (float*)take(np * 4);
    bf16_t* wb = (bf16_t*)take(nwb * 2);
    bf16_t* wtb = (bf16_t*)take(nwb * 2);
    bf16_t* A[17];
    const Vol* gl[17] = {&g0, &g0, &g0, &g1, &g1, &g1, &g2, &g2, &g2, &g1, &g1, &g1, &g1, &g0, &g0, &g0, &g0};
    const int cl[17] = {CIN0, C, C, C, C2, C2, C2, C4, C4, C4, C2, C2, C2, C2, C, C, C};
    for (int q = 0; q < 17; ++q) A[q] = act(*gl[q], cl[q]);
    float* y = (float*)take((size_t)g0.V * COUT * 4);
    bf16_t* G[21];
    const Vol* gg[21] = {&g0, &g0, &g0, &g0, &g0, &g1, &g1, &g1, &g1, &g1, &g2, &g2, &g2, &g2, &g1, &g1, &g1, &g1, &g0,
                         &g0, &g0};
    const int cg[21] = {COUT, C, C, C, C2, C2, C2, C2, C2, C4, C4, C4, C4, C2, C2, C2, C2, C, C, C, C};
    // gradient tensors only for a network that trains (max_samples > 0)
    for (int q = 0; q < 21; ++q) G[q] = c->max_samples > 0 ? act(*gg[q], cg[q]) : nullptr;
    bf16_t* sx = (bf16_t*)take((size_t)c->max_samples * g0.Vp * 16 * 2);
    float* stg = (float*)take((size_t)c->max_samples * g0.V * 4 * 4);
    double* vlast = (double*)take((size_t)g0.V * 3 * 8);
    float* dvp = (float*)take((size_t)g0.V * 4 * 4);
    double* loss = (double*)take(8);
    float* part = c->max_samples > 0 ? (float*)take(PART_FLOATS * 4) : nullptr;
    if (n) {
        n->g[0] = g0; n->g[1] = g1; n->g[2] = g2;
        std::memcpy(n->ch, ch, sizeof(ch));
        std::memcpy(n->woff, woff, sizeof(woff));
        std::memcpy(n->boff, boff, sizeof(boff));
        std::memcpy(n->wboff, wboff, sizeof(wboff));
        n->np = np; n->nwb = nwb;
        n->w = w; n->gr = gr; n->m = m; n->v = v; n->wb = wb; n->wtb = wtb;
        bf16_t** dst[17] = {&n->xin, &n->a0, &n->s0, &n->p0, &n->a1, &n->s1, &n->p1, &n->a2, &n->b2,
                            &n->u1, &n->r6, &n->c1, &n->d1, &n->u0, &n->r8, &n->c0, &n->d0};
        for (int q = 0; q < 17; ++q) *dst[q] = A[q];
        n->y = y;
        bf16_t** gd[21] = {&n->gy, &n->z9, &n->gc0, &n->z8, &n->t0, &n->gd1, &n->z7, &n->gc1, &n->z6, &n->t1, &n->gb2,
                           &n->z5, &n->z4, &n->t2, &n->gs1, &n->z3, &n->z2, &n->t3, &n->gs0, &n->z1, &n->z0};
        for (int q = 0; q < 21; ++q) *gd[q] = G[q];
        n->sx = sx; n->stg = stg; n->vlast = vlast; n->dvp = dvp; n->loss = loss; n->part = part;
    }
    return (off + 255) / 256 * 256;
}

// ---- launch helpers -------------------------------------------------------
template <int EPI>
void conv_epi(int nb, const bf16_t* X, int cin, const bf16_t* W, const float* b, void* Y, const bf16_t* M,
              const Vol& g, hipStream_t s)
{
    const dim3 grid((g.W + CB_X - 1) / CB_X, (g.H + CB_Y - 1) / CB_Y, (g.D + CB_Z - 1) / CB_Z);
    switch (nb) {
    case 1: k_conv<1, EPI><<<grid, 256, 0, s>>>(X, cin, W, b, Y, M, g); break;
    case 2: k_conv<2, EPI><<<grid, 256, 0, s>>>(X, cin, W, b, Y, M, g); break;
    case 4: k_conv<4, EPI><<<grid, 256, 0, s>>>(X, cin, W, b, Y, M, g); break;
    default: k_conv<8, EPI><<<grid, 256, 0, s>>>(X, cin, W, b, Y, M, g); break;
    }
}

void conv(int epi, int cout, const bf16_t* X, int cin, const bf16_t* W, const float* b, void* Y, const bf16_t* M,
          const Vol& g, hipStream_t s)
{
    const int nb = cout / 16;
    if (epi == EPI_RELU) conv_epi<EPI_RELU>(nb, X, cin, W, b, Y, M, g, s);
    else if (epi == EPI_LIN) conv_epi<EPI_LIN>(nb, X, cin, W, b, Y, M, g, s);
    else if (epi == EPI_MASK) conv_epi<EPI_MASK>(nb, X, cin, W, b, Y, M, g, s);
    else conv_epi<EPI_F32>(nb, X, cin, W, b, Y, M, g, s);
}

// Slabs of 128 voxels where neither tensor has more than 32 channels (fewer
// barriers per voxel; the two stages still take only 17 KB of LDS), else 64.
template <int NBO, int NBI>
void launch_wgrad(unsigned grid, const bf16_t* X, const bf16_t* G, float* part, const Vol& g, long vchunk,
                  hipStream_t s)
{
    constexpr int SL = (NBO <= 2 && NBI <= 2) ? 128 : 64;
    k_wgrad<NBO, NBI, SL><<<grid, 256, 0, s>>>(X, G, part, g, vchunk);
}

template <int NBO>
void wgrad_o(int nbi, const bf16_t* X, const bf16_t* G, float* part, float* dW, const Vol& g, hipStream_t s)
{
    // voxel chunks of at least 2048 voxels (a multiple of 128, so of either
    // slab size), at most 512 per tap (27 x 512 workgroups keep the staging
    // latency hidden) and as many as the partial-sum buffer holds
    const long E = 27L * NBO * 16 * nbi * 16;
    long nch = std::min<long>((g.V + 2047) / 2048, std::min<long>(512, PART_FLOATS / E));
    const long vchunk = ((g.V + nch - 1) / nch + 127) / 128 * 128;
    nch = (g.V + vchunk - 1) / vchunk;
    const unsigned grid = (unsigned)nch * 27u;
    switch (nbi) {
    case 1: launch_wgrad<NBO, 1>(grid, X, G, part, g, vchunk, s); break;
    case 2: launch_wgrad<NBO, 2>(grid, X, G, part, g, vchunk, s); break;
    case 4: launch_wgrad<NBO, 4>(grid, X, G, part, g, vchunk, s); break;
    default: launch_wgrad<NBO, 8>(grid, X, G, part, g, vchunk, s); break;
    }
    k_wsum<<<(unsigned)((E + 31) / 32), 256, 0, s>>>(part, nch, E, dW);
}

// Weight and bias gradients of one layer, added to dW and db through the
// partial-sum buffer part (PART_FLOATS floats), deterministically.
void wgrad(float* part, int cout, int cin, const bf16_t* X, const bf16_t* G, float* dW, float* db, const Vol& g,
           hipStream_t s)
{
    switch (cout / 16) {
    case 1: wgrad_o<1>(cin / 16, X, G, part, dW, g, s); break;
    case 2: wgrad_o<2>(cin / 16, X, G, part, dW, g, s); break;
    case 4: wgrad_o<4>(cin / 16, X, G, part, dW, g, s); break;
    default: wgrad_o<8>(cin / 16, X, G, part, dW, g, s); break;
    }
    const int nb = (int)std::min<long>(1024, (g.V * (cout / 8) + 255) / 256);
    k_bias_grad<<<(unsigned)nb, 256, 0, s>>>(G, cout, part, g);
    k_bsum<<<(unsigned)cout, 256, 0, s>>>(part, nb, cout, db);
}

void refresh_bf16(ep_net* n)
{
    for (int l = 0; l < NL; ++l) {
        const long cnt = (long)n->ch[l][1] * 27 * n->ch[l][0];
        k_wcopy<<<nblk(cnt), 256, 0, n->st>>>(n->w + n->woff[l], n->wb + n->wboff[l], n->wtb + n->wboff[l],
                                              n->ch[l][1], n->ch[l][0]);
    }
}

const bf16_t* slot_x(const ep_net* n, int slot) { return slot < 0 ? n->xin : n->sx + (size_t)slot * n->g[0].Vp * 16; }
float* slot_t(const ep_net* n, int slot) { return n->stg + (size_t)slot * n->g[0].V * 4; }

void forward(ep_net* n, const bf16_t* x)
{
    hipStream_t s = n->st;
    const Vol &g0 = n->g[0], &g1 = n->g[1], &g2 = n->g[2];
    const int C = n->cfg.base, C2 = 2 * C, C4 = 4 * C;
    auto W = [&](int l) { return n->wb + n->wboff[l]; };
    auto B = [&](int l) { return n->w + n->boff[l]; };
    conv(EPI_RELU, C, x, CIN0, W(0), B(0), n->a0, nullptr, g0, s);
    conv(EPI_RELU, C, n->a0, C, W(1), B(1), n->s0, nullptr, g0, s);
    k_pool<<<nblk(g1.V * C), 256, 0, s>>>(n->s0, n->p0, C, g0, g1);
    conv(EPI_RELU, C2, n->p0, C, W(2), B(2), n->a1, nullptr, g1, s);
    conv(EPI_RELU, C2, n->a1, C2, W(3), B(3), n->s1, nullptr, g1, s);
    k_pool<<<nblk(g2.V * C2), 256, 0, s>>>(n->s1, n->p1, C2, g1, g2);
    conv(EPI_RELU, C4, n->p1, C2, W(4), B(4), n->a2, nullptr, g2, s);
    conv(EPI_RELU, C4, n->a2, C4, W(5), B(5), n->b2, nullptr, g2, s);
    k_up<<<nblk(g1.V * C4), 256, 0, s>>>(n->b2, n->u1, C4, g1, g2);
    conv(EPI_RELU, C2, n->u1, C4, W(6), B(6), n->r6, nullptr, g1, s);
    k_add<<<nblk(g1.V * C2), 256, 0, s>>>(n->r6, n->s1, n->c1, C2, g1);
    conv(EPI_RELU, C2, n->c1, C2, W(7), B(7), n->d1, nullptr, g1, s);
    k_up<<<nblk(g0.V * C2), 256, 0, s>>>(n->d1, n->u0, C2, g0, g1);
    conv(EPI_RELU, C, n->u0, C2, W(8), B(8), n->r8, nullptr, g0, s);
    k_add<<<nblk(g0.V * C), 256, 0, s>>>(n->r8, n->s0, n->c0, C, g0);
    conv(EPI_RELU, C, n->c0, C, W(9), B(9), n->d0, nullptr, g0, s);
    conv(EPI_F32, COUT, n->d0, C, W(10), B(10), n->y, nullptr, g0, s);
}

// Gradient of the loss of the current forward pass with respect to all
// parameters, accumulated into n->gr (cleared first).
void backward(ep_net* n, const bf16_t* x)
{
    hipStream_t s = n->st;
    const Vol &g0 = n->g[0], &g1 = n->g[1], &g2 = n->g[2];
    const int C = n->cfg.base, C2 = 2 * C, C4 = 4 * C;
    auto WT = [&](int l) { return n->wtb + n->wboff[l]; };
    auto GW = [&](int l) { return n->gr + n->woff[l]; };
    auto GB = [&](int l) { return n->gr + n->boff[l]; };
    k_fill_f<<<nblk(n->np), 256, 0, s>>>(n->gr, 0.f, n->np);
    wgrad(n->part, COUT, C, n->d0, n->gy, GW(10), GB(10), g0, s);
    conv(EPI_MASK, C, n->gy, COUT, WT(10), nullptr, n->z9, n->d0, g0, s);
    wgrad(n->part, C, C, n->c0, n->z9, GW(9), GB(9), g0, s);
    conv(EPI_LIN, C, n->z9, C, WT(9), nullptr, n->gc0, nullptr, g0, s);
    k_mask<<<nblk(g0.V * C), 256, 0, s>>>(n->gc0, n->r8, n->z8, C, g0);
    wgrad(n->part, C, C2, n->u0, n->z8, GW(8), GB(8), g0, s);
    conv(EPI_LIN, C2, n->z8, C, WT(8), nullptr, n->t0, nullptr, g0, s);
    k_up_dx<<<nblk(g1.V * C2), 256, 0, s>>>(n->t0, n->gd1, C2, g0, g1);
    k_mask<<<nblk(g1.V * C2), 256, 0, s>>>(n->gd1, n->d1, n->z7, C2, g1);
    wgrad(n->part, C2, C2, n->c1, n->z7, GW(7), GB(7), g1, s);
    conv(EPI_LIN, C2, n->z7, C2, WT(7), nullptr, n->gc1, nullptr, g1, s);
    k_mask<<<nblk(g1.V * C2), 256, 0, s>>>(n->gc1, n->r6, n->z6, C2, g1);
    wgrad(n->part, C2, C4, n->u1, n->z6, GW(6), GB(6), g1, s);
    conv(EPI_LIN, C4, n->z6, C2, WT(6), nullptr, n->t1, nullptr, g1, s);
    k_up_dx<<<nblk(g2.V * C4), 256, 0, s>>>(n->t1, n->gb2, C4, g1, g2);
    k_mask<<<nblk(g2.V * C4), 256, 0, s>>>(n->gb2, n->b2, n->z5, C4, g2);
    wgrad(n->part, C4, C4, n->a2, n->z5, GW(5), GB(5), g2, s);
    conv(EPI_MASK, C4, n->z5, C4, WT(5), nullptr, n->z4, n->a2, g2, s);
    wgrad(n->part, C4, C2, n->p1, n->z4, GW(4), GB(4), g2, s);
    conv(EPI_LIN, C2, n->z4, C4, WT(4), nullptr, n->t2, nullptr, g2, s);
    k_add_pool_dx<<<nblk(g1.V * C2), 256, 0, s>>>(n->gc1, n->t2, n->gs1, C2, g1, g2);
    k_mask<<<nblk(g1.V * C2), 256, 0, s>>>(n->gs1, n->s1, n->z3, C2, g1);
    wgrad(n->part, C2, C2, n->a1, n->z3, GW(3), GB(3), g1, s);
    conv(EPI_MASK, C2, n->z3, C2, WT(3), nullptr, n->z2, n->a1, g1, s);
    wgrad(n->part, C2, C, n->p0, n->z2, GW(2), GB(2), g1, s);
    conv(EPI_LIN, C, n->z2, C2, WT(2), nullptr, n->t3, nullptr, g1, s);
    k_add_pool_dx<<<nblk(g0.V * C), 256, 0, s>>>(n->gc0, n->t3, n->gs0, C, g0, g1);
    k_mask<<<nblk(g0.V * C), 256, 0, s>>>(n->gs0, n->s0, n->z1, C, g0);
    wgrad(n->part, C, C, n->a0, n->z1, GW(1), GB(1), g0, s);
    conv(EPI_MASK, C, n->z1, C, WT(1), nullptr, n->z0, n->a0, g0, s);
    wgrad(n->part, C, CIN0, x, n->z0, GW(0), GB(0), g0, s);
}

float inv_count(const ep_net* n)
{
    const long nf = (long)(n->cfg.nx - 1) * n->cfg.ny * n->cfg.nz + (long)n->cfg.nx * (n->cfg.ny - 1) * n->cfg.nz +
                    (long)n->cfg.nx * n->cfg.ny * (n->cfg.nz - 1);
    return 1.f / (float)nf;
}

int loss_and_grad(ep_net* n, int slot, double* loss_out)
{
    hipStream_t s = n->st;
    const bf16_t* x = slot_x(n, slot);
    forward(n, x);
    const Vol& g0 = n->g[0];
    const unsigned nb = std::min(nblk(g0.V), 1024u);
    k_loss<<<nb, 256, 0, s>>>(n->y, slot_t(n, slot), n->gy, g0, n->cfg.nx, n->cfg.ny, n->cfg.nz, inv_count(n),
                              (double*)n->part);
    k_lsum<<<1, 256, 0, s>>>((const double*)n->part, (int)nb, n->loss);
    backward(n, x);
    if (loss_out) {
        NCHK(n, hipMemcpyAsync(loss_out, n->loss, 8, hipMemcpyDeviceToHost, s));
        NCHK(n, hipStreamSynchronize(s));
    }
    NCHK(n, hipGetLastError());
    return EP_OK;
}

SolverView view_of(const ep_handle* h)
{
    SolverView v;
    double* const* it = h->it64[h->cur64];
    v.txx = it[F_TXX]; v.tyy = it[F_TYY]; v.txy = it[F_TXY]; v.txz = it[F_TXZ]; v.tyz = it[F_TYZ];
    v.p = it[F_P]; v.epsp = h->epsp64;
    v.vx = it[F_VX]; v.vy = it[F_VY]; v.vz = it[F_VZ];
    v.nx = h->nx; v.ny = h->ny; v.nz = h->nz; v.sy = h->sy; v.sz = h->sz;
    return v;
}

int check_handle(ep_net* n, ep_handle* h)
{
    if (!h) return nerr(n, EP_EINVAL, "no solver handle");
    if (h->ndim != 3 || h->nx != n->cfg.nx || h->ny != n->cfg.ny || h->nz != n->cfg.nz)
        return nerr(n, EP_EINVAL, "solver grid %dx%dx%d does not match the network's %dx%dx%d", h->nx, h->ny, h->nz,
                    n->cfg.nx, n->cfg.ny, n->cfg.nz);
    ensure_it64(h);
    return EP_OK;
}

}  // namespace

// =========================================================================
extern "C" {

int ep_net_workspace_size(const ep_net_config* c, size_t* bytes)
{
    if (!bytes || validate_cfg(c) != EP_OK) return EP_EINVAL;
    *bytes = net_carve(c, nullptr, nullptr);
    return EP_OK;
}

int ep_net_init(const ep_net_config* c, void* d_workspace, size_t ws_bytes, void* stream, ep_net** out)
{
    if (!out) return EP_EINVAL;
    *out = nullptr;
    if (validate_cfg(c) != EP_OK) return EP_EINVAL;
    const size_t need = net_carve(c, nullptr, nullptr);
    if (!d_workspace || ws_bytes < need) return EP_ENOMEM;
    if (((uintptr_t)d_workspace & 255) != 0) return EP_EINVAL;
    ep_net* n = new (std::nothrow) ep_net();
    if (!n) return EP_ENOMEM;
    n->cfg = *c;
    n->st = (hipStream_t)stream;
    net_carve(c, n, (char*)d_workspace);
    auto fail = [&](int code) { delete n; return code; };
    if (hipMemsetAsync(d_workspace, 0, need, n->st) != hipSuccess) return fail(EP_EDEVICE);
    // He-normal initialisation (std sqrt(2 / (27 Cin))), zero biases, zero head
    std::vector<float> w(n->np, 0.f);
    std::mt19937_64 rng((unsigned long long)c->seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int l = 0; l < NL - 1; ++l) {
        const double sd = std::sqrt(2.0 / (27.0 * n->ch[l][0]));
        const long cnt = (long)n->ch[l][1] * 27 * n->ch[l][0];
        for (long q = 0; q < cnt; ++q) w[n->woff[l] + q] = (float)(nd(rng) * sd);
    }
    if (hipMemcpyAsync(n->w, w.data(), n->np * 4, hipMemcpyHostToDevice, n->st) != hipSuccess) return fail(EP_EDEVICE);
    refresh_bf16(n);
    if (hipStreamSynchronize(n->st) != hipSuccess || hipGetLastError() != hipSuccess) return fail(EP_EDEVICE);
    *out = n;
    return EP_OK;
}

void ep_net_destroy(ep_net* n) { delete n; }

const char* ep_net_last_error(const ep_net* n) { return n ? n->err : "no network"; }

long ep_net_param_count(const ep_net* n) { return n ? n->np : EP_EINVAL; }

int ep_net_params(ep_net* n, int dir, float* host, size_t count)
{
    if (!n || !host || (dir != EP_GET && dir != EP_SET)) return EP_EINVAL;
    if (count != (size_t)n->np) return nerr(n, EP_EINVAL, "count %zu, expected %ld", count, n->np);
    if (dir == EP_GET) {
        NCHK(n, hipMemcpyAsync(host, n->w, n->np * 4, hipMemcpyDeviceToHost, n->st));
    } else {
        NCHK(n, hipMemcpyAsync(n->w, host, n->np * 4, hipMemcpyHostToDevice, n->st));
        k_fill_f<<<nblk(n->np), 256, 0, n->st>>>(n->m, 0.f, n->np);
        k_fill_f<<<nblk(n->np), 256, 0, n->st>>>(n->v, 0.f, n->np);
        n->adam_t = 0;
        refresh_bf16(n);
    }
    NCHK(n, hipStreamSynchronize(n->st));
    NCHK(n, hipGetLastError());
    return EP_OK;
}

int ep_net_sample(ep_net* n, int slot, int dir, float* x, float* t)
{
    if (!n || slot < 0 || slot >= n->cfg.max_samples || (dir != EP_GET && dir != EP_SET)) return EP_EINVAL;
    const Vol& g = n->g[0];
    if (x) {
        bf16_t* dev = const_cast<bf16_t*>(slot_x(n, slot));
        std::vector<bf16_t> pad((size_t)g.Vp * 16, 0);
        if (dir == EP_GET) {
            NCHK(n, hipMemcpyAsync(pad.data(), dev, pad.size() * 2, hipMemcpyDeviceToHost, n->st));
            NCHK(n, hipStreamSynchronize(n->st));
        }
        for (int z = 0; z < g.D; ++z)
            for (int y = 0; y < g.H; ++y)
                for (int xx = 0; xx < g.W; ++xx) {
                    const long v = ((long)z * g.H + y) * g.W + xx;
                    const long p = (((long)z + 1) * g.Hp + y + 1) * g.Wp + xx + 1;
                    for (int c = 0; c < 16; ++c) {
                        if (dir == EP_GET) x[v * 16 + c] = host_bf2f(pad[p * 16 + c]);
                        else pad[p * 16 + c] = host_f2bf(x[v * 16 + c]);
                    }
                }
        if (dir == EP_SET) {
            NCHK(n, hipMemcpyAsync(dev, pad.data(), pad.size() * 2, hipMemcpyHostToDevice, n->st));
            NCHK(n, hipStreamSynchronize(n->st));
        }
    }
    if (t) {
        if (dir == EP_GET) NCHK(n, hipMemcpyAsync(t, slot_t(n, slot), g.V * 16, hipMemcpyDeviceToHost, n->st));
        else NCHK(n, hipMemcpyAsync(slot_t(n, slot), t, g.V * 16, hipMemcpyHostToDevice, n->st));
        NCHK(n, hipStreamSynchronize(n->st));
    }
    return EP_OK;
}

int ep_net_record(ep_net* n, ep_handle* h, int slot)
{
    if (!n || slot < -1 || slot >= n->cfg.max_samples) return EP_EINVAL;
    int rc = check_handle(n, h);
    if (rc) return rc;
    const Vol& g = n->g[0];
    k_features<<<nblk(g.V), 256, 0, n->st>>>(view_of(h), n->dvp, const_cast<bf16_t*>(slot_x(n, slot)), g,
                                             1.f / n->cfg.scale[0], 1.f / n->cfg.scale[1], 1.f / n->cfg.scale[2]);
    NCHK(n, hipGetLastError());
    return EP_OK;
}

int ep_net_observe(ep_net* n, ep_handle* h, int slot)
{
    if (!n || slot < -1 || slot >= n->cfg.max_samples) return EP_EINVAL;
    int rc = check_handle(n, h);
    if (rc) return rc;
    const Vol& g = n->g[0];
    k_observe<<<nblk(g.V), 256, 0, n->st>>>(view_of(h), n->vlast, n->dvp, slot >= 0 ? slot_t(n, slot) : nullptr, g,
                                            n->have_last ? 0 : 1, 1.f / n->cfg.scale[3]);
    n->have_last = true;
    NCHK(n, hipStreamSynchronize(n->st));
    NCHK(n, hipGetLastError());
    return EP_OK;
}

int ep_net_reset(ep_net* n)
{
    if (!n) return EP_EINVAL;
    n->have_last = false;
    return EP_OK;
}

int ep_net_forward(ep_net* n, int slot, float* y)
{
    if (!n || slot < -1 || slot >= n->cfg.max_samples) return EP_EINVAL;
    forward(n, slot_x(n, slot));
    if (y) NCHK(n, hipMemcpyAsync(y, n->y, n->g[0].V * COUT * 4, hipMemcpyDeviceToHost, n->st));
    NCHK(n, hipStreamSynchronize(n->st));
    NCHK(n, hipGetLastError());
    return EP_OK;
}

int ep_net_gradient(ep_net* n, int slot, double* loss, float* grad)
{
    if (!n || slot < 0 || slot >= n->cfg.max_samples) return EP_EINVAL;
    int rc = loss_and_grad(n, slot, loss);
    if (rc) return rc;
    if (grad) {
        NCHK(n, hipMemcpyAsync(grad, n->gr, n->np * 4, hipMemcpyDeviceToHost, n->st));
        NCHK(n, hipStreamSynchronize(n->st));
    }
    return EP_OK;
}

int ep_net_train(ep_net* n, const int* slots, int nslots, int nsteps, float lr, float* losses)
{
    if (!n || !slots || nslots <= 0 || nsteps < 0 || !(lr > 0)) return EP_EINVAL;
    for (int q = 0; q < nslots; ++q)
        if (slots[q] < 0 || slots[q] >= n->cfg.max_samples) return EP_EINVAL;
    for (int k = 0; k < nsteps; ++k) {
        double l = 0;
        int rc = loss_and_grad(n, slots[k % nslots], losses ? &l : nullptr);
        if (rc) return rc;
        if (losses) losses[k] = (float)l;
        ++n->adam_t;
        const float c1 = 1.f - std::pow(0.9f, (float)n->adam_t), c2 = 1.f - std::pow(0.999f, (float)n->adam_t);
        k_adam<<<nblk(n->np), 256, 0, n->st>>>(n->w, n->gr, n->m, n->v, n->np, lr, c1, c2);
        refresh_bf16(n);
    }
    NCHK(n, hipStreamSynchronize(n->st));
    NCHK(n, hipGetLastError());
    return EP_OK;
}

int ep_net_predict(ep_net* n, ep_handle* h)
{
    if (!n) return EP_EINVAL;
    int rc = ep_net_record(n, h, -1);
    if (rc) return rc;
    forward(n, n->xin);
    const long nf = (long)(h->nx + 1) * (h->ny + 1) * (h->nz + 1);
    k_apply_guess<<<nblk(nf), 256, 0, n->st>>>(view_of(h), n->y, h->vguess64[0], h->vguess64[1], h->vguess64[2],
                                               n->g[0], n->cfg.scale[3]);
    NCHK(n, hipGetLastError());
    h->guess_ready = true;
    return EP_OK;
}

}  // extern "C"
