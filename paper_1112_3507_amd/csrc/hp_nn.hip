// hp_nn.hip -- the learned warm start / preconditioner: a small 3D U-Net in BF16 on the gfx950
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), with hand-written forward,
// backward-data, backward-weight, pooling, head, loss and Adam kernels.
//
// Network (levels n, n/2, n/4; channels 16/32/64; 3x3x3 convolutions with periodic padding in
// x and y and zero padding in z, like the solver's boundaries):
//   e1 = relu(conv(relu(conv(in, 4->16)), 16->16))
//   e2 = relu(conv(relu(conv(pool(e1), 16->32)), 32->32))
//   e3 = relu(conv(relu(conv(pool(e2), 32->64)), 64->64))
//   d2 = relu(conv(relu(conv([up(e3), e2], 96->32)), 32->32))
//   d1 = relu(conv(relu(conv([up(d2), e1], 48->16)), 16->16))
//   y  = d1 . w_out + b_out
// pool = 2x2x2 mean, up = nearest 2x copy, [.,.] = channel concatenation (never materialised:
// the convolution reads the two tensors, and the upsampled one at half the coordinates).
//
// Layout: activations channels-last ([voxel][channel], x fastest) in bfloat16, gradients in
// FP32. Parameters are one flat FP32 vector: per convolution W[o][tap][c] then b[o], then
// w_out[16], b_out; taps t = (dz+1)*9 + (dy+1)*3 + (dx+1).
//
// Convolution as a GEMM on the matrix cores: D[o][v] = sum_k W[o][k] X[k][v] with k = (tap, c).
// A 256-thread workgroup owns a 16 x 4 x (4 SPW) brick of output voxels; the input brick with its
// one-voxel halo is staged in LDS one channel chunk at a time (each thread loading whole halo
// voxels at indices fixed for the launch); every wave64 owns SPW z-slices of the brick (four
// 16-voxel rows each). With one 16-channel output tile the weights of the chunk are staged in
// LDS and held in registers, and the products run input row by input row, each B fragment read
// once and fed to every output row it reaches (up to 9 products per LDS read); with several
// tiles each K step of 32 feeds one MFMA per tile and row. ReLU, the bfloat16 rounding and (in
// inference) the network head run in the epilogue. The backward-data pass is the same kernel with the weights
// flipped in space and transposed in channels; the backward-weight pass contracts over voxels
// with both operands transposed through LDS.
#include "hp.h"
#include "hp_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace hpnn {

typedef unsigned short bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BX = 16, BY = 4, BZ = 4;                 // output brick
constexpr int HX = BX + 2, HY = BY + 2, HZ = BZ + 2;  // input brick with halo
constexpr int HV = HX * HY * HZ;                       // 648 halo voxels
constexpr int NCONV = 10;
constexpr int CIN[NCONV] = {4, 16, 16, 32, 32, 64, 96, 32, 48, 16};
constexpr int COUT[NCONV] = {16, 16, 32, 32, 64, 64, 32, 32, 16, 16};
constexpr int HEAD = 16;

__host__ __device__ inline int cin_pad(int l) { return CIN[l] < 8 ? 8 : CIN[l]; }

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((unsigned)h << 16); }
// round to nearest even
__device__ __forceinline__ bf16_t f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// two floats to two bfloat16 (round to nearest even) in one word, low half first: one
// v_cvt_pk_bf16_f32 on gfx950
__device__ __forceinline__ unsigned pack_bf2(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------------------------------------
// convolution forward (also backward-data with transformed weights)

struct ConvArgs {
    const bf16_t* a;  // first input tensor (ca channels), half resolution if a_up
    int ca, a_up;
    const bf16_t* b;  // second input tensor (cb channels), full resolution
    int cb;
    const bf16_t* w;  // [cout][27 * (ca + cb)]
    const float* bias;
    void* out;        // [voxel][cout], bf16 or f32
    int cout;
    int nx, ny, nz;
    int relu;
    // non-null (one output tile only): the network head is applied in the epilogue and out is
    // y[voxel] (FP32) = sum_c bf16(act[voxel][c]) head[c] + head[16]; act itself is not stored
    const float* head;
    // non-null (one output tile, two z-slices per wave, bf16 output): the 2x2x2 mean of the
    // stored activation is written here as well ([coarse voxel][16], grid sizes halved)
    bf16_t* pool_out;
};

// SPW z-slices per wave: the output brick is 16 x 4 x (4 SPW) voxels.
template <int CT, int G, int SPW, bool OUT_F32>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvArgs p) {
    constexpr int CC = 8 * G;                  // channels per LDS chunk
    constexpr int FZ = 4 * SPW, FHZ = FZ + 2, FHV = HX * HY * FHZ;
    constexpr int NV = (FHV + 255) / 256;      // halo voxels per thread (G 16-byte loads each)
    constexpr int NSTEPS = (27 * CC + 31) / 32;
    // one output tile (16 channels): its weights of the chunk are staged in LDS too
    constexpr bool WL = (CT == 1);
    constexpr int NWL = WL ? 16 * 27 * G : 0;  // 16-byte weight groups of the chunk
    constexpr int NUW = (NWL + 255) / 256;
    // LDS layout: the halo brick as G planes [8-channel group][halo voxel], so the 16 lanes that
    // read one B fragment row touch 16 consecutive 16-byte words; the weight rows at an odd
    // stride of 16-byte words for the same reason on the A fragment
    constexpr int WS = (27 * G) | 1;
    __shared__ uint4 lds[FHV * G + (WL ? 16 * WS : 0)];
    const int cin = p.ca + p.cb;
    const int bxn = (p.nx + BX - 1) / BX, byn = (p.ny + BY - 1) / BY;
    const int bid = blockIdx.x;
    const int x0 = (bid % bxn) * BX;
    const int y0 = ((bid / bxn) % byn) * BY;
    const int z0 = (bid / (bxn * byn)) * FZ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, grp = lane >> 4;
    const int anx = p.a_up ? p.nx >> 1 : p.nx, any = p.a_up ? p.ny >> 1 : p.ny;
    const int Ktot = 27 * cin;

    // The thread's halo voxels (hv = tid + 256 i): their voxel index in the full-resolution
    // tensor b and in tensor a (half resolution when upsampled), -1 outside the grid (zero
    // padding in z; a brick wider than the grid reaches past the periodic image in x or y,
    // and those voxels only feed outputs outside the grid). Fixed for the whole launch.
    int vb[NV], va[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int hv = tid + 256 * i;
        const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
        int gx = x0 + hx - 1, gy = y0 + hy - 1;
        const int gz = z0 + hz - 1;
        gx = gx < 0 ? gx + p.nx : (gx >= p.nx ? gx - p.nx : gx);
        gy = gy < 0 ? gy + p.ny : (gy >= p.ny ? gy - p.ny : gy);
        const bool in = hv < FHV && gz >= 0 && gz < p.nz && gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny;
        vb[i] = in ? (gz * p.ny + gy) * p.nx + gx : -1;
        va[i] = !in ? -1 : (p.a_up ? ((gz >> 1) * any + (gy >> 1)) * anx + (gx >> 1) : vb[i]);
    }
    // accumulators start from the bias: this lane's outputs are channels ct*16 + 4 grp + e
    f32x4 acc[4 * SPW][CT];  // row r of slice sl at 4 sl + r
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        f32x4 b0 = {0.f, 0.f, 0.f, 0.f};
        if (p.bias) {
#pragma unroll
            for (int e = 0; e < 4; ++e) b0[e] = p.bias[ct * 16 + 4 * grp + e];
        }
#pragma unroll
        for (int r = 0; r < 4 * SPW; ++r) acc[r][ct] = b0;
    }
    // weight fragment of K step s: 8 consecutive k of output row ct*16 + li
    auto wload = [&](int c0, int s, uint4* w) {
        const int kk = s * 32 + grp * 8;
        const int tap = kk / CC, c = kk - tap * CC;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            w[ct] = tap < 27 ? *(const uint4*)(p.w + (int64_t)(ct * 16 + li) * Ktot + tap * cin + c0 + c)
                             : uint4{0u, 0u, 0u, 0u};
    };

    for (int c0 = 0; c0 < cin; c0 += CC) {
        // stage the chunk: all loads of a thread in flight before its LDS stores; a thread takes
        // whole halo voxels (the chunk's CC channels are G consecutive 16-byte words in memory)
        const bool from_a = c0 < p.ca;
        const bf16_t* base = from_a ? p.a + c0 : p.b + (c0 - p.ca);
        const int cstride = from_a ? p.ca : p.cb;
        uint4 v[NV][G];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            // outside the grid: a harmless load of voxel 0, replaced by zeros
            const int idx = from_a ? va[i] : vb[i];
            const uint4* src = (const uint4*)(base + (int64_t)(idx < 0 ? 0 : idx) * cstride);
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const uint4 t = src[q];
                v[i][q] = idx >= 0 ? t : uint4{0u, 0u, 0u, 0u};
            }
        }
        uint4 wcur[CT], wnext[CT];
        uint4 wv[NUW > 0 ? NUW : 1];
        if (WL) {
            // weight row o, tap, 8-channel group of the chunk -> lds[FHV G + o WS + tap G + group]
#pragma unroll
            for (int i = 0; i < NUW; ++i) {
                const int u = tid + 256 * i;
                wv[i] = uint4{0u, 0u, 0u, 0u};
                if ((i + 1) * 256 <= NWL || u < NWL) {
                    const int o = u / (27 * G), kq = u - o * (27 * G);
                    const int tap = kq / G, c8 = kq - tap * G;
                    wv[i] = *(const uint4*)(p.w + (int64_t)o * Ktot + tap * cin + c0 + c8 * 8);
                }
            }
        } else {
            wload(c0, 0, wcur);
        }
        __syncthreads();  // the previous chunk's reads of lds are done
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const int hv = tid + 256 * i;
            if ((i + 1) * 256 <= FHV || hv < FHV) {
#pragma unroll
                for (int q = 0; q < G; ++q) lds[q * FHV + hv] = v[i][q];
            }
        }
        if (WL) {
#pragma unroll
            for (int i = 0; i < NUW; ++i) {
                const int u = tid + 256 * i;
                if ((i + 1) * 256 <= NWL || u < NWL) lds[FHV * G + (u / (27 * G)) * WS + u % (27 * G)] = wv[i];
            }
        }
        __syncthreads();
        if constexpr (WL) {
            // One output tile: the products are taken input row by input row, so that each B
            // fragment read from LDS feeds every output row that needs it (up to 9). A K step holds
            // TPS taps of one (dz, dy) pair, neighbouring in dx, times the CC channels of the
            // chunk; its A fragments (weights) stay in registers for the whole chunk. Taps past
            // dx = 2 have zero weights (a quarter or a third of the products when TPS > 1).
            constexpr int TPS = 32 / CC;             // taps per K step (1, 2 or 4)
            constexpr int NT = (3 + TPS - 1) / TPS;  // K steps per (dz, dy)
            const int tin = (grp * 8) / CC, cg = ((grp * 8) % CC) >> 3;
            bf16x8 aw[9][NT];
#pragma unroll
            for (int q = 0; q < 9; ++q)
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int dx = t * TPS + tin;
                    const uint4 w = lds[FHV * G + li * WS + (q * 3 + (dx < 3 ? dx : 2)) * G + cg];
                    aw[q][t] = as_bf8(dx < 3 ? w : uint4{0u, 0u, 0u, 0u});
                }
#pragma unroll
            for (int iz = 0; iz < SPW + 2; ++iz)
#pragma unroll
                for (int iy = 0; iy < HY; ++iy)
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        // past dx = 2 the A side is zero; B reads the dx = 2 voxel (finite)
                        const int dx = t * TPS + tin;
                        const int hv = ((wave * SPW + iz) * HY + iy) * HX + li + (dx < 3 ? dx : 2);
                        const bf16x8 bf = as_bf8(lds[cg * FHV + hv]);
#pragma unroll
                        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                            for (int dy = 0; dy < 3; ++dy) {
                                const int sl = iz - dz, r = iy - dy;
                                if (sl < 0 || sl >= SPW || r < 0 || r >= 4) continue;
                                acc[sl * 4 + r][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    aw[dz * 3 + dy][t], bf, acc[sl * 4 + r][0], 0, 0, 0);
                            }
                    }
        } else {
            // several output tiles: K step by K step, each B fragment feeding CT products
#pragma unroll 2
            for (int s = 0; s < NSTEPS; ++s) {
                // next step's weights in flight while this step's products run
                if (s + 1 < NSTEPS) wload(c0, s + 1, wnext);
                const int kk = s * 32 + grp * 8;
                const int tap = kk / CC, c = kk - tap * CC;
                const bool kv = tap < 27;
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                bf16x8 af[CT];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) af[ct] = as_bf8(wcur[ct]);
#pragma unroll
                for (int sr = 0; sr < 4 * SPW; ++sr) {
                    const int sl = sr >> 2, r = sr & 3;
                    uint4 xv = {0u, 0u, 0u, 0u};
                    if (kv) {
                        const int hv = ((wave * SPW + sl + dz) * HY + (r + dy)) * HX + (li + dx);
                        xv = lds[(c >> 3) * FHV + hv];
                    }
                    const bf16x8 bf = as_bf8(xv);
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                        acc[sr][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ct], bf, acc[sr][ct], 0, 0, 0);
                }
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) wcur[ct] = wnext[ct];
            }
        }
    }
    // epilogue: this lane holds D[o = ct*16 + 4*grp + e][voxel li of row r of slice sl] (bias
    // included); a brick inside the grid needs no bounds checks
    const bool full = x0 + BX <= p.nx && y0 + BY <= p.ny && z0 + FZ <= p.nz;
    const int gx = x0 + li;
    constexpr bool POOL = (CT == 1 && SPW == 2 && !OUT_F32);
    uint2 stored[POOL ? 4 * SPW : 1];  // the bfloat16 pairs written for each row (pooling)
#pragma unroll
    for (int sr = 0; sr < (POOL ? 4 * SPW : 1); ++sr) stored[sr] = uint2{0u, 0u};
#pragma unroll
    for (int sr = 0; sr < 4 * SPW; ++sr) {
        const int gz = z0 + wave * SPW + (sr >> 2), gy = y0 + (sr & 3);
        if (!full && (gx >= p.nx || gy >= p.ny || gz >= p.nz)) continue;
        const int64_t vox = ((int64_t)gz * p.ny + gy) * p.nx + gx;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int o = ct * 16 + 4 * grp;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = p.relu ? fmaxf(acc[sr][ct][e], 0.f) : acc[sr][ct][e];
            if (CT == 1 && p.head) {
                // the activation as it would be stored (bfloat16), dotted with the head weights;
                // the four lanes of a voxel hold channels 4 grp .. 4 grp + 3
                const unsigned q0 = pack_bf2(v[0], v[1]), q1 = pack_bf2(v[2], v[3]);
                float part = __uint_as_float(q0 << 16) * p.head[o] + __uint_as_float(q0 & 0xffff0000u) * p.head[o + 1] +
                             __uint_as_float(q1 << 16) * p.head[o + 2] + __uint_as_float(q1 & 0xffff0000u) * p.head[o + 3];
                part += __shfl_xor(part, 16, 64);
                part += __shfl_xor(part, 32, 64);
                if (grp == 0) ((float*)p.out)[vox] = part + p.head[HEAD];
                continue;
            }
            if (OUT_F32) {
                *(float4*)((float*)p.out + vox * p.cout + o) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                uint2 pk;
                pk.x = pack_bf2(v[0], v[1]);
                pk.y = pack_bf2(v[2], v[3]);
                *(uint2*)((bf16_t*)p.out + vox * p.cout + o) = pk;
                if constexpr (POOL) stored[sr] = pk;
            }
        }
    }
    if constexpr (POOL) {
        if (p.pool_out) {
            // 2x2x2 mean of the stored activation: the wave holds two z-slices and four y rows, and
            // the x pair sits in lanes li, li + 1. The eight values of each channel are summed in
            // z, y, x order (x fastest) in FP32, then halved three times and rounded.
            const int cx = p.nx >> 1, cy = p.ny >> 1;
            const int X = gx >> 1, Z = (z0 + wave * SPW) >> 1;
#pragma unroll
            for (int yp = 0; yp < 2; ++yp) {
                float sum[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int zc = 0; zc < 2; ++zc)
#pragma unroll
                    for (int yc = 0; yc < 2; ++yc) {
                        const uint2 own = stored[zc * 4 + 2 * yp + yc];
                        const uint2 nxt = uint2{(unsigned)__shfl_down((int)own.x, 1, 64),
                                                (unsigned)__shfl_down((int)own.y, 1, 64)};
                        const unsigned w[2][2] = {{own.x, own.y}, {nxt.x, nxt.y}};
#pragma unroll
                        for (int xc = 0; xc < 2; ++xc) {
                            sum[0] += __uint_as_float(w[xc][0] << 16);
                            sum[1] += __uint_as_float(w[xc][0] & 0xffff0000u);
                            sum[2] += __uint_as_float(w[xc][1] << 16);
                            sum[3] += __uint_as_float(w[xc][1] & 0xffff0000u);
                        }
                    }
                const int Y = (y0 >> 1) + yp;
                if (!(li & 1) && gx < p.nx && 2 * Y < p.ny && 2 * Z < p.nz) {
                    uint2 pk;
                    pk.x = pack_bf2(sum[0] * 0.125f, sum[1] * 0.125f);
                    pk.y = pack_bf2(sum[2] * 0.125f, sum[3] * 0.125f);
                    *(uint2*)(p.pool_out + (((int64_t)Z * cy + Y) * cx + X) * 16 + 4 * grp) = pk;
                }
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// backward weights: dW[o][t][c] = sum_v g[v][o] x[v + d_t][c]
// One workgroup: a range of bricks, one 16-channel input chunk, all 27 taps (wave w owns taps
// w, w+4, ...). Operands are transposed into LDS so both MFMA fragments are 8 consecutive voxels.

struct BwdWArgs {
    const bf16_t* g;  // [voxel][cout] gradient at the convolution output (after the ReLU mask)
    int cout;
    const bf16_t* a;  // conv input tensors as in ConvArgs
    int ca, a_up;
    const bf16_t* b;
    int cb;
    float* partial;   // [gridDim.x][cin_chunks][cout][27][16]
    int nx, ny, nz;
};

constexpr int XROW = 24;  // padded halo row in LDS (16-byte aligned rows)

template <int CT>
__global__ __launch_bounds__(256) void k_conv_bwd_w(BwdWArgs p) {
    __shared__ bf16_t gt[64 * 256];                 // [o][v] of one brick
    __shared__ bf16_t xt[16 * HZ * HY * XROW];      // [c][hz][hy][XROW]
    const int cin = p.ca + p.cb;
    const int chunk = blockIdx.y, c0 = chunk * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, grp = lane >> 4;
    const int bxn = (p.nx + BX - 1) / BX, byn = (p.ny + BY - 1) / BY, bzn = (p.nz + BZ - 1) / BZ;
    const int nbricks = bxn * byn * bzn;
    const int anx = p.a_up ? p.nx >> 1 : p.nx, any = p.a_up ? p.ny >> 1 : p.ny;
    constexpr int NT = 7;  // taps per wave (27 taps over 4 waves)
    f32x4 acc[NT][CT];
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[q][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int br = blockIdx.x; br < nbricks; br += gridDim.x) {
        const int x0 = (br % bxn) * BX, y0 = ((br / bxn) % byn) * BY, z0 = (br / (bxn * byn)) * BZ;
        __syncthreads();
        // g brick transposed: gt[o][v], v = (z * BY + y) * BX + x
        for (int u = tid; u < 256 * (p.cout / 8); u += 256) {
            const int v = u / (p.cout / 8), og = u - v * (p.cout / 8);
            const int gx = x0 + (v % BX), gy = y0 + (v / BX) % BY, gz = z0 + v / (BX * BY);
            uint4 val = {0u, 0u, 0u, 0u};
            if (gx < p.nx && gy < p.ny && gz < p.nz)
                val = *(const uint4*)(p.g + (((int64_t)gz * p.ny + gy) * p.nx + gx) * p.cout + og * 8);
            const bf16_t* e = (const bf16_t*)&val;
#pragma unroll
            for (int q = 0; q < 8; ++q) gt[(og * 8 + q) * 256 + v] = e[q];
        }
        // input halo brick, channels [c0, c0+16), transposed: xt[c][hz][hy][hx]
        for (int u = tid; u < HV * 2; u += 256) {
            const int hv = u >> 1, cg = u & 1;
            const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
            int gx = x0 + hx - 1, gy = y0 + hy - 1;
            const int gz = z0 + hz - 1;
            gx = gx < 0 ? gx + p.nx : (gx >= p.nx ? gx - p.nx : gx);
            gy = gy < 0 ? gy + p.ny : (gy >= p.ny ? gy - p.ny : gy);
            const int ch = c0 + cg * 8;
            uint4 val = {0u, 0u, 0u, 0u};
            // past the periodic image (a brick wider than the grid): zero, as its gradient is
            if (gz >= 0 && gz < p.nz && gx >= 0 && gx < p.nx && gy >= 0 && gy < p.ny && ch < cin) {
                if (ch < p.ca) {
                    int ax = gx, ay = gy, az = gz;
                    if (p.a_up) { ax >>= 1; ay >>= 1; az >>= 1; }
                    val = *(const uint4*)(p.a + (((int64_t)az * any + ay) * anx + ax) * p.ca + ch);
                } else {
                    val = *(const uint4*)(p.b + (((int64_t)gz * p.ny + gy) * p.nx + gx) * p.cb + (ch - p.ca));
                }
            }
            const bf16_t* e = (const bf16_t*)&val;
#pragma unroll
            for (int q = 0; q < 8; ++q) xt[((cg * 8 + q) * HZ * HY + hz * HY + hy) * XROW + hx] = e[q];
        }
        __syncthreads();
        // 8 K steps of 32 voxels: lane group grp covers voxels 32s + 8grp .. +7 (one row half)
#pragma unroll 1
        for (int s = 0; s < 8; ++s) {
            const int v0 = s * 32 + grp * 8;
            const int vz = v0 / (BX * BY), vy = (v0 / BX) % BY, vx = v0 % BX;
            bf16x8 af[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                af[ct] = as_bf8(*(const uint4*)&gt[(ct * 16 + li) * 256 + v0]);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                const int tap = wave + 4 * q;
                if (tap < 27) {
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    const bf16_t* row = &xt[(li * HZ * HY + (vz + dz) * HY + (vy + dy)) * XROW];
                    const uint4 lo = *(const uint4*)(row + vx);
                    const uint4 hi = *(const uint4*)(row + vx + 8);
                    uint4 xv;
                    if (dx == 0) {
                        xv = lo;
                    } else if (dx == 1) {
                        xv.x = __builtin_amdgcn_alignbit(lo.y, lo.x, 16);
                        xv.y = __builtin_amdgcn_alignbit(lo.z, lo.y, 16);
                        xv.z = __builtin_amdgcn_alignbit(lo.w, lo.z, 16);
                        xv.w = __builtin_amdgcn_alignbit(hi.x, lo.w, 16);
                    } else {
                        xv.x = lo.y;
                        xv.y = lo.z;
                        xv.z = lo.w;
                        xv.w = hi.x;
                    }
                    const bf16x8 bf = as_bf8(xv);
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
                        acc[q][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[ct], bf, acc[q][ct], 0, 0, 0);
                }
            }
        }
    }
    // lane holds D[o = ct*16 + 4*grp + e][c = li] for tap wave + 4q
    float* out = p.partial + ((int64_t)blockIdx.x * gridDim.y + chunk) * (int64_t)p.cout * 27 * 16;
#pragma unroll
    for (int q = 0; q < NT; ++q) {
        const int tap = wave + 4 * q;
        if (tap >= 27) continue;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = ct * 16 + 4 * grp + e;
                out[((int64_t)o * 27 + tap) * 16 + li] = acc[q][ct][e];
            }
    }
}

// sum the per-workgroup partials in a fixed order into the flat gradient W[o][t][c] (c < creal)
__global__ void k_reduce_dw(const float* __restrict__ partial, int nparts, int nchunks, int cout,
                            int creal, float* __restrict__ gw) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // over cout * 27 * creal
    if (idx >= cout * 27 * creal) return;
    const int c = idx % creal, t = (idx / creal) % 27, o = idx / (creal * 27);
    const int chunk = c / 16, cl = c % 16;
    double s = 0.0;
    for (int q = 0; q < nparts; ++q)
        s += partial[(((int64_t)q * nchunks + chunk) * cout * 27 + (int64_t)o * 27 + t) * 16 + cl];
    gw[idx] = (float)s;
}

// ------------------------------------------------------------------------------------------
// elementwise and small kernels

// network input: [b/s, log rho, log c2, p_prev/s, 0, 0, 0, 0] in bf16; s = sqrt(scal[0])
// (c2 may be null: then log c2 = -log(rho m) from the mass term m = 1/(rho c2))
// Position of natural-order cell v in the red-black split storage of an nx x ny x nz level (each x
// row holds its red cells, then its black cells; nx even): where the solver keeps its finest-level
// vectors.
__device__ __forceinline__ int64_t split_pos(int64_t v, int nx, int ny) {
    const int64_t row = v / nx;
    const int i = (int)(v - row * nx);
    const int j = (int)(row % ny);
    const int64_t k = row / ny;
    const int c = (int)((i + j + k) & 1);
    return row * nx + c * (nx >> 1) + (i >> 1);
}

// b and pprev in natural order or (split != 0) in the split storage of the nx x ny grid; rho,
// c2 and m always in natural order
__global__ void k_features(const double* __restrict__ b, const double* __restrict__ rho,
                           const double* __restrict__ c2, const double* __restrict__ m,
                           const double* __restrict__ pprev, const double* __restrict__ ss,
                           bf16_t* __restrict__ out, int64_t n, int split, int nx, int ny) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int64_t vb = split ? split_pos(v, nx, ny) : v;
    const double inv = 1.0 / ss[1];
    const double lc2 = c2 ? log(c2[v]) : -log(rho[v] * m[v]);
    uint4 pk;
    pk.x = (unsigned)f2bf((float)(b[vb] * inv)) | ((unsigned)f2bf((float)log(rho[v])) << 16);
    pk.y = (unsigned)f2bf((float)lc2) | ((unsigned)f2bf((float)(pprev ? pprev[vb] * inv : 0.0)) << 16);
    pk.z = 0u;
    pk.w = 0u;
    *(uint4*)(out + v * 8) = pk;
}

// scale: ss[0] = sum b^2 (from a reduction), ss[1] = sqrt(mean b^2) (1 when b = 0)
__global__ void k_scale(double* ss, double n) {
    const double m = ss[0] / n;
    ss[1] = m > 0.0 ? sqrt(m) : 1.0;
}

__global__ void k_sumsq_partial(const double* __restrict__ b, int64_t n, double* partial) {
    double acc = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        acc += b[v] * b[v];
    __shared__ double ws[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ void k_sum_partials(const double* partial, int n, double* out) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) acc += partial[q];
    __shared__ double ws[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) *out = ws[0] + ws[1] + ws[2] + ws[3];
}

// 2x2x2 mean (bf16 in/out), coarse dims (cx, cy, cz), c channels (a multiple of 8): one thread
// per coarse voxel and 8-channel group, 16-byte loads
__global__ void k_pool(const bf16_t* __restrict__ in, bf16_t* __restrict__ out, int cx, int cy,
                       int cz, int c) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int cg = c >> 3;
    const int64_t total = (int64_t)cx * cy * cz * cg;
    if (idx >= total) return;
    const int g = (int)(idx % cg);
    const int64_t v = idx / cg;
    const int x = (int)(v % cx), y = (int)((v / cx) % cy), z = (int)(v / ((int64_t)cx * cy));
    const int fx = 2 * cx, fy = 2 * cy;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t fv = ((int64_t)(2 * z + (q >> 2)) * fy + (2 * y + ((q >> 1) & 1))) * fx + (2 * x + (q & 1));
        const uint4 w = *(const uint4*)(in + fv * c + 8 * g);
        const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            s[2 * e] += __uint_as_float(u[e] << 16);
            s[2 * e + 1] += __uint_as_float(u[e] & 0xffff0000u);
        }
    }
    uint4 r;
    r.x = pack_bf2(s[0] * 0.125f, s[1] * 0.125f);
    r.y = pack_bf2(s[2] * 0.125f, s[3] * 0.125f);
    r.z = pack_bf2(s[4] * 0.125f, s[5] * 0.125f);
    r.w = pack_bf2(s[6] * 0.125f, s[7] * 0.125f);
    *(uint4*)(out + v * c + 8 * g) = r;
}

// gradient of pool: g_fine[v][c] += g_coarse[v/2][c] / 8   (FP32)
__global__ void k_pool_bwd_add(const float* __restrict__ gc, float* __restrict__ gf, int fx, int fy,
                               int fz, int c) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)fx * fy * fz * c;
    if (idx >= total) return;
    const int ch = (int)(idx % c);
    const int64_t v = idx / c;
    const int x = (int)(v % fx), y = (int)((v / fx) % fy), z = (int)(v / ((int64_t)fx * fy));
    const int64_t cv = ((int64_t)(z >> 1) * (fy >> 1) + (y >> 1)) * (fx >> 1) + (x >> 1);
    gf[idx] += gc[cv * c + ch] * 0.125f;
}

// split the backward-data result of a concatenated input: channels [0, ca) go to ga (summed over
// the 8 children when that input was upsampled: ga has the coarse size), channels [ca, ca+cb)
// are added to gb.
__global__ void k_split_grad(const float* __restrict__ gin, int ca, int cb, int a_up,
                             float* __restrict__ ga, float* __restrict__ gb, int nx, int ny, int nz) {
    const int cin = ca + cb;
    if (a_up) {
        const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
        const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const int64_t total_a = (int64_t)cx * cy * cz * ca;
        if (idx < total_a) {
            const int ch = (int)(idx % ca);
            const int64_t v = idx / ca;
            const int x = (int)(v % cx), y = (int)((v / cx) % cy), z = (int)(v / ((int64_t)cx * cy));
            float s = 0.f;
            for (int q = 0; q < 8; ++q) {
                const int64_t fv = ((int64_t)(2 * z + (q >> 2)) * ny + (2 * y + ((q >> 1) & 1))) * nx + (2 * x + (q & 1));
                s += gin[fv * cin + ch];
            }
            ga[idx] = s;
        }
    }
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (int64_t)nx * ny * nz;
    if (cb > 0 && idx < nv * cb) {
        const int ch = (int)(idx % cb);
        const int64_t v = idx / cb;
        gb[idx] += gin[v * cin + ca + ch];
    }
    if (!a_up && idx < nv * ca) {
        const int ch = (int)(idx % ca);
        const int64_t v = idx / ca;
        ga[idx] = gin[v * cin + ch];
    }
}

// ReLU backward: gp = g * (out > 0) as bf16 (MFMA operand); per-workgroup channel sums of gp
// (bias gradient partials, partial[block][c])
__global__ void k_relu_bwd(const float* __restrict__ g, const bf16_t* __restrict__ out,
                           bf16_t* __restrict__ gp, int64_t nv, int c, float* __restrict__ partial) {
    __shared__ float sums[256];
    const int tid = threadIdx.x;
    // each thread handles channel (tid % c) of voxels strided: c divides 256
    const int ch = tid % c, vstep = 256 / c;
    float acc = 0.f;
    const int64_t vpb = 64;  // voxels per workgroup
    const int64_t v0 = (int64_t)blockIdx.x * vpb;
    for (int64_t v = v0 + tid / c; v < v0 + vpb && v < nv; v += vstep) {
        const int64_t i = v * c + ch;
        const float val = bf2f(out[i]) > 0.f ? g[i] : 0.f;
        const bf16_t h = f2bf(val);
        gp[i] = h;
        acc += val;
    }
    sums[tid] = acc;
    __syncthreads();
    if (tid < c) {
        float s = 0.f;
        for (int q = tid; q < 256; q += c) s += sums[q];
        partial[(int64_t)blockIdx.x * c + tid] = s;
    }
}

// column sums of partial[nrows][c]: one workgroup per column, fixed-order tree
__global__ __launch_bounds__(256) void k_reduce_cols(const float* __restrict__ partial, int nrows, int c,
                                                     float* __restrict__ out) {
    __shared__ double sm[256];
    const int ch = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int q = tid; q < nrows; q += 256) s += partial[(int64_t)q * c + ch];
    sm[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) sm[tid] += sm[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[ch] = (float)sm[0];
}

// head: y[v] = sum_c d1[v][c] w[c] + b
__global__ void k_head(const bf16_t* __restrict__ d1, const float* __restrict__ wb, float* __restrict__ y,
                       int64_t nv) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    float s = wb[HEAD];
#pragma unroll
    for (int c = 0; c < HEAD; ++c) s += bf2f(d1[v * HEAD + c]) * wb[c];
    y[v] = s;
}

// loss = mean (y - t)^2 ; gy = 2 (y - t) / n ; block partial sums of the squared error
__global__ void k_loss(const float* __restrict__ y, const float* __restrict__ t, float* __restrict__ gy,
                       int64_t n, double* __restrict__ partial) {
    double acc = 0.0;
    const double inv = 2.0 / (double)n;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)y[v] - (double)t[v];
        acc += d * d;
        gy[v] = (float)(d * inv);
    }
    __shared__ double ws[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// head backward: gd1[v][c] = gy[v] w[c]; partial[block][c] = sum_v gy d1[v][c]; partial[.][16] = sum gy
__global__ void k_head_bwd(const float* __restrict__ gy, const bf16_t* __restrict__ d1,
                           const float* __restrict__ wb, float* __restrict__ gd1, int64_t nv,
                           float* __restrict__ partial) {
    __shared__ float sums[17][64];
    const int tid = threadIdx.x;  // 64 threads, one voxel each per step
    float acc[17];
#pragma unroll
    for (int c = 0; c < 17; ++c) acc[c] = 0.f;
    const int64_t vpb = 256;
    const int64_t v0 = (int64_t)blockIdx.x * vpb;
    for (int64_t v = v0 + tid; v < v0 + vpb && v < nv; v += 64) {
        const float g = gy[v];
#pragma unroll
        for (int c = 0; c < HEAD; ++c) {
            gd1[v * HEAD + c] = g * wb[c];
            acc[c] += g * bf2f(d1[v * HEAD + c]);
        }
        acc[16] += g;
    }
#pragma unroll
    for (int c = 0; c < 17; ++c) sums[c][tid] = acc[c];
    __syncthreads();
    if (tid < 17) {
        float s = 0.f;
        for (int q = 0; q < 64; ++q) s += sums[tid][q];
        partial[(int64_t)blockIdx.x * 17 + tid] = s;
    }
}

// x_out = scale * y (scale = s * out_scale), FP64 output
// x (natural order, or split storage with split != 0) = s * out_scale * y
__global__ void k_output(const float* __restrict__ y, const double* __restrict__ ss, double oscale,
                         double* __restrict__ x, int64_t n, int split, int nx, int ny) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) x[split ? split_pos(v, nx, ny) : v] = (double)y[v] * ss[1] * oscale;
}

__global__ void k_output_minus(const float* __restrict__ y, const double* __restrict__ ss, double oscale,
                               const double* __restrict__ x, double* __restrict__ d, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) d[v] = (double)y[v] * ss[1] * oscale - x[v];
}

__global__ void k_scaled_grad(const double* __restrict__ q, const double* __restrict__ ss, double oscale,
                              double coef, float* __restrict__ gy, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) gy[v] = (float)(coef * ss[1] * oscale * q[v]);
}

// target in network units: t = x / (s * out_scale)
__global__ void k_target(const double* __restrict__ x, const double* __restrict__ ss, double oscale,
                         float* __restrict__ t, int64_t n) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) t[v] = (float)(x[v] / (ss[1] * oscale));
}

// FP32 master parameters -> bf16 forward weights [o][27*cinp] (zero padded channels) and
// backward-data weights [c][27*o] (flipped taps, transposed channels)
__global__ void k_pack(const float* __restrict__ w, int cin, int cinp, int cout,
                       bf16_t* __restrict__ wf, bf16_t* __restrict__ wbk) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // over cout * 27 * cinp
    if (idx >= cout * 27 * cinp) return;
    const int c = idx % cinp, t = (idx / cinp) % 27, o = idx / (cinp * 27);
    const float val = c < cin ? w[((int64_t)o * 27 + t) * cin + c] : 0.f;
    const bf16_t h = f2bf(val);
    wf[idx] = h;
    if (c < cin) wbk[((int64_t)c * 27 + (26 - t)) * cout + o] = h;
}

// Adam (Kingma and Ba) with bias correction, FP32 state
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_zero_f32(float* x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

// ------------------------------------------------------------------------------------------
// host side

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

struct Level {
    int nx, ny, nz;
    int64_t nv;
};

}  // namespace hpnn

using namespace hpnn;

struct hp_net {
    hipStream_t stream = nullptr;
    Level lv[3];
    int training = 0;
    int64_t nparam = 0;
    int64_t woff[NCONV], boff[NCONV], hoff = 0;  // parameter offsets
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    bf16_t *wf[NCONV] = {}, *wbk[NCONV] = {};
    // activations (bf16): input, conv outputs, pools
    bf16_t* x0 = nullptr;
    bf16_t* act[NCONV] = {};
    bf16_t *p1 = nullptr, *p2 = nullptr;
    float* y = nullptr;
    // training buffers
    float *t = nullptr, *gy = nullptr;
    float* gact[NCONV] = {};  // FP32 gradient at each conv output (pre-mask)
    float *gp1 = nullptr, *gp2 = nullptr;
    bf16_t* gpre = nullptr;   // masked gradient (bf16), max size
    float* gin = nullptr;     // backward-data output, max size
    float* wpart = nullptr;   // backward-weight partials
    int64_t wpart_cap = 0;
    float* cpart = nullptr;   // column partials (bias / head)
    int64_t cpart_cap = 0;
    double* ss = nullptr;     // [sum b^2, s, loss]
    double* dpart = nullptr;
    double out_scale = 1.0;
    int step = 0;
    std::vector<void*> allocs;
};

namespace {

thread_local std::string g_nn_err;

int nfail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_nn_err = buf;
    return code;
}

template <typename T>
int nalloc(hp_net* N, T** p, int64_t n) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess)
        return nfail(HP_ENOMEM, "network workspace allocation of %lld elements failed", (long long)n);
    N->allocs.push_back(q);
    *p = (T*)q;
    return HP_OK;
}

int level_of_conv(int l) {
    static const int lvl[NCONV] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0};
    return lvl[l];
}

int check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nfail(HP_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return HP_OK;
}

// returns whether the launch also wrote the 2x2x2 mean into `pool` (one 16-channel output tile
// with two z-slices per wave and bf16 output; else the caller pools)
bool conv_launch(hp_net* N, int l, const bf16_t* a, int ca, int a_up, const bf16_t* b, int cb,
                 const bf16_t* w, const float* bias, void* out, int cout, int relu, bool out_f32,
                 const float* head = nullptr, bf16_t* pool = nullptr) {
    const Level& L = N->lv[level_of_conv(l)];
    ConvArgs p{a, ca, a_up, b, cb, w, bias, out, cout, L.nx, L.ny, L.nz, relu, head, pool};
    const int ct = cout / 16;
    const int cin = ca + cb;
    // two z-slices per wave for the 16-channel outputs (more products per staged brick; four
    // were slower: the larger brick leaves room for fewer workgroups per CU)
    const int g = (cin % 32 == 0) ? 4 : ((cin % 16 == 0) ? 2 : 1);  // 16-byte groups per chunk voxel
    const int spw = (ct == 1 && g <= 2) ? 2 : 1;
    const unsigned blocks = (unsigned)(((L.nx + BX - 1) / BX) * ((L.ny + BY - 1) / BY) *
                                       ((L.nz + 4 * spw - 1) / (4 * spw)));
#define CONV_LAUNCH2(CTV, GV, SV)                                                                    \
    if (out_f32)                                                                                     \
        hipLaunchKernelGGL((k_conv_fwd<CTV, GV, SV, true>), dim3(blocks), dim3(256), 0, N->stream, p); \
    else                                                                                             \
        hipLaunchKernelGGL((k_conv_fwd<CTV, GV, SV, false>), dim3(blocks), dim3(256), 0, N->stream, p);
#define CONV_LAUNCH(CTV, GV)                                                                         \
    if (CTV == 1 && GV <= 2 && spw == 2) { CONV_LAUNCH2(CTV, GV, 2) } else { CONV_LAUNCH2(CTV, GV, 1) }
#define CONV_CASE(CTV)                                                                           \
    case CTV:                                                                                    \
        if (g == 4) { CONV_LAUNCH(CTV, 4) }                                                      \
        else if (g == 2) { CONV_LAUNCH(CTV, 2) }                                                 \
        else { CONV_LAUNCH(CTV, 1) }                                                             \
        break;
    switch (ct) {
        CONV_CASE(1)
        CONV_CASE(2)
        CONV_CASE(3)
        CONV_CASE(4)
        CONV_CASE(6)
        default: break;
    }
#undef CONV_CASE
#undef CONV_LAUNCH
#undef CONV_LAUNCH2
    return pool && ct == 1 && spw == 2 && !out_f32;
}

// conv input tensors of layer l in the forward pass
struct ConvIn {
    const bf16_t* a;
    int ca, a_up;
    const bf16_t* b;
    int cb;
};

ConvIn conv_inputs(hp_net* N, int l) {
    switch (l) {
        case 0: return {N->x0, 8, 0, nullptr, 0};
        case 1: return {N->act[0], 16, 0, nullptr, 0};
        case 2: return {N->p1, 16, 0, nullptr, 0};
        case 3: return {N->act[2], 32, 0, nullptr, 0};
        case 4: return {N->p2, 32, 0, nullptr, 0};
        case 5: return {N->act[4], 64, 0, nullptr, 0};
        case 6: return {N->act[5], 64, 1, N->act[3], 32};
        case 7: return {N->act[6], 32, 0, nullptr, 0};
        case 8: return {N->act[7], 32, 1, N->act[1], 16};
        default: return {N->act[8], 16, 0, nullptr, 0};
    }
}

int pack_weights(hp_net* N) {
    for (int l = 0; l < NCONV; ++l) {
        const int n = COUT[l] * 27 * cin_pad(l);
        hipLaunchKernelGGL(k_pack, dim3(nblk(n)), dim3(256), 0, N->stream, N->theta + N->woff[l],
                           CIN[l], cin_pad(l), COUT[l], N->wf[l], N->wbk[l]);
    }
    return check();
}

int forward_net(hp_net* N) {
    bool pooled1 = false;  // layer 1 wrote pool(e1) in its epilogue
    for (int l = 0; l < NCONV; ++l) {
        if (l == 2 && !pooled1) {
            const Level& L = N->lv[1];
            hipLaunchKernelGGL(k_pool, dim3(nblk(L.nv * 2)), dim3(256), 0, N->stream, N->act[1], N->p1,
                               L.nx, L.ny, L.nz, 16);
        }
        if (l == 4) {
            const Level& L = N->lv[2];
            hipLaunchKernelGGL(k_pool, dim3(nblk(L.nv * 4)), dim3(256), 0, N->stream, N->act[3], N->p2,
                               L.nx, L.ny, L.nz, 32);
        }
        ConvIn in = conv_inputs(N, l);
        // without training the last layer's activation is only needed by the head, which then
        // runs in that convolution's epilogue
        const bool fuse_head = l == NCONV - 1 && !N->training;
        const bool done = conv_launch(N, l, in.a, in.ca, in.a_up, in.b, in.cb, N->wf[l], N->theta + N->boff[l],
                                      fuse_head ? (void*)N->y : (void*)N->act[l], COUT[l], 1, false,
                                      fuse_head ? N->theta + N->hoff : nullptr, l == 1 ? N->p1 : nullptr);
        if (l == 1) pooled1 = done;
    }
    if (N->training) {
        const Level& L = N->lv[0];
        hipLaunchKernelGGL(k_head, dim3(nblk(L.nv)), dim3(256), 0, N->stream, N->act[9],
                           N->theta + N->hoff, N->y, L.nv);
    }
    return check();
}

int rhs_scale(hp_net* N, const double* b) {
    const int64_t n = N->lv[0].nv;
    const int nb = 1024;
    hipLaunchKernelGGL(k_sumsq_partial, dim3(nb), dim3(256), 0, N->stream, b, n, N->dpart);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, N->stream, N->dpart, nb, N->ss);
    hipLaunchKernelGGL(k_scale, dim3(1), dim3(1), 0, N->stream, N->ss, (double)n);
    return check();
}

// backward of one conv layer: gradient at its output gact[l] (FP32, before the ReLU mask) ->
// parameter gradients, and (if l > 0) the gradient of its input written into gin.
int backward_conv(hp_net* N, int l) {
    const Level& L = N->lv[level_of_conv(l)];
    const int co = COUT[l], cinp = cin_pad(l);
    // mask + bias gradient partials
    const int64_t rows = (L.nv + 63) / 64;
    hipLaunchKernelGGL(k_relu_bwd, dim3((unsigned)rows), dim3(256), 0, N->stream, N->gact[l], N->act[l],
                       N->gpre, L.nv, co, N->cpart);
    hipLaunchKernelGGL(k_reduce_cols, dim3(co), dim3(256), 0, N->stream, N->cpart, (int)rows, co,
                       N->grad + N->boff[l]);
    // weight gradient
    ConvIn in = conv_inputs(N, l);
    const int chunks = (cinp + 15) / 16;
    const int nbr = ((L.nx + BX - 1) / BX) * ((L.ny + BY - 1) / BY) * ((L.nz + BZ - 1) / BZ);
    int parts = std::min(nbr, 96);
    BwdWArgs bw{N->gpre, co, in.a, in.ca, in.a_up, in.b, in.cb, N->wpart, L.nx, L.ny, L.nz};
    {
        // channel chunks of 16 (the first layer's 8 padded channels read as 8 + 8 zeros)
        dim3 grid(parts, chunks);
        switch (co / 16) {
            case 1: hipLaunchKernelGGL((k_conv_bwd_w<1>), grid, dim3(256), 0, N->stream, bw); break;
            case 2: hipLaunchKernelGGL((k_conv_bwd_w<2>), grid, dim3(256), 0, N->stream, bw); break;
            default: hipLaunchKernelGGL((k_conv_bwd_w<4>), grid, dim3(256), 0, N->stream, bw); break;
        }
        const int n = co * 27 * CIN[l];
        hipLaunchKernelGGL(k_reduce_dw, dim3(nblk(n)), dim3(256), 0, N->stream, N->wpart, parts, chunks,
                           co, CIN[l], N->grad + N->woff[l]);
    }
    if (l == 0) return check();
    // input gradient: forward conv of the masked gradient with flipped/transposed weights
    conv_launch(N, l, N->gpre, co, 0, nullptr, 0, N->wbk[l], nullptr, N->gin, CIN[l], 0, true);
    return check();
}

}  // namespace

// =============================================================================================
// C ABI of the network

extern "C" {

const char* hp_nn_last_error(void) { return g_nn_err.c_str(); }

long long hp_nn_num_params(void) {
    long long n = 0;
    for (int l = 0; l < NCONV; ++l) n += 27LL * CIN[l] * COUT[l] + COUT[l];
    return n + HEAD + 1;
}

void hp_nn_free(hp_net* N) {
    if (!N) return;
    if (N->stream) (void)hipStreamSynchronize(N->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : N->allocs) (void)hipFree(p);
    delete N;
}

int hp_nn_create(int nx, int ny, int nz, int training, hp_net** out) {
    g_nn_err.clear();
    if (!out) return nfail(HP_EINVAL, "out must be non-null");
    *out = nullptr;
    if (nx < 4 || ny < 4 || nz < 4 || nx % 4 || ny % 4 || nz % 4)
        return nfail(HP_EINVAL, "network grid sizes must be multiples of 4 (got %d x %d x %d)", nx, ny, nz);
    // the convolutions index voxels with 32-bit integers
    if ((int64_t)nx * ny * nz >= ((int64_t)1 << 31))
        return nfail(HP_EINVAL, "network grid of %d x %d x %d cells exceeds 2^31 - 1 cells", nx, ny, nz);
    hp_net* N = new hp_net();
    N->training = training ? 1 : 0;
    for (int q = 0; q < 3; ++q) {
        N->lv[q].nx = nx >> q;
        N->lv[q].ny = ny >> q;
        N->lv[q].nz = nz >> q;
        N->lv[q].nv = (int64_t)(nx >> q) * (ny >> q) * (nz >> q);
    }
    int64_t off = 0;
    for (int l = 0; l < NCONV; ++l) {
        N->woff[l] = off;
        off += 27LL * CIN[l] * COUT[l];
        N->boff[l] = off;
        off += COUT[l];
    }
    N->hoff = off;
    N->nparam = off + HEAD + 1;
    int rc = HP_OK;
    auto bail = [&](int code) {
        hp_nn_free(N);
        return code;
    };
    if ((rc = nalloc(N, &N->theta, N->nparam))) return bail(rc);
    for (int l = 0; l < NCONV; ++l) {
        if ((rc = nalloc(N, &N->wf[l], (int64_t)COUT[l] * 27 * cin_pad(l))) ||
            (rc = nalloc(N, &N->wbk[l], (int64_t)COUT[l] * 27 * cin_pad(l))))
            return bail(rc);
        if ((rc = nalloc(N, &N->act[l], N->lv[level_of_conv(l)].nv * COUT[l]))) return bail(rc);
    }
    const int64_t V = N->lv[0].nv;
    if ((rc = nalloc(N, &N->x0, V * 8)) || (rc = nalloc(N, &N->p1, N->lv[1].nv * 16)) ||
        (rc = nalloc(N, &N->p2, N->lv[2].nv * 32)) || (rc = nalloc(N, &N->y, V)) ||
        (rc = nalloc(N, &N->ss, 4)) || (rc = nalloc(N, &N->dpart, 1024)))
        return bail(rc);
    if (N->training) {
        if ((rc = nalloc(N, &N->grad, N->nparam)) || (rc = nalloc(N, &N->m, N->nparam)) ||
            (rc = nalloc(N, &N->v, N->nparam)) || (rc = nalloc(N, &N->t, V)) || (rc = nalloc(N, &N->gy, V)))
            return bail(rc);
        for (int l = 0; l < NCONV; ++l)
            if ((rc = nalloc(N, &N->gact[l], N->lv[level_of_conv(l)].nv * COUT[l]))) return bail(rc);
        if ((rc = nalloc(N, &N->gp1, N->lv[1].nv * 16)) || (rc = nalloc(N, &N->gp2, N->lv[2].nv * 32)) ||
            (rc = nalloc(N, &N->gpre, V * 16 > N->lv[1].nv * 32 ? V * 16 : N->lv[1].nv * 32)) ||
            (rc = nalloc(N, &N->gin, std::max(V * 48, N->lv[1].nv * 96))))
            return bail(rc);
        N->wpart_cap = 96LL * 6 * 64 * 27 * 16;
        N->cpart_cap = std::max<int64_t>((V + 63) / 64 * 16, (V + 255) / 256 * 17) + 64;
        if ((rc = nalloc(N, &N->wpart, N->wpart_cap)) || (rc = nalloc(N, &N->cpart, N->cpart_cap)))
            return bail(rc);
        hipLaunchKernelGGL(k_zero_f32, dim3(nblk(N->nparam)), dim3(256), 0, 0, N->m, N->nparam);
        hipLaunchKernelGGL(k_zero_f32, dim3(nblk(N->nparam)), dim3(256), 0, 0, N->v, N->nparam);
    }
    hipLaunchKernelGGL(k_zero_f32, dim3(nblk(N->nparam)), dim3(256), 0, 0, N->theta, N->nparam);
    if ((rc = check())) return bail(rc);
    if (hipDeviceSynchronize() != hipSuccess) return bail(nfail(HP_EHIP, "device synchronisation failed"));
    *out = N;
    return HP_OK;
}

int hp_nn_set_stream(hp_net* N, void* stream) {
    if (!N) return nfail(HP_EINVAL, "null network");
    N->stream = (hipStream_t)stream;
    return HP_OK;
}

int hp_nn_set_params(hp_net* N, const float* params) {
    if (!N || !params) return nfail(HP_EINVAL, "null argument");
    if (hipMemcpyAsync(N->theta, params, N->nparam * sizeof(float), hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        return nfail(HP_EHIP, "parameter copy failed");
    return pack_weights(N);
}

int hp_nn_get_params(hp_net* N, float* params) {
    if (!N || !params) return nfail(HP_EINVAL, "null argument");
    if (hipMemcpyAsync(params, N->theta, N->nparam * sizeof(float), hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        return nfail(HP_EHIP, "parameter copy failed");
    return HP_OK;
}

int hp_nn_get_grad(hp_net* N, float* grad) {
    if (!N || !grad || !N->training) return nfail(HP_EINVAL, "null argument or not a training network");
    if (hipMemcpyAsync(grad, N->grad, N->nparam * sizeof(float), hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        return nfail(HP_EHIP, "gradient copy failed");
    return HP_OK;
}

static const char kCkptMagic[8] = {'H', 'P', 'N', 'E', 'T', '0', '1', '\0'};

int hp_nn_save(hp_net* N, const char* path) {
    g_nn_err.clear();
    if (!N || !path) return nfail(HP_EINVAL, "null argument");
    std::vector<float> host((size_t)N->nparam);
    if (hipMemcpyAsync(host.data(), N->theta, N->nparam * sizeof(float), hipMemcpyDeviceToHost, N->stream) !=
            hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess)
        return nfail(HP_EHIP, "parameter copy failed");
    FILE* f = std::fopen(path, "wb");
    if (!f) return nfail(HP_EIO, "cannot open %s for writing", path);
    const int64_t count = N->nparam;
    const double scale = N->out_scale;
    bool ok = std::fwrite(kCkptMagic, 1, 8, f) == 8 && std::fwrite(&count, sizeof count, 1, f) == 1 &&
              std::fwrite(&scale, sizeof scale, 1, f) == 1 &&
              std::fwrite(host.data(), sizeof(float), host.size(), f) == host.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? HP_OK : nfail(HP_EIO, "cannot write %s", path);
}

int hp_nn_load(hp_net* N, const char* path) {
    g_nn_err.clear();
    if (!N || !path) return nfail(HP_EINVAL, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return nfail(HP_EIO, "cannot open %s", path);
    char magic[8];
    int64_t count = -1;
    double scale = 0.0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kCkptMagic, 8) == 0 &&
              std::fread(&count, sizeof count, 1, f) == 1 && std::fread(&scale, sizeof scale, 1, f) == 1;
    if (!ok || count != N->nparam) {
        std::fclose(f);
        return nfail(HP_EIO, "%s is not a checkpoint of this network (%lld parameters expected)", path,
                     (long long)N->nparam);
    }
    std::vector<float> host((size_t)count);
    ok = std::fread(host.data(), sizeof(float), host.size(), f) == host.size();
    std::fclose(f);
    if (!ok) return nfail(HP_EIO, "%s is truncated", path);
    if (!(scale > 0.0) || !std::isfinite(scale)) return nfail(HP_EIO, "%s holds an invalid output scale", path);
    if (hipMemcpyAsync(N->theta, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice, N->stream) !=
            hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess)
        return nfail(HP_EHIP, "parameter copy failed");
    N->out_scale = scale;
    return pack_weights(N);
}

int hp_nn_set_output_scale(hp_net* N, double s) {
    if (!N || !(s > 0.0) || !std::isfinite(s)) return nfail(HP_EINVAL, "output scale must be positive");
    N->out_scale = s;
    return HP_OK;
}

// raw network: input features [voxel][8] bf16 -> y [voxel] FP32
int hp_nn_forward_raw(hp_net* N, const unsigned short* in, float* y) {
    if (!N || !in || !y) return nfail(HP_EINVAL, "null argument");
    if (hipMemcpyAsync(N->x0, in, N->lv[0].nv * 8 * sizeof(bf16_t), hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        return nfail(HP_EHIP, "input copy failed");
    int rc = forward_net(N);
    if (rc) return rc;
    if (hipMemcpyAsync(y, N->y, N->lv[0].nv * sizeof(float), hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        return nfail(HP_EHIP, "output copy failed");
    return HP_OK;
}

// backward pass from the output gradient in gy (FP32, network units) to the parameter gradient
int backward_net(hp_net* N) {
    const Level& L0 = N->lv[0];
    const int64_t V = L0.nv;
    int rc;
    // head
    const int64_t hrows = (V + 255) / 256;
    hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)hrows), dim3(64), 0, N->stream, N->gy, N->act[9],
                       N->theta + N->hoff, N->gact[9], V, N->cpart);
    hipLaunchKernelGGL(k_reduce_cols, dim3(17), dim3(256), 0, N->stream, N->cpart, (int)hrows, 17,
                       N->grad + N->hoff);
    // decoder and encoder in reverse
    const Level& L1 = N->lv[1];
    const Level& L2 = N->lv[2];
    if ((rc = backward_conv(N, 9))) return rc;                 // gin = d(act8) (16 ch, n)
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(V * 16)), dim3(256), 0, N->stream, N->gin, 16, 0, 0,
                       N->gact[8], nullptr, L0.nx, L0.ny, L0.nz);
    if ((rc = backward_conv(N, 8))) return rc;                 // gin = d[up(act7), act1] (48 ch, n)
    hipLaunchKernelGGL(k_zero_f32, dim3(nblk(V * 16)), dim3(256), 0, N->stream, N->gact[1], V * 16);
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(std::max(V * 16, L1.nv * 32))), dim3(256), 0, N->stream,
                       N->gin, 32, 16, 1, N->gact[7], N->gact[1], L0.nx, L0.ny, L0.nz);
    if ((rc = backward_conv(N, 7))) return rc;                 // gin = d(act6) (32 ch, n/2)
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(L1.nv * 32)), dim3(256), 0, N->stream, N->gin, 32, 0, 0,
                       N->gact[6], nullptr, L1.nx, L1.ny, L1.nz);
    if ((rc = backward_conv(N, 6))) return rc;                 // gin = d[up(act5), act3] (96 ch, n/2)
    hipLaunchKernelGGL(k_zero_f32, dim3(nblk(L1.nv * 32)), dim3(256), 0, N->stream, N->gact[3], L1.nv * 32);
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(std::max(L1.nv * 32, L2.nv * 64))), dim3(256), 0, N->stream,
                       N->gin, 64, 32, 1, N->gact[5], N->gact[3], L1.nx, L1.ny, L1.nz);
    if ((rc = backward_conv(N, 5))) return rc;                 // gin = d(act4) (64 ch, n/4)
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(L2.nv * 64)), dim3(256), 0, N->stream, N->gin, 64, 0, 0,
                       N->gact[4], nullptr, L2.nx, L2.ny, L2.nz);
    if ((rc = backward_conv(N, 4))) return rc;                 // gin = d(p2) (32 ch, n/4)
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblk(L1.nv * 32)), dim3(256), 0, N->stream, N->gin, N->gact[3],
                       L1.nx, L1.ny, L1.nz, 32);
    if ((rc = backward_conv(N, 3))) return rc;                 // gin = d(act2) (32 ch, n/2)
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(L1.nv * 32)), dim3(256), 0, N->stream, N->gin, 32, 0, 0,
                       N->gact[2], nullptr, L1.nx, L1.ny, L1.nz);
    if ((rc = backward_conv(N, 2))) return rc;                 // gin = d(p1) (16 ch, n/2)
    hipLaunchKernelGGL(k_pool_bwd_add, dim3(nblk(V * 16)), dim3(256), 0, N->stream, N->gin, N->gact[1],
                       L0.nx, L0.ny, L0.nz, 16);
    if ((rc = backward_conv(N, 1))) return rc;                 // gin = d(act0) (16 ch, n)
    hipLaunchKernelGGL(k_split_grad, dim3(nblk(V * 16)), dim3(256), 0, N->stream, N->gin, 16, 0, 0,
                       N->gact[0], nullptr, L0.nx, L0.ny, L0.nz);
    if ((rc = backward_conv(N, 0))) return rc;
    return check();
}

// mean squared error loss and gradient for the input already in x0 and the target in t
int loss_grad(hp_net* N, double* loss) {
    const int64_t V = N->lv[0].nv;
    int rc = forward_net(N);
    if (rc) return rc;
    const int nb = 1024;
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, N->stream, N->y, N->t, N->gy, V, N->dpart);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, N->stream, N->dpart, nb, N->ss + 2);
    if ((rc = backward_net(N))) return rc;
    if (loss) {
        double h[4];
        if (hipMemcpyAsync(h, N->ss, 4 * sizeof(double), hipMemcpyDeviceToHost, N->stream) != hipSuccess ||
            hipStreamSynchronize(N->stream) != hipSuccess)
            return nfail(HP_EHIP, "loss copy failed");
        *loss = h[2] / (double)V;
    }
    return HP_OK;
}

int adam(hp_net* N, float lr) {
    N->step++;
    const float c1 = 1.0f - powf(0.9f, (float)N->step);
    const float c2 = 1.0f - powf(0.999f, (float)N->step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(N->nparam)), dim3(256), 0, N->stream, N->theta, N->grad, N->m,
                       N->v, N->nparam, lr, c1, c2);
    return pack_weights(N);
}

// network input from (b, rho, c2 or m, p_prev): scale, features into x0
int features(hp_net* N, const double* b, const double* rho, const double* c2, const double* m,
             const double* pprev, int split = 0) {
    int rc = rhs_scale(N, b);
    if (rc) return rc;
    const Level& L = N->lv[0];
    hipLaunchKernelGGL(k_features, dim3(nblk(L.nv)), dim3(256), 0, N->stream, b, rho, c2, m, pprev, N->ss,
                       N->x0, L.nv, split, L.nx, L.ny);
    return check();
}

}  // namespace

extern "C" {

// raw loss and gradient: input features [voxel][8] bf16 and target [voxel] FP32 (network
// units); the gradient goes to the network's gradient buffer (hp_nn_get_grad)
int hp_nn_loss_grad_raw(hp_net* N, const unsigned short* in, const float* target, double* loss) {
    if (!N || !in || !target || !N->training) return nfail(HP_EINVAL, "null argument or not a training network");
    const int64_t V = N->lv[0].nv;
    if (hipMemcpyAsync(N->x0, in, V * 8 * sizeof(bf16_t), hipMemcpyDeviceToDevice, N->stream) != hipSuccess ||
        hipMemcpyAsync(N->t, target, V * sizeof(float), hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        return nfail(HP_EHIP, "input copy failed");
    return loss_grad(N, loss);
}

int hp_nn_adam(hp_net* N, float lr) {
    if (!N || !N->training) return nfail(HP_EINVAL, "not a training network");
    if (!(lr > 0.f)) return nfail(HP_EINVAL, "learning rate must be positive");
    return adam(N, lr);
}

int hp_nn_forward(hp_net* N, const double* b, const double* rho, const double* c2,
                  const double* p_prev, double* x) {
    if (!N || !b || !rho || !c2 || !x) return nfail(HP_EINVAL, "null argument");
    int rc = features(N, b, rho, c2, nullptr, p_prev);
    if (rc) return rc;
    if ((rc = forward_net(N))) return rc;
    const int64_t V = N->lv[0].nv;
    hipLaunchKernelGGL(k_output, dim3(nblk(V)), dim3(256), 0, N->stream, N->y, N->ss, N->out_scale, x, V, 0,
                       N->lv[0].nx, N->lv[0].ny);
    return check();
}

int hp_nn_train_step(hp_net* N, const double* b, const double* rho, const double* c2,
                     const double* p_prev, const double* x_target, float lr, double* loss) {
    if (!N || !b || !rho || !c2 || !x_target || !N->training)
        return nfail(HP_EINVAL, "null argument or not a training network");
    if (!(lr > 0.f)) return nfail(HP_EINVAL, "learning rate must be positive");
    int rc = features(N, b, rho, c2, nullptr, p_prev);
    if (rc) return rc;
    const int64_t V = N->lv[0].nv;
    hipLaunchKernelGGL(k_target, dim3(nblk(V)), dim3(256), 0, N->stream, x_target, N->ss, N->out_scale,
                       N->t, V);
    if ((rc = loss_grad(N, loss))) return rc;
    return adam(N, lr);
}

}  // extern "C"

// ---- used by the solver's learned mode (hp_solver.hip) ----
namespace hp {
int nn_grid(const hp_net* N, int* nx, int* ny, int* nz) {
    *nx = N->lv[0].nx;
    *ny = N->lv[0].ny;
    *nz = N->lv[0].nz;
    return HP_OK;
}
// z = s * out_scale * net(r / s, log rho, -log(rho m), p_prev / s), s = RMS(r)
int nn_apply(hp_net* N, hipStream_t stream, const double* r, const double* rho, const double* m,
             const double* pprev, double* z, int split) {
    N->stream = stream;
    int rc = features(N, r, rho, nullptr, m, pprev, split);
    if (rc) return rc;
    if ((rc = forward_net(N))) return rc;
    const Level& L = N->lv[0];
    hipLaunchKernelGGL(k_output, dim3(nblk(L.nv)), dim3(256), 0, N->stream, N->y, N->ss, N->out_scale, z, L.nv,
                       split, L.nx, L.ny);
    return check();
}
const char* nn_error() { return g_nn_err.c_str(); }

int nn_train_forward(hp_net* N, hipStream_t stream, const double* b, const double* rho,
                     const double* m, const double* pprev) {
    if (!N->training) return nfail(HP_EINVAL, "not a training network");
    N->stream = stream;
    int rc = features(N, b, rho, nullptr, m, pprev);
    if (rc) return rc;
    return forward_net(N);
}

// d = s * out_scale * y - x (physical units, FP64)
int nn_output_minus(hp_net* N, const double* x, double* d) {
    const int64_t V = N->lv[0].nv;
    hipLaunchKernelGGL(k_output_minus, dim3(nblk(V)), dim3(256), 0, N->stream, N->y, N->ss, N->out_scale,
                       x, d, V);
    return check();
}

// gy = coef * s * out_scale * q  (chain rule from physical to network units), then backward + Adam
int nn_train_backward(hp_net* N, const double* q, double coef, float lr) {
    const int64_t V = N->lv[0].nv;
    hipLaunchKernelGGL(k_scaled_grad, dim3(nblk(V)), dim3(256), 0, N->stream, q, N->ss, N->out_scale, coef,
                       N->gy, V);
    int rc = backward_net(N);
    if (rc) return rc;
    return adam(N, lr);
}
}  // namespace hp
