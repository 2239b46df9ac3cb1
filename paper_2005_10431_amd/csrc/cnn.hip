// Learned initial density for the SCF (the warm start that replaces the
// superposition of atomic densities of Sec. 2.1 when it is close enough):
// Gaussian atom features, a three-layer periodic 3x3x3 convolutional network
// (3 -> 16 -> 16 -> 1 channels, ReLU, softplus output rescaled to N_e
// electrons), its gradient for a mean-squared density loss, and Adam.
//
// Layouts: a field of C channels is C x N_d float32, channel-major, grid
// order p = ix + nx (iy + ny iz).  Parameters are one flat float32 vector
// W1 (16,3,27), b1 (16), W2 (16,16,27), b2 (16), W3 (1,16,27), b3 (1) with
// tap index k = 9 (dz+1) + 3 (dy+1) + (dx+1) for the neighbour p + (dx,dy,dz):
//   conv(W, u)[o, p] = b[o] + sum_i sum_k W[o, i, k] u[i, p + d(k)]
// with periodic wrap.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace sg {

namespace {

constexpr int kT = 8;            // output tile edge
constexpr int kH = kT + 2;       // input tile edge (one-point halo)
constexpr int kTile = kT * kT * kT;
constexpr int kHalo = kH * kH * kH;
constexpr int kOff1 = 3 * 16 * 27;             // b1
constexpr int kOff2 = kOff1 + 16;              // W2
constexpr int kOff3 = kOff2 + 16 * 16 * 27;    // b2
constexpr int kOff4 = kOff3 + 16;              // W3
constexpr int kOff5 = kOff4 + 16 * 27;         // b3
constexpr int kNParams = kOff5 + 1;
static_assert(kNParams == 8673, "parameter count");

struct Grid3 {
    int nx, ny, nz, tx, ty, tz;   // grid and tile counts
};

__device__ inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Load the halo tile of C channels starting at grid point (x0-1, y0-1, z0-1).
template <int C>
__device__ inline void load_tile(float* tile, const float* __restrict__ u, long nd, const Grid3& g, int x0, int y0,
                                 int z0) {
    for (int q = threadIdx.x; q < C * kHalo; q += blockDim.x) {
        const int c = q / kHalo, r = q - c * kHalo;
        const int lz = r / (kH * kH), ly = (r / kH) % kH, lx = r % kH;
        const int x = wrap(x0 + lx - 1, g.nx), y = wrap(y0 + ly - 1, g.ny), z = wrap(z0 + lz - 1, g.nz);
        tile[q] = u[(long)c * nd + x + (long)g.nx * (y + (long)g.ny * z)];
    }
}

__device__ inline void tile_origin(const Grid3& g, int& x0, int& y0, int& z0) {
    int b = blockIdx.x;
    const int bx = b % g.tx;
    b /= g.tx;
    const int by = b % g.ty;
    const int bz = b / g.ty;
    x0 = bx * kT;
    y0 = by * kT;
    z0 = bz * kT;
}

}  // namespace

// MODE 0: out = act(conv(W, in) + b) with ReLU when RELU.
// MODE 1: transposed: out[j, p] = mask[j, p] > 0 ? sum_o sum_k W[o, j, 26-k] in[o, p + d(k)] : 0
//         (the input gradient of a forward layer with weights W (CO x CI),
//          masked by that layer's ReLU input activation).
template <int CI, int CO, int MODE, bool RELU>
__global__ __launch_bounds__(512) void k_conv(const float* __restrict__ in, const float* __restrict__ W,
                                              const float* __restrict__ bias, const float* __restrict__ mask,
                                              float* __restrict__ out, Grid3 g) {
    __shared__ float tile[CI * kHalo];
    const long nd = (long)g.nx * g.ny * g.nz;
    int x0, y0, z0;
    tile_origin(g, x0, y0, z0);
    load_tile<CI>(tile, in, nd, g, x0, y0, z0);
    __syncthreads();
    const int t = threadIdx.x;
    const int lx = t % kT, ly = (t / kT) % kT, lz = t / (kT * kT);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    if (x >= g.nx || y >= g.ny || z >= g.nz) return;
    float acc[CO];
#pragma unroll
    for (int o = 0; o < CO; ++o) acc[o] = (MODE == 0) ? bias[o] : 0.0f;
    for (int i = 0; i < CI; ++i) {
        const float* ti = tile + i * kHalo;
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            const int dz = k / 9, dy = (k / 3) % 3, dx = k % 3;
            const float v = ti[(lz + dz) * kH * kH + (ly + dy) * kH + (lx + dx)];
#pragma unroll
            for (int o = 0; o < CO; ++o) {
                const float w = (MODE == 0) ? W[(o * CI + i) * 27 + k] : W[(i * CO + o) * 27 + (26 - k)];
                acc[o] = fmaf(w, v, acc[o]);
            }
        }
    }
    const long p = x + (long)g.nx * (y + (long)g.ny * z);
#pragma unroll
    for (int o = 0; o < CO; ++o) {
        float r = acc[o];
        if (MODE == 0 && RELU) r = fmaxf(r, 0.0f);
        if (MODE == 1) r = (mask[(long)o * nd + p] > 0.0f) ? r : 0.0f;
        out[(long)o * nd + p] = r;
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// The 16 -> 16 layer (either MODE of k_conv) as an implicit GEMM on the FP32
// matrix cores: D[o][p] = sum over (tap, i) of A[o][tap, i] B[tap, i][p], A
// the weights (M = 16 output channels), B channel i at p + d(tap) (N = 16
// points), K = 27 taps x 16 channels in steps of four channels of one tap
// (MFMA 16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]; register
// r of lane l receives D[4 (l/16) + r][l%16]).  K-step (tap, g) takes the
// channels i = 4 g + l/16.
//
// Output tiles are 8 x 8 x TZ made of 16-point blocks, an x-row at two
// consecutive z; wave w owns the four blocks at y = 4 (w % 2) + j (j < 4)
// and z = 2 (w / 2) + {0, 1}.  LDS holds the halo tile as float4 of the
// channels i % 4 + {0, 4, 8, 12} per point (one plane of channel quad
// i % 4 after another) and the weights as wq[tap][lane] = float4 over g, so
// that one 16-byte read at a per-lane base plus a compile-time offset gives
// a lane its operands for the four K-steps of a tap.
//
// The workgroups are persistent: the weights are staged once; while a tile
// is computed, the previous tile's results are stored and this tile's mask
// read (first taps) and the next tile's halo is loaded into registers (last
// taps), two accesses per tap, so that no wait on memory stands between the
// tiles' MFMAs; operands are read two taps ahead of their MFMAs, the taps
// kept apart by scheduling barriers.
template <int TZ>
struct Conv16Shape {
    static constexpr int NT = 64 * TZ;                 // threads
    static constexpr int PQ = kH * kH;                 // plane pitch (float4)
    static constexpr int NH = (TZ + 2) * kH * kH;      // halo points (= channel-quad stride)
    static constexpr int NQ = (NH + NT - 1) / NT;      // halo points per thread
    static constexpr int NL = NQ * 16;                 // halo loads per thread
    static_assert(TZ % 2 == 0 && NL <= 2 * 27 && NL % 2 == 0, "two halo loads per tap");
};

template <int TZ, int MODE, bool RELU>
__global__ __launch_bounds__(64 * TZ) void k_conv16_mfma(const float* __restrict__ in, const float* __restrict__ W,
                                                         const float* __restrict__ bias,
                                                         const float* __restrict__ mask, float* __restrict__ out,
                                                         Grid3 g, int ntile) {
    using S = Conv16Shape<TZ>;
    __shared__ float4 tile4[4 * S::NH];
    __shared__ float4 wq[27 * 64];
    const long nd = (long)g.nx * g.ny * g.nz;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, pl = lane & 15;
    float bo[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bo[r] = MODE == 0 ? bias[4 * (lane >> 4) + r] : 0.0f;
    // grid offsets of this thread's halo points in a tile
    auto halo_offsets = [&](int tile, long (&gp)[S::NQ]) {
        const int x0 = (tile % g.tx) * kT;
        const int y0 = ((tile / g.tx) % g.ty) * kT;
        const int z0 = (tile / (g.tx * g.ty)) * TZ;
#pragma unroll
        for (int i = 0; i < S::NQ; ++i) {
            // threads past the halo re-read its last point (the value is unused)
            const int q = min((int)threadIdx.x + i * S::NT, S::NH - 1);
            const int lz = q / (kH * kH), ly = (q / kH) % kH, lx = q % kH;
            gp[i] = wrap(x0 + lx - 1, g.nx) +
                    (long)g.nx * (wrap(y0 + ly - 1, g.ny) + (long)g.ny * wrap(z0 + lz - 1, g.nz));
        }
    };
    float hr[S::NQ][16];
    long gp[S::NQ];
    // results of the previous tile (block j, register r) and their grid
    // points, stored during the next tile's first taps
    float res[4][4];
    long pp[4];
    int vp = 0;   // bit j: block j of the previous tile lies in the grid
    {
        // destination order: consecutive threads write consecutive floats
        float* wf = reinterpret_cast<float*>(wq);
        for (int d = threadIdx.x; d < 27 * 64 * 4; d += S::NT) {
            const int gq = d & 3, ln = (d >> 2) & 63, tap = d >> 8;
            const int o = ln & 15, ci = 4 * gq + (ln >> 4);
            wf[d] = MODE == 0 ? W[(o * 16 + ci) * 27 + tap] : W[(ci * 16 + o) * 27 + 26 - tap];
        }
    }
    int t = blockIdx.x;
    if (t < ntile) {
        halo_offsets(t, gp);
#pragma unroll
        for (int i = 0; i < S::NQ; ++i)
#pragma unroll
            for (int c = 0; c < 16; ++c) hr[i][c] = in[c * nd + gp[i]];
    }
    for (; t < ntile; t += gridDim.x) {
        __syncthreads();   // the previous tile's reads of the halo are done
#pragma unroll
        for (int i = 0; i < S::NQ; ++i) {
            const int q = threadIdx.x + i * S::NT;
            if (i * S::NT + S::NT <= S::NH || q < S::NH) {
#pragma unroll
                for (int cq = 0; cq < 4; ++cq)
                    tile4[cq * S::NH + q] = make_float4(hr[i][cq], hr[i][cq + 4], hr[i][cq + 8], hr[i][cq + 12]);
            }
        }
        __syncthreads();
        // the last tile re-reads its own halo (branch-free; values unused)
        halo_offsets(t + (int)gridDim.x < ntile ? t + (int)gridDim.x : t, gp);
        const float4* bp =
            tile4 + (lane >> 4) * S::NH + (2 * (wv >> 1) + (pl >> 3)) * S::PQ + 4 * (wv & 1) * kH + (pl & 7);
        const float4* wp = wq + lane;
        long pc[4];
        int vc = 0;
        {
            const int x = (t % g.tx) * kT + (pl & 7);
            const int y0 = ((t / g.tx) % g.ty) * kT + 4 * (wv & 1);
            const int z = (t / (g.tx * g.ty)) * TZ + 2 * (wv >> 1) + (pl >> 3);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool in_grid = x < g.nx && y0 + j < g.ny && z < g.nz;
                pc[j] = in_grid ? x + (long)g.nx * (y0 + j + (long)g.ny * z) : 0;
                vc |= (int)in_grid << j;
            }
        }
        float mk[4][4];
        f32x4 acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[j][r] = bo[r];
        constexpr int kPipe = 2;
        float4 oa[kPipe + 1], ob[kPipe + 1][4];
        auto operands = [&](int tap, float4& a, float4 (&v)[4]) {
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
            a = wp[tap * 64];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = bp[j * kH + dz * S::PQ + dy * kH + dx];
        };
#pragma unroll
        for (int tap = 0; tap < kPipe; ++tap) operands(tap, oa[tap], ob[tap]);
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            if (tap + kPipe < 27)
                operands(tap + kPipe, oa[(tap + kPipe) % (kPipe + 1)], ob[(tap + kPipe) % (kPipe + 1)]);
            if (tap < 8) {
                // the previous tile's results, then this tile's mask
#pragma unroll
                for (int e = 2 * tap; e < 2 * tap + 2; ++e) {
                    const int j = e >> 2, r = e & 3;
                    if (vp >> j & 1) out[(long)(4 * (lane >> 4) + r) * nd + pp[j]] = res[j][r];
                    if (MODE == 1) mk[j][r] = mask[(long)(4 * (lane >> 4) + r) * nd + pc[j]];
                }
            }
            if (tap >= 27 - S::NL / 2) {
#pragma unroll
                for (int h = 2 * (tap - (27 - S::NL / 2)); h < 2 * (tap - (27 - S::NL / 2)) + 2; ++h)
                    hr[h >> 4][h & 15] = in[(h & 15) * nd + gp[h >> 4]];
            }
            const float4 a = oa[tap % (kPipe + 1)];
            const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
            for (int gq = 0; gq < 4; ++gq)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 v = ob[tap % (kPipe + 1)][j];
                    const float bv = gq == 0 ? v.x : gq == 1 ? v.y : gq == 2 ? v.z : v.w;
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[gq], bv, acc[j], 0, 0, 0);
                }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[j][r];
                if (MODE == 0 && RELU) v = fmaxf(v, 0.0f);
                if (MODE == 1) v = mk[j][r] > 0.0f ? v : 0.0f;
                res[j][r] = v;
            }
            pp[j] = pc[j];
        }
        vp = vc;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (vp >> j & 1) out[(long)(4 * (lane >> 4) + r) * nd + pp[j]] = res[j][r];
}

// Per-tile partial gradients of one layer.  Work item j < CI*27 owns the
// taps (i = j / 27, k = j % 27) for every output channel, item CI*27 + o the
// bias of channel o; S threads share an item, thread s summing the tile
// points [s 512/S, (s+1) 512/S) in order, and the S partial sums are then
// added in increasing s.  part[tile][CO*CI*27 + CO] in the parameter order.
template <int CI, int CO, int S>
__global__ __launch_bounds__(1024) void k_wgrad(const float* __restrict__ u, const float* __restrict__ gr,
                                                float* __restrict__ part, Grid3 g) {
    constexpr int NI = CI * 27 + CO;   // work items
    extern __shared__ float lds_wg[];
    float* ut = lds_wg;                 // CI * kHalo
    float* gt = lds_wg + CI * kHalo;    // kTile x CO, point-major
    float* red = gt + CO * kTile;       // S * NI * CO partial sums
    const long nd = (long)g.nx * g.ny * g.nz;
    int x0, y0, z0;
    tile_origin(g, x0, y0, z0);
    load_tile<CI>(ut, u, nd, g, x0, y0, z0);
    for (int q = threadIdx.x; q < CO * kTile; q += blockDim.x) {
        const int o = q / kTile, r = q - o * kTile;
        const int x = x0 + r % kT, y = y0 + (r / kT) % kT, z = z0 + r / (kT * kT);
        gt[r * CO + o] =
            (x < g.nx && y < g.ny && z < g.nz) ? gr[(long)o * nd + x + (long)g.nx * (y + (long)g.ny * z)] : 0.0f;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int item = t % NI, sg = t / NI;
    if (sg < S) {
        const int r0 = sg * kTile / S, r1 = (sg + 1) * kTile / S;
        float acc[CO];
#pragma unroll
        for (int o = 0; o < CO; ++o) acc[o] = 0.0f;
        if (item < CI * 27) {
            const int i = item / 27, k = item % 27;
            const int dz = k / 9, dy = (k / 3) % 3, dx = k % 3;
            const float* ui = ut + i * kHalo + dz * kH * kH + dy * kH + dx;
            for (int r = r0; r < r1; ++r) {
                const float v = ui[(r >> 6) * kH * kH + ((r >> 3) & 7) * kH + (r & 7)];
                if constexpr (CO % 4 == 0) {
                    // the point's CO channels as 16-byte reads (gt and r CO are
                    // 16-byte aligned)
                    const float4* g4 = reinterpret_cast<const float4*>(gt + r * CO);
#pragma unroll
                    for (int o4 = 0; o4 < CO / 4; ++o4) {
                        const float4 gv = g4[o4];
                        acc[4 * o4] = fmaf(gv.x, v, acc[4 * o4]);
                        acc[4 * o4 + 1] = fmaf(gv.y, v, acc[4 * o4 + 1]);
                        acc[4 * o4 + 2] = fmaf(gv.z, v, acc[4 * o4 + 2]);
                        acc[4 * o4 + 3] = fmaf(gv.w, v, acc[4 * o4 + 3]);
                    }
                } else {
#pragma unroll
                    for (int o = 0; o < CO; ++o) acc[o] = fmaf(gt[r * CO + o], v, acc[o]);
                }
            }
        } else {
            const int o = item - CI * 27;
            float sum = 0.0f;
            for (int r = r0; r < r1; ++r) sum += gt[r * CO + o];
            acc[0] = sum;
        }
#pragma unroll
        for (int o = 0; o < CO; ++o) red[(sg * NI + item) * CO + o] = acc[o];
    }
    __syncthreads();
    float* pp = part + (long)blockIdx.x * (CO * CI * 27 + CO);
    for (int q = t; q < CI * 27 * CO; q += blockDim.x) {
        // q = item * CO + o; parameter (o, i, k) = (o * CI + i) * 27 + k
        const int it = q / CO, o = q - it * CO;
        float sum = 0.0f;
        for (int s2 = 0; s2 < S; ++s2) sum += red[(s2 * NI + it) * CO + o];
        pp[o * CI * 27 + it] = sum;
    }
    for (int o = t; o < CO; o += blockDim.x) {
        float sum = 0.0f;
        for (int s2 = 0; s2 < S; ++s2) sum += red[(s2 * NI + CI * 27 + o) * CO];
        pp[CO * CI * 27 + o] = sum;
    }
}

// Per-tile partial gradient of the 16 -> 16 layer on the FP32 matrix cores:
// dW[o][i][k] = sum over the tile's points p of gr[o][p] u[i][p + d(k)], a
// GEMM per tap k with M = 16 (o), N = 16 (i) and K = the 512 points in steps
// of four (lane l supplies A[o = l%16][p = 4s + l/16] and
// B[p = 4s + l/16][i = l%16]; register r of lane l receives D[4 (l/16) + r]
// [l%16]).  LDS holds the input halo and the tile of gr point-major (the 16
// channels of a point contiguous), so that both operand reads of a step are
// 64 consecutive floats.  Wave w owns the taps w, w+8, w+16 and, for w < 3,
// w+24; wave 3 adds the bias sum sum_p gr[o][p] as a fourth GEMM against
// ones, so that each SIMD (waves w and w+4) issues seven GEMMs.  Each step's
// gr read serves all of the wave's GEMMs.  part[tile][(o*16 + i)*27 + k],
// bias at part[tile][16*16*27 + o], as k_wgrad<16, 16>.
template <int NSL, bool BIAS>
__device__ inline void wgrad16_gemms(const float* gt, const float* uh, int w, int lane, float* pp) {
    f32x4 acc[NSL];
#pragma unroll
    for (int k = 0; k < NSL; ++k) acc[k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const float* bt[NSL];
#pragma unroll
    for (int k = 0; k < NSL; ++k) {
        const int tap = w + 8 * k, dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        bt[k] = uh + (dz * kH * kH + dy * kH + dx) * 16 + lane;
    }
    const float* at = gt + lane;
#pragma unroll
    for (int s = 0; s < kTile / 4; ++s) {
        // the four points 4s .. 4s+3: x = 4 (s % 2) + l/16, y = (s / 2) % 8, z = s / 16
        const int hp = (s / 16) * kH * kH + ((s / 2) % 8) * kH + 4 * (s % 2);
        const float a = at[64 * s];
#pragma unroll
        for (int k = 0; k < NSL; ++k) {
            const float b = (BIAS && k == NSL - 1) ? 1.0f : bt[k][hp * 16];
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
        }
    }
#pragma unroll
    for (int k = 0; k < NSL; ++k) {
        const int i = lane & 15;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = 4 * (lane >> 4) + r;
            if (BIAS && k == NSL - 1) {
                if (i == 0) pp[16 * 16 * 27 + o] = acc[k][r];
            } else {
                pp[(o * 16 + i) * 27 + w + 8 * k] = acc[k][r];
            }
        }
    }
}

__global__ __launch_bounds__(512) void k_wgrad16_mfma(const float* __restrict__ u, const float* __restrict__ gr,
                                                      float* __restrict__ part, Grid3 g) {
    __shared__ float uh[kHalo * 16];
    __shared__ float gt[kTile * 16];
    const long nd = (long)g.nx * g.ny * g.nz;
    int x0, y0, z0;
    tile_origin(g, x0, y0, z0);
    for (int q = threadIdx.x; q < kHalo; q += blockDim.x) {
        const int lz = q / (kH * kH), ly = (q / kH) % kH, lx = q % kH;
        const long gp = wrap(x0 + lx - 1, g.nx) +
                        (long)g.nx * (wrap(y0 + ly - 1, g.ny) + (long)g.ny * wrap(z0 + lz - 1, g.nz));
        float v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = u[c * nd + gp];
#pragma unroll
        for (int c = 0; c < 16; c += 4)
            *reinterpret_cast<float4*>(uh + q * 16 + c) = make_float4(v[c], v[c + 1], v[c + 2], v[c + 3]);
    }
    {
        const int r = threadIdx.x;   // one tile point per thread
        const int x = x0 + r % kT, y = y0 + (r / kT) % kT, z = z0 + r / (kT * kT);
        const bool in_grid = x < g.nx && y < g.ny && z < g.nz;
        const long p = in_grid ? x + (long)g.nx * (y + (long)g.ny * z) : 0;
        float v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = in_grid ? gr[c * nd + p] : 0.0f;
#pragma unroll
        for (int c = 0; c < 16; c += 4)
            *reinterpret_cast<float4*>(gt + r * 16 + c) = make_float4(v[c], v[c + 1], v[c + 2], v[c + 3]);
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float* pp = part + (long)blockIdx.x * (16 * 16 * 27 + 16);
    if (w < 3)
        wgrad16_gemms<4, false>(gt, uh, w, lane, pp);
    else if (w == 3)
        wgrad16_gemms<4, true>(gt, uh, w, lane, pp);
    else
        wgrad16_gemms<3, false>(gt, uh, w, lane, pp);
}

// grad[off + j] = sum over tiles of part[tile][j] in FP64 and a fixed
// order: thread (j, q) of a 64 x 16 workgroup sums the tiles b = q (mod 16)
// in increasing b, then the 16 partial sums of j are added in increasing q.
constexpr int kRedJ = 64, kRedQ = 16;
__global__ __launch_bounds__(kRedJ* kRedQ) void k_wgrad_reduce(const float* __restrict__ part, int ntiles, int np,
                                                               float* __restrict__ grad) {
    __shared__ double ps[kRedQ][kRedJ];
    const int jl = threadIdx.x % kRedJ, q = threadIdx.x / kRedJ;
    const int j = blockIdx.x * kRedJ + jl;
    double s = 0.0;
    if (j < np)
        for (int b = q; b < ntiles; b += kRedQ) s += (double)part[(long)b * np + j];
    ps[q][jl] = s;
    __syncthreads();
    if (q == 0 && j < np) {
        double t = 0.0;
        for (int k = 0; k < kRedQ; ++k) t += ps[k][jl];
        grad[j] = (float)t;
    }
}

__device__ inline double softplus_d(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }
__device__ inline double sigmoid_d(double z) { return 0.5 * (1.0 + tanh(0.5 * z)); }

// Block partial sums (FP64) of up to 3 quantities; out[block * 3 + q].
__device__ inline void block_reduce3(double a, double b, double c, double* out) {
    __shared__ double red[3][256];
    const int t = threadIdx.x;
    red[0][t] = a;
    red[1][t] = b;
    red[2][t] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
            red[2][t] += red[2][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[blockIdx.x * 3 + 0] = red[0][0];
        out[blockIdx.x * 3 + 1] = red[1][0];
        out[blockIdx.x * 3 + 2] = red[2][0];
    }
}

// out[q] = sum over blocks of part[block * 3 + q]: one workgroup of 256,
// thread t summing the blocks t (mod 256) in increasing order, then the
// fixed tree of block_reduce3.
__global__ __launch_bounds__(256) void k_reduce3_final(const double* part, int nblk, double* out) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q] += part[b * 3 + q];
    block_reduce3(s[0], s[1], s[2], out);
}

// sum of softplus(z)
__global__ __launch_bounds__(256) void k_head_sum(const float* __restrict__ z, long n, double* part) {
    double s = 0.0;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x)
        s += softplus_d((double)z[p]);
    block_reduce3(s, 0.0, 0.0, part);
}

// rho = N_e softplus(z) / (dV S)
__global__ void k_head_rho(const float* __restrict__ z, long n, const double* S, double scale,
                           double* __restrict__ rho) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) rho[p] = scale * softplus_d((double)z[p]) / S[0];
}

// loss = sum (rho - t)^2 / n ; G = sum g s with g = 2 (rho - t) / n
__global__ __launch_bounds__(256) void k_head_loss(const float* __restrict__ z, const double* __restrict__ rho,
                                                   const double* __restrict__ tgt, long n, double* part) {
    double l = 0.0, gs = 0.0;
    const double inv = 1.0 / (double)n;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const double d = rho[p] - tgt[p];
        l += d * d * inv;
        gs += 2.0 * d * inv * softplus_d((double)z[p]);
    }
    block_reduce3(l, gs, 0.0, part);
}

// dz = (c g - (c / S) G) sigmoid(z),  c = N_e / (dV S)
__global__ void k_head_dz(const float* __restrict__ z, const double* __restrict__ rho, const double* __restrict__ tgt,
                          long n, const double* S, const double* LG, double ne_over_dv, float* __restrict__ dz) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double Sv = S[0];
    const double cc = ne_over_dv / Sv;
    const double g = 2.0 * (rho[p] - tgt[p]) / (double)n;
    dz[p] = (float)((cc * g - cc / Sv * LG[1]) * sigmoid_d((double)z[p]));
}

// Gaussian features: channel c at p = sum over atoms and periodic images
// within 6 w_c of exp(-r^2 / (2 w_c^2)).
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ pos, int na, double w0, double w1,
                                                  double w2, int nx, int ny, int nz, double hx, double hy, double hz,
                                                  double Lx, double Ly, double Lz, float* __restrict__ out) {
    const long nd = (long)nx * ny * nz;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nd) return;
    const int ix = (int)(p % nx), iy = (int)((p / nx) % ny), iz = (int)(p / ((long)nx * ny));
    const double X = ix * hx, Y = iy * hy, Z = iz * hz;
    const double ws[3] = {w0, w1, w2};
    for (int c = 0; c < 3; ++c) {
        const double w = ws[c], rcut = 6.0 * w, rc2 = rcut * rcut, i2w2 = 1.0 / (2.0 * w * w);
        const int Kx = (int)ceil((rcut + Lx) / Lx), Ky = (int)ceil((rcut + Ly) / Ly), Kz = (int)ceil((rcut + Lz) / Lz);
        double acc = 0.0;
        for (int a = 0; a < na; ++a) {
            double Rx = fmod(pos[3 * a], Lx), Ry = fmod(pos[3 * a + 1], Ly), Rz = fmod(pos[3 * a + 2], Lz);
            if (Rx < 0.0) Rx += Lx;
            if (Ry < 0.0) Ry += Ly;
            if (Rz < 0.0) Rz += Lz;
            for (int i = -Kx; i <= Kx; ++i) {
                const double dx = (X - Rx) - i * Lx;
                if (fabs(dx) > rcut) continue;
                for (int j = -Ky; j <= Ky; ++j) {
                    const double dy = (Y - Ry) - j * Ly;
                    if (fabs(dy) > rcut) continue;
                    for (int k = -Kz; k <= Kz; ++k) {
                        const double dz = (Z - Rz) - k * Lz;
                        const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(dz, dz), __dmul_rn(dy, dy)), __dmul_rn(dx, dx));
                        if (r2 <= rc2) acc += exp(-r2 * i2w2);
                    }
                }
            }
        }
        out[(long)c * nd + p] = (float)acc;
    }
}

// Adam (Kingma & Ba) on float32 parameters, moments in float32, arithmetic
// in FP64.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, double lr, double b1, double b2, double eps, double c1,
                       double c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
    const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
    m[i] = (float)mi;
    v[i] = (float)vi;
    w[i] = (float)((double)w[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
}

// dV sum |a - b| and the count of non-finite a (into part, then final).
__global__ __launch_bounds__(256) void k_l1(const double* __restrict__ a, const double* __restrict__ b, long n,
                                            double* part) {
    double s = 0.0, bad = 0.0;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (long)gridDim.x * blockDim.x) {
        const double x = a[p];
        if (!isfinite(x)) bad += 1.0;
        else s += fabs(x - b[p]);
    }
    block_reduce3(s, bad, 0.0, part);
}

__global__ void k_copy_d(const double* a, double* b, long n) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) b[p] = a[p];
}

// ------------------------------------------------------------ host side

static Grid3 grid3(sparc_gpu_ctx c) {
    Grid3 g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.nz = c->nz;
    g.tx = div_up(c->nx, kT);
    g.ty = div_up(c->ny, kT);
    g.tz = div_up(c->nz, kT);
    return g;
}

static int ntiles(const Grid3& g) { return g.tx * g.ty * g.tz; }

static sparc_status features_impl(sparc_gpu_ctx c, const double w[3], float* feat) {
    for (int k = 0; k < 3; ++k)
        if (!(w[k] > 0.0) || !std::isfinite(w[k])) return set_err(c, SPARC_ERR_ARG, "features: widths must be > 0");
    if (c->n_atoms > 0 && !c->atom_pos) return set_err(c, SPARC_ERR_ARG, "features: no atoms");
    k_features<<<div_up(c->nd, 256), 256, 0, c->stream>>>(c->atom_pos, c->n_atoms, w[0], w[1], w[2], c->nx, c->ny,
                                                         c->nz, c->hx, c->hy, c->hz, c->Lx, c->Ly, c->Lz, feat);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

// Threads sharing a work item of k_wgrad<CI, CO, S>, and its launch.
template <int CI, int CO>
constexpr int wgrad_split() {
    return CI == 3 ? 5 : 1;
}

template <int CI, int CO>
static void wgrad_launch(sparc_gpu_ctx c, const Grid3& g, const float* u, const float* gr, float* part) {
    constexpr int S = wgrad_split<CI, CO>(), NI = CI * 27 + CO;
    const size_t lds = (size_t)(CI * kHalo + CO * kTile + S * NI * CO) * sizeof(float);
    const int threads = div_up(S * NI, 64) * 64;
    k_wgrad<CI, CO, S><<<ntiles(g), threads, lds, c->stream>>>(u, gr, part, g);
}

// One persistent workgroup per resident slot (LDS sets how many fit on a
// CU; the count is taken once per context), never more than there are tiles.
template <int TZ, int MODE, bool RELU>
static void conv16_launch(sparc_gpu_ctx c, const Grid3& g, const float* in, const float* W, const float* bias,
                          const float* mask, float* out) {
    int& per_cu = c->cnn_per_cu[TZ == 8][MODE];
    if (per_cu == 0 && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv16_mfma<TZ, MODE, RELU>,
                                                                      64 * TZ, 0) != hipSuccess ||
                        per_cu < 1))
        per_cu = 1;
    const int ntile = g.tx * g.ty * div_up(g.nz, TZ);
    const int nb = std::min(ntile, per_cu * c->prop.multiProcessorCount);
    k_conv16_mfma<TZ, MODE, RELU><<<nb, 64 * TZ, 0, c->stream>>>(in, W, bias, mask, out, g, ntile);
}

// The 16 -> 16 layer: the matrix-core kernel on 8 x 8 x cnn_tz tiles, or
// the vector kernel when cnn_tz is 0.
template <int MODE, bool RELU>
static void conv16(sparc_gpu_ctx c, const Grid3& g, const float* in, const float* W, const float* bias,
                   const float* mask, float* out) {
    if (c->cnn_tz == 0)
        k_conv<16, 16, MODE, RELU><<<ntiles(g), 512, 0, c->stream>>>(in, W, bias, mask, out, g);
    else if (c->cnn_tz == 4)
        conv16_launch<4, MODE, RELU>(c, g, in, W, bias, mask, out);
    else
        conv16_launch<8, MODE, RELU>(c, g, in, W, bias, mask, out);
}

// head scalars live in scal[S_CNN .. S_CNN+5]: S, -, -, loss, G, -
static sparc_status forward_impl(sparc_gpu_ctx c, const float* w, const float* feat, float* act, double* rho) {
    const Grid3 g = grid3(c);
    const long nd = c->nd;
    float* a1 = act;
    float* a2 = act + 16 * nd;
    float* z = act + 32 * nd;
    const int nt = ntiles(g);
    const int slot = prof_begin(c, PK_CNN_FWD);
    k_conv<3, 16, 0, true><<<nt, 512, 0, c->stream>>>(feat, w, w + kOff1, nullptr, a1, g);
    const int slot2 = prof_begin(c, PK_CNN_CONV2);
    conv16<0, true>(c, g, a1, w + kOff2, w + kOff3, nullptr, a2);
    prof_end(c, slot2);
    k_conv<16, 1, 0, false><<<nt, 512, 0, c->stream>>>(a2, w + kOff4, w + kOff5, nullptr, z, g);
    SG_CHECK_LAUNCH(c);
    const int nblk = (int)std::min<long>(1024, div_up(nd, 256));
    sparc_status st = ensure_red(c, 3 * (size_t)nblk);
    if (st != SPARC_OK) return st;
    k_head_sum<<<nblk, 256, 0, c->stream>>>(z, nd, c->red);
    k_reduce3_final<<<1, 256, 0, c->stream>>>(c->red, nblk, c->scal + S_CNN);
    k_head_rho<<<div_up(nd, 256), 256, 0, c->stream>>>(z, nd, c->scal + S_CNN, c->n_electrons / c->dV, rho);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    return SPARC_OK;
}

static sparc_status ensure_cnn(sparc_gpu_ctx c, size_t floats) {
    return ensure_work(c, floats * sizeof(float));
}

static sparc_status backward_impl(sparc_gpu_ctx c, const float* w, const float* feat, const float* act,
                                  const double* rho, const double* tgt, float* grad, double* loss) {
    const Grid3 g = grid3(c);
    const long nd = c->nd;
    const float* a1 = act;
    const float* a2 = act + 16 * nd;
    const float* z = act + 32 * nd;
    const int nt = ntiles(g);
    const int np1 = 16 * 3 * 27 + 16, np2 = 16 * 16 * 27 + 16, np3 = 16 * 27 + 1;
    // scratch: dz (nd), d2 (16 nd), d1 (16 nd), partials (nt * np2)
    const size_t need = 33 * (size_t)nd + (size_t)nt * np2;
    sparc_status st = ensure_cnn(c, need);
    if (st != SPARC_OK) return st;
    float* dz = (float*)c->work;
    float* d2 = dz + nd;
    float* d1 = d2 + 16 * nd;
    float* part = d1 + 16 * nd;
    const int nblk = (int)std::min<long>(1024, div_up(nd, 256));
    if ((st = ensure_red(c, 3 * (size_t)nblk)) != SPARC_OK) return st;
    const int slot = prof_begin(c, PK_CNN_BWD);
    // the forward's softplus sum is recomputed so that backward depends only
    // on its arguments
    k_head_sum<<<nblk, 256, 0, c->stream>>>(z, nd, c->red);
    k_reduce3_final<<<1, 256, 0, c->stream>>>(c->red, nblk, c->scal + S_CNN);
    k_head_loss<<<nblk, 256, 0, c->stream>>>(z, rho, tgt, nd, c->red);
    k_reduce3_final<<<1, 256, 0, c->stream>>>(c->red, nblk, c->scal + S_CNN + 3);
    k_head_dz<<<div_up(nd, 256), 256, 0, c->stream>>>(z, rho, tgt, nd, c->scal + S_CNN, c->scal + S_CNN + 3,
                                                      c->n_electrons / c->dV, dz);
    SG_CHECK_LAUNCH(c);
    // layer 3
    wgrad_launch<16, 1>(c, g, a2, dz, part);
    k_wgrad_reduce<<<div_up(np3, kRedJ), kRedJ * kRedQ, 0, c->stream>>>(part, nt, np3, grad + kOff4);
    k_conv<1, 16, 1, false><<<nt, 512, 0, c->stream>>>(dz, w + kOff4, nullptr, a2, d2, g);
    // layer 2
    if (c->cnn_tz == 0)
        wgrad_launch<16, 16>(c, g, a1, d2, part);
    else
        k_wgrad16_mfma<<<nt, 512, 0, c->stream>>>(a1, d2, part, g);
    k_wgrad_reduce<<<div_up(np2, kRedJ), kRedJ * kRedQ, 0, c->stream>>>(part, nt, np2, grad + kOff2);
    conv16<1, false>(c, g, d2, w + kOff2, nullptr, a1, d1);
    // layer 1
    wgrad_launch<3, 16>(c, g, feat, d1, part);
    k_wgrad_reduce<<<div_up(np1, kRedJ), kRedJ * kRedQ, 0, c->stream>>>(part, nt, np1, grad);
    SG_CHECK_LAUNCH(c);
    prof_end(c, slot);
    if (loss)
        SG_HIP(c, hipMemcpyAsync(loss, c->scal + S_CNN + 3, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return SPARC_OK;
}

}  // namespace sg

using namespace sg;

extern "C" {

sparc_status sparc_gpu_features(sparc_gpu_ctx c, const double* widths, float* d_feat) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!widths || !d_feat) return set_err(c, SPARC_ERR_ARG, "features: null pointer");
    return features_impl(c, widths, d_feat);
}

sparc_status sparc_gpu_cnn_forward(sparc_gpu_ctx c, const float* d_w, const float* d_feat, float* d_act,
                                   double* d_rho) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_w || !d_feat || !d_act || !d_rho) return set_err(c, SPARC_ERR_ARG, "cnn_forward: null pointer");
    return forward_impl(c, d_w, d_feat, d_act, d_rho);
}

sparc_status sparc_gpu_cnn_backward(sparc_gpu_ctx c, const float* d_w, const float* d_feat, const float* d_act,
                                    const double* d_rho, const double* d_target, float* d_grad, double* d_loss) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_w || !d_feat || !d_act || !d_rho || !d_target || !d_grad)
        return set_err(c, SPARC_ERR_ARG, "cnn_backward: null pointer");
    return backward_impl(c, d_w, d_feat, d_act, d_rho, d_target, d_grad, d_loss);
}

sparc_status sparc_gpu_adam_step(sparc_gpu_ctx c, float* d_w, const float* d_grad, float* d_m, float* d_v, int n,
                                 int t, double lr, double beta1, double beta2, double eps) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_w || !d_grad || !d_m || !d_v) return set_err(c, SPARC_ERR_ARG, "adam_step: null pointer");
    if (n < 1 || t < 1) return set_err(c, SPARC_ERR_ARG, "adam_step: n and t must be >= 1");
    if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
        return set_err(c, SPARC_ERR_ARG, "adam_step: bad hyper-parameters");
    const double c1 = 1.0 - std::pow(beta1, t), c2 = 1.0 - std::pow(beta2, t);
    k_adam<<<div_up(n, 256), 256, 0, c->stream>>>(d_w, d_grad, d_m, d_v, n, lr, beta1, beta2, eps, c1, c2);
    SG_CHECK_LAUNCH(c);
    return SPARC_OK;
}

sparc_status sparc_gpu_warm_start(sparc_gpu_ctx c, const float* d_w, double max_l1, double* d_rho, int* used_cnn) {
    if (!c) return SPARC_ERR_ARG;
    c->err.clear();
    if (!d_w || !d_rho) return set_err(c, SPARC_ERR_ARG, "warm_start: null pointer");
    if (!(max_l1 >= 0.0)) return set_err(c, SPARC_ERR_ARG, "warm_start: max_l1 must be >= 0");
    const long nd = c->nd;
    // scratch: features (3 nd) + activations (33 nd) floats, SAD in field 0
    sparc_status st = ensure_cnn(c, 36 * (size_t)nd);
    if (st != SPARC_OK) return st;
    if ((st = ensure_fields(c, 6)) != SPARC_OK) return st;
    float* feat = (float*)c->work;
    float* act = feat + 3 * nd;
    double* sad = c->field;
    const double widths[3] = {0.5, 1.0, 2.0};
    if ((st = features_impl(c, widths, feat)) != SPARC_OK) return st;
    if ((st = forward_impl(c, d_w, feat, act, d_rho)) != SPARC_OK) return st;
    if ((st = sparc_gpu_sad_density(c, sad)) != SPARC_OK) return st;
    const int nblk = (int)std::min<long>(1024, div_up(nd, 256));
    if ((st = ensure_red(c, 3 * (size_t)nblk)) != SPARC_OK) return st;
    k_l1<<<nblk, 256, 0, c->stream>>>(d_rho, sad, nd, c->red);
    k_reduce3_final<<<1, 256, 0, c->stream>>>(c->red, nblk, c->scal + S_CNN);
    SG_CHECK_LAUNCH(c);
    double h[3];
    SG_HIP(c, hipMemcpyAsync(h, c->scal + S_CNN, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SG_HIP(c, hipStreamSynchronize(c->stream));
    const double l1 = c->dV * h[0] / c->n_electrons;
    const bool ok = (h[1] == 0.0) && std::isfinite(l1) && l1 <= max_l1;
    if (!ok) {
        k_copy_d<<<div_up(nd, 256), 256, 0, c->stream>>>(sad, d_rho, nd);
        SG_CHECK_LAUNCH(c);
        SG_HIP(c, hipStreamSynchronize(c->stream));
    }
    if (used_cnn) *used_cnn = ok ? 1 : 0;
    return SPARC_OK;
}

}  // extern "C"
