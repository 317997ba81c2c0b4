// Kernels of the per-patch MLP local solver, gfx950.
//
// GEMM: a workgroup of four waves owns a (32 TI) x (32 TJ) tile of C, each
// wave a (16 TI) x (16 TJ) quarter built from 16 x 16 MFMA blocks
// (v_mfma_f32_16x16x32_bf16 for BF16 operands, v_mfma_f32_16x16x4_f32 for FP32
// operands).  Both operand tiles sit in LDS with k contiguous ([row][k]), so
// a lane's fragment (8 consecutive k for BF16) is one 16-byte LDS read; the
// next k-slab is prefetched into registers while the current one is
// multiplied.  Split-K (deterministic: partial tiles, then a sum) keeps the
// long-K weight-gradient products from running on a handful of CUs.
#include "mlp_kernels.hpp"
#include "xcd.hpp"

#include <algorithm>
#include <cmath>

namespace smg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int GBK = 32;     // k per slab
constexpr int GNT = 256;    // threads per workgroup

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

template <typename TOP> struct Op;
template <> struct Op<__bf16> {
    static constexpr int PAD = 8;   // row stride 40 elements = 80 bytes
};
template <> struct Op<float> {
    static constexpr int PAD = 4;   // row stride 36 floats
};

struct GemmArgs {
    int M, N, K;
    const float* A;
    int lda;
    const int* arows;
    const float* B;
    int ldb;
    float* C;
    int ldc;
    const float* bias;
    float* Z;
    int ldz;
    int kslabs_per_split;   // k slabs handled by one blockIdx.z
    size_t split_stride;    // floats between the partial C of consecutive splits
};

// One operand tile of R rows x GBK k, R = 32 T: thread t fetches 16 elements
// (R x GBK / GNT = 16 when T = 4, 8 when T = 2).
template <int R, bool KCONTIG>
struct TileLoader {
    static constexpr int PER = R * GBK / GNT;   // elements per thread
    float v[PER];

    // KCONTIG: element (r, kk) at src[row(r) ld + k0 + kk]; else at src[row(k0 + kk) ld + r0 + r]
    __device__ inline void load(const float* __restrict__ src, int ld, const int* __restrict__ rows, int r0,
                                int rmax, int k0, int kmax, int t) {
        if constexpr (KCONTIG) {
            constexpr int TPR = GBK / PER;           // threads per row
            const int r = t / TPR, kk = (t % TPR) * PER;
            const int gr = r0 + r, gk = k0 + kk;
            if (gr < rmax) {
                const float* p = src + size_t(rows ? rows[gr] : gr) * ld + gk;
                if (gk + PER <= kmax) {
#pragma unroll
                    for (int i = 0; i < PER; i += 4) {
                        const float4 q = *reinterpret_cast<const float4*>(p + i);
                        v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < PER; ++i) v[i] = (gk + i < kmax) ? p[i] : 0.0f;
                }
            } else {
#pragma unroll
                for (int i = 0; i < PER; ++i) v[i] = 0.0f;
            }
        } else {
            constexpr int TPK = R / PER;             // threads per k
            const int kk = t / TPK, r = (t % TPK) * PER;
            const int gk = k0 + kk, gr = r0 + r;
            if (gk < kmax) {
                const float* p = src + size_t(rows ? rows[gk] : gk) * ld + gr;
                if (gr + PER <= rmax) {
#pragma unroll
                    for (int i = 0; i < PER; i += 4) {
                        const float4 q = *reinterpret_cast<const float4*>(p + i);
                        v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < PER; ++i) v[i] = (gr + i < rmax) ? p[i] : 0.0f;
                }
            } else {
#pragma unroll
                for (int i = 0; i < PER; ++i) v[i] = 0.0f;
            }
        }
    }

    template <typename TOP>
    __device__ inline void store(TOP* __restrict__ s, int t) const {
        constexpr int LD = GBK + Op<TOP>::PAD;
        if constexpr (KCONTIG) {
            constexpr int TPR = GBK / PER;
            const int r = t / TPR, kk = (t % TPR) * PER;
            TOP* d = s + r * LD + kk;
#pragma unroll
            for (int i = 0; i < PER; ++i) d[i] = TOP(v[i]);
        } else {
            constexpr int TPK = R / PER;
            const int kk = t / TPK, r = (t % TPK) * PER;
#pragma unroll
            for (int i = 0; i < PER; ++i) s[(r + i) * LD + kk] = TOP(v[i]);
        }
    }
};

template <typename TOP, int TI, int TJ, bool TA, bool TB, Epi EPI>
__global__ void __launch_bounds__(GNT) gemm_kernel(GemmArgs g) {
    constexpr int BM = 32 * TI, BN = 32 * TJ, LD = GBK + Op<TOP>::PAD;
    __shared__ __attribute__((aligned(16))) TOP As[BM * LD];
    __shared__ __attribute__((aligned(16))) TOP Bs[BN * LD];

    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = w & 1, wn = w >> 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int nslab_total = (g.K + GBK - 1) / GBK;
    const int s_begin = blockIdx.z * g.kslabs_per_split;
    const int s_end = min(nslab_total, s_begin + g.kslabs_per_split);

    // A element (m, k): !TA -> A[row(m) lda + k] (k contiguous); TA -> A[row(k) lda + m]
    TileLoader<BM, !TA> la;
    // B element (k, n): !TB -> B[k ldb + n] (n contiguous); TB -> B[n ldb + k]
    TileLoader<BN, TB> lb;

    f32x4 acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    if (s_begin < s_end) {
        la.load(g.A, g.lda, g.arows, m0, g.M, s_begin * GBK, g.K, t);
        lb.load(g.B, g.ldb, nullptr, n0, g.N, s_begin * GBK, g.K, t);
    }
    const int fr = lane & 15, fq = lane >> 4;
    for (int s = s_begin; s < s_end; ++s) {
        __syncthreads();   // previous slab fully consumed
        la.store(As, t);
        lb.store(Bs, t);
        __syncthreads();
        if (s + 1 < s_end) {
            la.load(g.A, g.lda, g.arows, m0, g.M, (s + 1) * GBK, g.K, t);
            lb.load(g.B, g.ldb, nullptr, n0, g.N, (s + 1) * GBK, g.K, t);
        }
        if constexpr (sizeof(TOP) == 2) {
            bf16x8 a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * 16 * TI + i * 16 + fr) * LD + fq * 8]);
#pragma unroll
            for (int j = 0; j < TJ; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn * 16 * TJ + j * 16 + fr) * LD + fq * 8]);
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int q = 0; q < GBK / 4; ++q) {
                float a[TI], b[TJ];
#pragma unroll
                for (int i = 0; i < TI; ++i) a[i] = As[(wm * 16 * TI + i * 16 + fr) * LD + 4 * q + fq];
#pragma unroll
                for (int j = 0; j < TJ; ++j) b[j] = Bs[(wn * 16 * TJ + j * 16 + fr) * LD + 4 * q + fq];
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
    }

    // C[row][col]: row = tile row + 4 (lane / 16) + e, col = tile col + lane % 16
    float* C = g.C + blockIdx.z * g.split_stride;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int col = n0 + wn * 16 * TJ + j * 16 + fr;
            if (col >= g.N) continue;
            float bv = 0.0f;
            if constexpr (EPI == Epi::Bias || EPI == Epi::BiasGelu) bv = g.bias[col];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 16 * TI + i * 16 + 4 * fq + e;
                if (row >= g.M) continue;
                float v = acc[i][j][e];
                if constexpr (EPI == Epi::Bias) v += bv;
                if constexpr (EPI == Epi::BiasGelu) {
                    v += bv;
                    if (g.Z) g.Z[size_t(row) * g.ldz + col] = v;
                    v = gelu(v);
                }
                if constexpr (EPI == Epi::GeluGrad) v *= gelu_grad(g.Z[size_t(row) * g.ldz + col]);
                C[size_t(row) * g.ldc + col] = v;
            }
        }
}

// C = sum over `splits` partial tiles (ld = ldc, stride `stride` floats)
__global__ void split_sum_kernel(const float* __restrict__ P, int splits, size_t stride, int M, int N, int ldc,
                                 float* __restrict__ C) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= size_t(M) * N) return;
    const size_t row = i / N, col = i % N, off = row * ldc + col;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += P[z * stride + off];
    C[off] = s;
}

template <typename TOP, int TI, int TJ, Epi EPI>
hipError_t gemm_dispatch_t(bool ta, bool tb, const GemmArgs& g, dim3 grid, hipStream_t st) {
    if (!ta && !tb) hipLaunchKernelGGL((gemm_kernel<TOP, TI, TJ, false, false, EPI>), grid, dim3(GNT), 0, st, g);
    else if (!ta && tb) hipLaunchKernelGGL((gemm_kernel<TOP, TI, TJ, false, true, EPI>), grid, dim3(GNT), 0, st, g);
    else if (ta && !tb) hipLaunchKernelGGL((gemm_kernel<TOP, TI, TJ, true, false, EPI>), grid, dim3(GNT), 0, st, g);
    else hipLaunchKernelGGL((gemm_kernel<TOP, TI, TJ, true, true, EPI>), grid, dim3(GNT), 0, st, g);
    return hipGetLastError();
}

template <typename TOP, int TI, int TJ>
hipError_t gemm_dispatch_e(Epi epi, bool ta, bool tb, const GemmArgs& g, dim3 grid, hipStream_t st) {
    switch (epi) {
        case Epi::Store: return gemm_dispatch_t<TOP, TI, TJ, Epi::Store>(ta, tb, g, grid, st);
        case Epi::Bias: return gemm_dispatch_t<TOP, TI, TJ, Epi::Bias>(ta, tb, g, grid, st);
        case Epi::BiasGelu: return gemm_dispatch_t<TOP, TI, TJ, Epi::BiasGelu>(ta, tb, g, grid, st);
        case Epi::GeluGrad: return gemm_dispatch_t<TOP, TI, TJ, Epi::GeluGrad>(ta, tb, g, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gemm(bool bf16, Epi epi, bool ta, bool tb, int M, int N, int K, const float* A, int lda,
                       const int* arows, const float* B, int ldb, float* C, int ldc, const float* bias, float* Z,
                       int ldz, float* split_ws, size_t split_ws_floats, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs g{M, N, K, A, lda, arows, B, ldb, C, ldc, bias, Z, ldz, 0, 0};
    const int nslab = std::max(1, (K + GBK - 1) / GBK);
    // 128 x 128 tiles when they still give two workgroups per CU, else 64 x 64
    const bool big = size_t((M + 127) / 128) * ((N + 127) / 128) >= 512;
    const int bt = big ? 128 : 64;
    dim3 grid((N + bt - 1) / bt, (M + bt - 1) / bt, 1);
    g.kslabs_per_split = nslab;
    int splits = 1;
    const size_t tiles = size_t(grid.x) * grid.y;
    if (epi == Epi::Store && split_ws != nullptr && tiles < 256 && nslab >= 16) {
        splits = int(std::min<size_t>({size_t(16), (512 + tiles - 1) / tiles, size_t(nslab / 4)}));
        g.kslabs_per_split = (nslab + splits - 1) / splits;
        splits = (nslab + g.kslabs_per_split - 1) / g.kslabs_per_split;
        if (splits > 1 && size_t(splits) * M * ldc <= split_ws_floats) {
            g.C = split_ws;
            g.split_stride = size_t(M) * ldc;
            grid.z = splits;
        } else {
            splits = 1;
            g.kslabs_per_split = nslab;
        }
    }
    hipError_t e;
    if (big) e = bf16 ? gemm_dispatch_e<__bf16, 4, 4>(epi, ta, tb, g, grid, st)
                      : gemm_dispatch_e<float, 4, 4>(epi, ta, tb, g, grid, st);
    else e = bf16 ? gemm_dispatch_e<__bf16, 2, 2>(epi, ta, tb, g, grid, st)
                  : gemm_dispatch_e<float, 2, 2>(epi, ta, tb, g, grid, st);
    if (e != hipSuccess || splits == 1) return e;
    const size_t total = size_t(M) * N;
    hipLaunchKernelGGL(split_sum_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, split_ws, splits,
                       g.split_stride, M, N, ldc, C);
    return hipGetLastError();
}

// ---------------------------------------------------------------- loss, sums, Adam

namespace {

__global__ void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T, const int* __restrict__ trows,
                                int rows, int cols, float* __restrict__ dY, double* __restrict__ partial) {
    __shared__ double red[256];
    const size_t total = size_t(rows) * cols;
    const float scale = 2.0f / float(total);
    double acc = 0.0;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
        const size_t r = i / cols, c = i % cols;
        const float d = Y[i] - T[size_t(trows ? trows[r] : r) * cols + c];
        dY[i] = scale * d;
        acc += double(d) * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const double* __restrict__ partial, int nb, double denom, float* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = float(red[0] / denom);
}

__global__ void colsum_partial_kernel(const float* __restrict__ G, int ldg, int rows, int cols,
                                      float* __restrict__ partial) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const int per = (rows + gridDim.y - 1) / gridDim.y;
    const int r0 = blockIdx.y * per, r1 = min(rows, r0 + per);
    float s = 0.0f;
    for (int r = r0; r < r1; ++r) s += G[size_t(r) * ldg + c];
    partial[size_t(blockIdx.y) * cols + c] = s;
}

__global__ void colsum_final_kernel(const float* __restrict__ partial, int splits, int cols, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += partial[size_t(z) * cols + c];
    out[c] = s;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace

hipError_t launch_mse_grad(const float* Y, const float* T, const int* trows, int rows, int cols, float* dY,
                           double* partial, float* loss_out, hipStream_t st) {
    hipLaunchKernelGGL(mse_grad_kernel, dim3(kLossBlocks), dim3(256), 0, st, Y, T, trows, rows, cols, dY, partial);
    hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, partial, kLossBlocks,
                       double(rows) * double(cols), loss_out);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int ldg, int rows, int cols, float* partial, float* out, hipStream_t st) {
    if (cols <= 0) return hipSuccess;
    const dim3 grid((cols + 255) / 256, kColsumSplit);
    hipLaunchKernelGGL(colsum_partial_kernel, grid, dim3(256), 0, st, G, ldg, rows, cols, partial);
    hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, partial, kColsumSplit,
                       cols, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st) {
    const int blocks = int(std::min<size_t>((n + 255) / 256, 2048));
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

// ---------------------------------------------------------------- patch gather / scatter

PatchGroups colour_groups(int n, int colour, bool all_types) {
    PatchGroups pg{};
    struct Range {
        int first, cnt, type;
    };
    Range r1[3][3];
    int nr[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        const int par = (colour >> d) & 1;
        const int ci = interior_count_1d(n, par);
        if (!all_types) {
            if (ci > 0) r1[d][nr[d]++] = {par ? 3 : 2, ci, 0};
        } else if (n == 2) {
            if (par == 1) r1[d][nr[d]++] = {1, 1, 3};
        } else if (n >= 3) {
            if (par == 1) r1[d][nr[d]++] = {1, 1, 1};
            if (ci > 0) r1[d][nr[d]++] = {par ? 3 : 2, ci, 0};
            if (((n - 1) & 1) == par) r1[d][nr[d]++] = {n - 1, 1, 2};
        }
    }
    int row = 0;
    for (int c = 0; c < nr[2]; ++c)
        for (int b = 0; b < nr[1]; ++b)
            for (int a = 0; a < nr[0]; ++a) {
                const Range* rg[3] = {&r1[0][a], &r1[1][b], &r1[2][c]};
                const int g = pg.ng++;
                pg.start[g] = row;
                int count = 1;
                for (int d = 0; d < 3; ++d) {
                    pg.first[g][d] = rg[d]->first;
                    pg.cnt[g][d] = rg[d]->cnt;
                    count *= rg[d]->cnt;
                }
                pg.mat[g] = rg[0]->type == 3 ? 27 : rg[0]->type + 3 * rg[1]->type + 9 * rg[2]->type;
                row += all_types ? (count + kGroupAlign - 1) / kGroupAlign * kGroupAlign : count;
            }
    pg.start[pg.ng] = row;
    return pg;
}

namespace {

struct PatchGeo {
    int n, k, lc, m, nvel, size, N1;
    size_t nc;
};

__host__ PatchGeo make_geo(int n, int k) {
    PatchGeo g;
    g.n = n; g.k = k; g.lc = 2 * k + 1; g.m = 2 * k + 2;
    g.nvel = g.lc * g.m * g.m;
    g.size = 3 * g.nvel + g.m * g.m * g.m;
    g.N1 = n * (k + 1);
    g.nc = size_t(g.N1 - 1) * g.N1 * g.N1;
    return g;
}

// global index of patch-local entry q of the patch around vertex v; pres = pressure row
__device__ inline size_t patch_index(const PatchGeo& g, const int v[3], int q, bool& pres) {
    const int base0 = (v[0] - 1) * (g.k + 1), base1 = (v[1] - 1) * (g.k + 1), base2 = (v[2] - 1) * (g.k + 1);
    if (q < 3 * g.nvel) {
        const int c = q / g.nvel, w = q - c * g.nvel;
        const int l0 = c == 0 ? g.lc : g.m, l1 = c == 1 ? g.lc : g.m;
        const int i0 = w % l0, i1 = (w / l0) % l1, i2 = w / (l0 * l1);
        const int e0 = c == 0 ? g.N1 - 1 : g.N1, e1 = c == 1 ? g.N1 - 1 : g.N1;
        pres = false;
        return size_t(c) * g.nc + (i0 + base0) + size_t(e0) * ((i1 + base1) + size_t(e1) * (i2 + base2));
    }
    const int w = q - 3 * g.nvel;
    const int i0 = w % g.m, i1 = (w / g.m) % g.m, i2 = w / (g.m * g.m);
    pres = true;
    return 3 * g.nc + (i0 + base0) + size_t(g.N1) * ((i1 + base1) + size_t(g.N1) * (i2 + base2));
}

// vertex of row `row` of a grouped row space; false for a padding row (uniform over a workgroup)
__device__ inline bool group_vertex(const PatchGroups& pg, int row, int v[3]) {
    int gi = 0;
    while (gi + 1 < pg.ng && pg.start[gi + 1] <= row) ++gi;
    const int p = row - pg.start[gi];
    const int c0 = pg.cnt[gi][0], c1 = pg.cnt[gi][1];
    if (p >= c0 * c1 * pg.cnt[gi][2]) return false;
    v[0] = pg.first[gi][0] + 2 * (p % c0);
    v[1] = pg.first[gi][1] + 2 * ((p / c0) % c1);
    v[2] = pg.first[gi][2] + 2 * (p / (c0 * c1));
    return true;
}

__device__ inline double block_sum(double x, double* red) {
    red[threadIdx.x] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <typename T>
__global__ void __launch_bounds__(256) patch_gather_kernel(const T* __restrict__ r, PatchGeo g, PatchGroups pg,
                                                           int r0, float* __restrict__ X, int ldx,
                                                           float* __restrict__ s) {
    __shared__ double red[256];
    float* row = X + size_t(blockIdx.x) * ldx;
    int v[3];
    if (!group_vertex(pg, r0 + blockIdx.x, v)) {
        for (int q = threadIdx.x; q < g.size; q += 256) row[q] = 0.0f;
        if (threadIdx.x == 0) s[blockIdx.x] = 0.0f;
        return;
    }
    const double ih = g.n, ih2 = double(g.n) * g.n;
    double acc = 0.0;
    for (int q = threadIdx.x; q < g.size; q += 256) {
        bool pres;
        const size_t gi = patch_index(g, v, q, pres);
        const double val = double(r[gi]) * (pres ? ih2 : ih);
        acc += val * val;
    }
    const double nrm = sqrt(block_sum(acc, red));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    for (int q = threadIdx.x; q < g.size; q += 256) {
        bool pres;
        const size_t gi = patch_index(g, v, q, pres);
        row[q] = float(double(r[gi]) * (pres ? ih2 : ih) * inv);
    }
    if (threadIdx.x == 0) s[blockIdx.x] = float(nrm);
}

template <typename T>
__global__ void __launch_bounds__(256) patch_scatter_kernel(T* __restrict__ x, PatchGeo g, PatchGroups pg, int r0,
                                                            const float* __restrict__ Y, int ldy,
                                                            const float* __restrict__ s, double omega) {
    __shared__ double red[256];
    int v[3];
    if (!group_vertex(pg, r0 + blockIdx.x, v)) return;
    const double sc = omega * double(s[blockIdx.x]);
    if (sc == 0.0) return;   // uniform over the workgroup: no barrier reached yet
    const float* row = Y + size_t(blockIdx.x) * ldy;
    // the exact correction K_j^+ R_j r has zero coefficient mean in the patch
    // pressure (it is orthogonal to the kernel of K_j): project the computed one
    double ps = 0.0;
    for (int q = 3 * g.nvel + threadIdx.x; q < g.size; q += 256) ps += row[q];
    const double pmean = block_sum(ps, red) / double(g.size - 3 * g.nvel);
    for (int q = threadIdx.x; q < g.size; q += 256) {
        bool pres;
        const size_t gi = patch_index(g, v, q, pres);
        const double val = pres ? sc * (row[q] - pmean) * double(g.n) : sc * row[q];
        x[gi] = T(double(x[gi]) + val);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) patch_gather_diff_kernel(const T* __restrict__ xn, const T* __restrict__ xo,
                                                                PatchGeo g, PatchGroups pg, int r0,
                                                                float* __restrict__ Tt, int ldt,
                                                                const float* __restrict__ s) {
    float* row = Tt + size_t(blockIdx.x) * ldt;
    int v[3];
    if (!group_vertex(pg, r0 + blockIdx.x, v)) {
        for (int q = threadIdx.x; q < g.size; q += 256) row[q] = 0.0f;
        return;
    }
    const float sc = s[blockIdx.x];
    const double inv = sc > 0.0f ? 1.0 / double(sc) : 0.0;
    const double h = 1.0 / g.n;
    for (int q = threadIdx.x; q < g.size; q += 256) {
        bool pres;
        const size_t gi = patch_index(g, v, q, pres);
        row[q] = float((double(xn[gi]) - (xo ? double(xo[gi]) : 0.0)) * (pres ? h : 1.0) * inv);
    }
}

}  // namespace

namespace {

hipError_t launch_group_gather(bool f64, const void* r, int n, int k, const PatchGroups& pg, int r0, int rows,
                               float* X, int ldx, float* s, hipStream_t st) {
    if (rows <= 0 || pg.ng <= 0) return hipSuccess;
    const PatchGeo g = make_geo(n, k);
    if (f64) hipLaunchKernelGGL(patch_gather_kernel<double>, dim3(rows), dim3(256), 0, st,
                                static_cast<const double*>(r), g, pg, r0, X, ldx, s);
    else hipLaunchKernelGGL(patch_gather_kernel<float>, dim3(rows), dim3(256), 0, st, static_cast<const float*>(r), g,
                            pg, r0, X, ldx, s);
    return hipGetLastError();
}

hipError_t launch_group_scatter(bool f64, void* x, int n, int k, const PatchGroups& pg, int r0, int rows,
                                const float* Y, int ldy, const float* s, double omega, hipStream_t st) {
    if (rows <= 0 || pg.ng <= 0) return hipSuccess;
    const PatchGeo g = make_geo(n, k);
    if (f64) hipLaunchKernelGGL(patch_scatter_kernel<double>, dim3(rows), dim3(256), 0, st, static_cast<double*>(x), g,
                                pg, r0, Y, ldy, s, omega);
    else hipLaunchKernelGGL(patch_scatter_kernel<float>, dim3(rows), dim3(256), 0, st, static_cast<float*>(x), g, pg,
                            r0, Y, ldy, s, omega);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_patch_gather(bool f64, const void* r, int n, int k, int colour, int p0, int np, float* X, int ldx,
                               float* s, hipStream_t st) {
    return launch_group_gather(f64, r, n, k, colour_groups(n, colour, false), p0, np, X, ldx, s, st);
}

hipError_t launch_patch_scatter(bool f64, void* x, int n, int k, int colour, int p0, int np, const float* Y, int ldy,
                                const float* s, double omega, hipStream_t st) {
    return launch_group_scatter(f64, x, n, k, colour_groups(n, colour, false), p0, np, Y, ldy, s, omega, st);
}

hipError_t launch_patch_gather_diff(bool f64, const void* xnew, const void* xold, int n, int k, int colour, int p0,
                                    int np, float* T, int ldt, const float* s, hipStream_t st) {
    if (np <= 0) return hipSuccess;
    const PatchGeo g = make_geo(n, k);
    const PatchGroups pg = colour_groups(n, colour, false);
    if (pg.ng <= 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(patch_gather_diff_kernel<double>, dim3(np), dim3(256), 0, st,
                                static_cast<const double*>(xnew), static_cast<const double*>(xold), g, pg, p0, T, ldt,
                                s);
    else hipLaunchKernelGGL(patch_gather_diff_kernel<float>, dim3(np), dim3(256), 0, st,
                            static_cast<const float*>(xnew), static_cast<const float*>(xold), g, pg, p0, T, ldt, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Direct solver: gather, GEMM, scatter fused

void direct_dims(int d, int* dk, int* dn) {
    const int cols = d <= 256 ? 256 : 768;   // columns of one workgroup: 4 waves x 4 or 8 waves x 6 blocks of 16
    *dk = (d + 63) / 64 * 64;
    *dn = (d + cols - 1) / cols * cols;
}

namespace {

struct DirectArgs {
    const void* r;     // residual (level vector)
    void* x;           // iterate (level vector), x += the patch corrections
    const void* Bt;    // per type: M padded to dn x dk, row-major [out][in] (k contiguous), BF16 or FP32
    size_t bstride;    // elements between two types' matrices (dn dk)
    int rows, d, dk;   // grouped row space of the colour, patch dimension, padded k extent
    PatchGeo geo;
    PatchGroups pg;
};

constexpr int kMaxPatchDk = 1856;   // k = 3: d = 3 * 7 * 64 + 512, a multiple of 64
constexpr int DBM = 64, DKC = 64, DPAD = 8, CLD = 17;

template <typename TOP> struct Frag;
template <> struct Frag<__bf16> {
    typedef __bf16 v __attribute__((ext_vector_type(8)));
};
template <> struct Frag<float> {
    typedef float v __attribute__((ext_vector_type(8)));
};

// Tables of patch-local entry q.  off: offset from its component's corner of
// the patch (the level-vector index is corner[comp] + off).  meta: the
// contiguous run of q it lies on (the entries of one component that differ
// only in the first index: consecutive in q and in memory) -- run start
// (bits 0..11), run length (12..15), component (16..17); entries q >= d are
// runs of their own.
__device__ inline void entry_tables(const PatchGeo& g, int d, int q, int& off, int& meta) {
    if (q >= d) {
        off = 0;
        meta = q | (1 << 12);
        return;
    }
    int c, w, l0, l1, e0, e1;
    if (q < 3 * g.nvel) {
        c = q / g.nvel;
        w = q - c * g.nvel;
        l0 = c == 0 ? g.lc : g.m;
        l1 = c == 1 ? g.lc : g.m;
        e0 = c == 0 ? g.N1 - 1 : g.N1;
        e1 = c == 1 ? g.N1 - 1 : g.N1;
    } else {
        c = 3;
        w = q - 3 * g.nvel;
        l0 = l1 = g.m;
        e0 = e1 = g.N1;
    }
    const int i0 = w % l0, i1 = (w / l0) % l1, i2 = w / (l0 * l1);
    off = i0 + e0 * (i1 + e1 * i2);
    meta = (q - i0) | (l0 << 12) | (c << 16);
}

// Element e (e < 64 W) of the 64 rows x [qw, qw + W) window, taken run
// segment by run segment (a run clipped to the window), and in a segment row
// by row with q fastest: consecutive e are consecutive entries of one patch
// and then the same entries of the next patch, which for neighbouring
// patches of a colour lie next to each other in memory.
__device__ inline void window_entry(const int* __restrict__ meta, int e, int qw, int W, int& row, int& q, int& c) {
    const int mt = meta[qw + (e >> 6)];
    const int ls = mt & 0xfff, l0 = (mt >> 12) & 15;
    const int ss = max(ls, qw), len = min(ls + l0, qw + W) - ss;
    const int rel = e - ((ss - qw) << 6);
    // rel < 64 len <= 512: (rel + 1/2) / len is at least 1/16 from an integer, far above the rounding
    row = int((float(rel) + 0.5f) * (1.0f / float(len)));
    q = ss + rel - row * len;
    c = mt >> 16;
}

// One workgroup (NW waves) owns 64 patch rows of a colour's grouped row
// space and NW x CB x 16 output columns (every column at k = 1, 2); each wave
// all 64 rows and CB column blocks.  Row i of the product is the normalized
// residual of patch i, (r_vel / h, r_pres / h^2), gathered from the level
// vector; the product with the patch type's map M (the row tile's group) is
// added into x as (U, h P) -> velocity U, pressure (h P) / h.
//   k loop: chunks of 64; a chunk of the gathered rows sits in LDS (double
//   buffered: the next chunk's loads are in flight during this chunk's
//   products), gathered along contiguous runs (window_entry); the M
//   fragments come straight from global memory (L2), one k-step ahead.  A
//   lane's fragments cover 8 consecutive k of a 32-wide k-step: one 16x16x32
//   BF16 MFMA, or eight 16x16x4 FP32 MFMAs taking the 8 k one at a time (the
//   same k order on both operands).
//   Epilogue: column block by column block through LDS, then along
//   contiguous runs into x (read all, then write all).  Within a colour the
//   patches are disjoint, so every x entry has exactly one writer.
// Column tiles of a row tile run on one XCD.
template <typename TOP, typename T, int NW, int CB>
__global__ void __launch_bounds__(64 * NW) direct_patch_kernel(DirectArgs a) {
    constexpr int NT = 64 * NW, BN = NW * CB * 16, LDA = DKC + DPAD, EPT = DBM * DKC / NT;
    typedef typename Frag<TOP>::v fragv;
    __shared__ __attribute__((aligned(32))) TOP As[2][DBM * LDA];
    __shared__ int off[kMaxPatchDk];
    __shared__ int meta[kMaxPatchDk];
    __shared__ long long rbase[DBM][4];
    __shared__ float Cs[NW][DBM * CLD];

    const PatchGeo& g = a.geo;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int fr = lane & 15, fq = lane >> 4;
    const int ntn = (a.d + BN - 1) / BN;
    const int tile = xcd_contiguous(blockIdx.x, gridDim.x);
    const int m0 = (tile / ntn) * DBM, n0 = (tile % ntn) * BN;

    for (int q = t; q < a.dk; q += NT) entry_tables(g, a.d, q, off[q], meta[q]);
    if (t < DBM) {
        int v[3];
        if (m0 + t < a.rows && group_vertex(a.pg, m0 + t, v)) {
            const long long b0 = (v[0] - 1) * (g.k + 1), b1 = (v[1] - 1) * (g.k + 1), b2 = (v[2] - 1) * (g.k + 1);
            const long long N1 = g.N1;
            rbase[t][0] = b0 + (N1 - 1) * (b1 + N1 * b2);
            rbase[t][1] = (long long)g.nc + b0 + N1 * (b1 + (N1 - 1) * b2);
            rbase[t][2] = 2 * (long long)g.nc + b0 + N1 * (b1 + N1 * b2);
            rbase[t][3] = 3 * (long long)g.nc + b0 + N1 * (b1 + N1 * b2);
        } else {
            rbase[t][0] = rbase[t][1] = rbase[t][2] = rbase[t][3] = -1;
        }
    }
    const TOP* Bt = static_cast<const TOP*>(a.Bt);
    {
        int gi = 0;   // the row tile lies in one group: groups start at multiples of 128
        while (gi + 1 < a.pg.ng && a.pg.start[gi + 1] <= m0) ++gi;
        Bt += size_t(a.pg.mat[gi]) * a.bstride;
    }
    __syncthreads();

    const T* __restrict__ r = static_cast<const T*>(a.r);
    const float sv = float(g.n), sp = float(g.n) * float(g.n);   // 1/h and 1/h^2, powers of two
    float gv[EPT];
    int gpos[EPT];   // row * LDA + q - k0 of each staged value
    auto gather_load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            int row, q, c;
            window_entry(meta, t + NT * i, k0, DKC, row, q, c);
            gpos[i] = row * LDA + q - k0;
            const long long b = rbase[row][c];
            gv[i] = (q < a.d && b >= 0) ? float(r[b + off[q]]) * (c == 3 ? sp : sv) : 0.0f;
        }
    };
    auto gather_store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) As[buf][gpos[i]] = TOP(gv[i]);
    };

    // M fragments: lane (fr, fq) of column block j reads M[col][k .. k + 7], col = n0 + (w CB + j) 16 + fr
    const TOP* bp[CB];
#pragma unroll
    for (int j = 0; j < CB; ++j) bp[j] = Bt + size_t(n0 + (w * CB + j) * 16 + fr) * a.dk + fq * 8;
    fragv bcur[CB], bnext[CB];
    auto b_load = [&](fragv* dst, int k) {
#pragma unroll
        for (int j = 0; j < CB; ++j) dst[j] = *reinterpret_cast<const fragv*>(bp[j] + k);
    };

    f32x4 acc[4][CB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    const int nchunk = a.dk / DKC, nstep = a.dk / 32;
    gather_load(0);
    gather_store(0);
    __syncthreads();
    if (nchunk > 1) gather_load(DKC);
    b_load(bcur, 0);
    for (int s = 0; s < nstep; ++s) {
        const int chunk = s >> 1, ks = s & 1;
        if (s + 1 < nstep) b_load(bnext, (s + 1) * 32);
        const TOP* Ab = As[chunk & 1] + ks * 32 + fq * 8;
        fragv af[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const fragv*>(Ab + (i * 16 + fr) * LDA);
        if constexpr (sizeof(TOP) == 2) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < CB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bcur[j], acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < CB; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][e], bcur[j][e], acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) bcur[j] = bnext[j];
        if (ks == 1 && chunk + 1 < nchunk) {
            // the buffer of chunk + 1 was last read in chunk - 1, before the previous barrier
            gather_store((chunk + 1) & 1);
            __syncthreads();
            if (chunk + 2 < nchunk) gather_load((chunk + 2) * DKC);
        }
    }

    // epilogue: block (rows 16 i + 4 (lane / 16) + e, columns lane % 16) -> Cs[w], then along runs into x
    T* __restrict__ x = static_cast<T*>(a.x);
    float* cw = Cs[w];
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        const int qw = n0 + (w * CB + j) * 16, W = min(16, a.d - qw);
        __syncthreads();   // previous block's Cs fully read
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) cw[(i * 16 + 4 * fq + e) * CLD + fr] = acc[i][j][e];
        __syncthreads();
        if (W <= 0) continue;
        long long idx[16];
        T xv[16];
        float yv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = lane + 64 * i;
            idx[i] = -1;
            if (e < 64 * W) {
                int row, q, c;
                window_entry(meta, e, qw, W, row, q, c);
                const long long b = rbase[row][c];
                if (b >= 0) {
                    idx[i] = b + off[q];
                    yv[i] = cw[row * CLD + q - qw] * (c == 3 ? sv : 1.0f);
                }
            }
            xv[i] = idx[i] >= 0 ? x[idx[i]] : T(0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (idx[i] >= 0) x[idx[i]] = T(xv[i] + T(yv[i]));
    }
}

template <typename TOP, typename T, int NW, int CB>
hipError_t direct_dispatch(const DirectArgs& a, hipStream_t st) {
    constexpr int BN = NW * CB * 16;
    const int tiles = (a.rows / DBM) * ((a.d + BN - 1) / BN);
    hipLaunchKernelGGL((direct_patch_kernel<TOP, T, NW, CB>), dim3(tiles), dim3(64 * NW), 0, st, a);
    return hipGetLastError();
}

// 8 waves x 6 column blocks = 768 columns (every column at k = 2); FP32 operands
// take twice the fragment registers: 8 x 3 (384 columns, a divisor of 768)
template <typename TOP, typename T>
hipError_t direct_dispatch_cb(const DirectArgs& a, hipStream_t st) {
    if (a.d <= 256) return direct_dispatch<TOP, T, 4, 4>(a, st);
    if constexpr (sizeof(TOP) == 2) return direct_dispatch<TOP, T, 8, 6>(a, st);
    else return direct_dispatch<TOP, T, 8, 3>(a, st);
}

}  // namespace

hipError_t launch_direct_patch(bool f64, bool bf16, const void* r, void* x, int n, int k, const PatchGroups& pg,
                               const void* Bt, hipStream_t st) {
    const int rows = pg.ng > 0 ? pg.start[pg.ng] : 0;
    if (rows <= 0) return hipSuccess;
    DirectArgs a;
    a.r = r;
    a.x = x;
    a.Bt = Bt;
    a.geo = make_geo(n, k);
    a.d = a.geo.size;
    int dn = 0;
    direct_dims(a.d, &a.dk, &dn);
    a.bstride = size_t(dn) * a.dk;
    a.rows = rows;
    a.pg = pg;
    static_assert(kGroupAlign % DBM == 0, "a row tile must not straddle two groups");
    if (a.dk > kMaxPatchDk || rows % DBM != 0) return hipErrorInvalidValue;
    if (bf16) return f64 ? direct_dispatch_cb<__bf16, double>(a, st) : direct_dispatch_cb<__bf16, float>(a, st);
    return f64 ? direct_dispatch_cb<float, double>(a, st) : direct_dispatch_cb<float, float>(a, st);
}

// ---------------------------------------------------------------- training helpers

namespace {

__device__ inline uint64_t mix64(uint64_t z) {
    // SplitMix64 output function (Steele, Lea & Flood 2014)
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// keyed balanced Feistel bijection of [0, 2^(2 half)), four rounds
__device__ inline uint64_t feistel(uint64_t x, int half, uint64_t key) {
    const uint64_t mask = (uint64_t(1) << half) - 1;
    uint64_t L = x >> half, R = x & mask;
    for (int r = 0; r < 4; ++r) {
        const uint64_t F = mix64(R ^ (key + 0x9e3779b97f4a7c15ULL * uint64_t(r + 1))) & mask;
        const uint64_t nL = R;
        R = L ^ F;
        L = nL;
    }
    return (L << half) | R;
}

__global__ void batch_rows_kernel(int* __restrict__ rows, int64_t start, int count, int64_t n, int half,
                                  uint64_t key) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    // cycle walking: the orbit of start + i < n returns below n
    uint64_t y = uint64_t(start + i);
    do {
        y = feistel(y, half, key);
    } while (y >= uint64_t(n));
    rows[i] = int(y);
}

template <typename T>
__global__ void add_kernel(T* __restrict__ x, const T* __restrict__ c, size_t n) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        x[i] += c[i];
}

__global__ void accumulate_kernel(const float* __restrict__ v, double* __restrict__ acc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *acc += double(*v);
}

}  // namespace

hipError_t launch_batch_rows(int* rows, int64_t start, int count, int64_t n, uint64_t key, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int bits = 2;
    while ((int64_t(1) << bits) < n) ++bits;
    bits += bits & 1;
    hipLaunchKernelGGL(batch_rows_kernel, dim3((count + 255) / 256), dim3(256), 0, st, rows, start, count, n,
                       bits / 2, key);
    return hipGetLastError();
}

hipError_t launch_add(bool f64, void* x, const void* c, size_t n, hipStream_t st) {
    const int blocks = int(std::min<size_t>((n + 255) / 256, 4096));
    if (blocks == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(add_kernel<double>, dim3(blocks), dim3(256), 0, st, static_cast<double*>(x),
                                static_cast<const double*>(c), n);
    else hipLaunchKernelGGL(add_kernel<float>, dim3(blocks), dim3(256), 0, st, static_cast<float*>(x),
                            static_cast<const float*>(c), n);
    return hipGetLastError();
}

hipError_t launch_accumulate(const float* v, double* acc, hipStream_t st) {
    hipLaunchKernelGGL(accumulate_kernel, dim3(1), dim3(64), 0, st, v, acc);
    return hipGetLastError();
}

}  // namespace smg
