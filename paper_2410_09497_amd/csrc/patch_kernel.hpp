// Local solves of the colourized vertex-patch smoother (Alg. 2, Sec. 3.2),
// one workgroup per patch of one colour, gfx950.
//
// For patch j with residual restriction (F, G) = R_j r the correction is the
// pseudo-inverse solution of the patch problem [[A, B^T], [B, 0]] (U, P) =
// (F, G) (Sec. 3.3 "Direct solver" reference) computed as in Sec. 3.2:
//   G <- G - mean(G)           (the part of G in the range of B)
//   S P = B A^{-1} F - G,  S = B A^{-1} B^T, by CG on mean-zero vectors
//   U = A^{-1} (F - B^T P)
// with A^{-1} applied by fast diagonalization per velocity component
// (three 1D eigenbasis contractions, a diagonal scaling, three back
// contractions) and B, B^T by the restricted 1D divergence block times the
// diagonal DG masses.  Everything lives in LDS; the update x += R_j^T (U, P)
// needs no atomics because the patches of one colour have disjoint DoF sets.
#pragma once

#include <hip/hip_runtime.h>

#include "patch_tables.hpp"
#include "xcd.hpp"

namespace smg {

// threads per patch: NT_OVERRIDE if positive, else by degree (measured on
// MI355X: one wave for k = 1, two for k = 2, four for k = 3 and 4, eight for
// k = 5, whose patch vectors take most of a CU's LDS so one workgroup runs
// per CU).  LDS per workgroup: 2 velocity-sized and 4 pressure-sized arrays
// and the entry table, 86 KB at k = 4 and 150 KB at k = 5 in FP64.
template <int K, int NT_OVERRIDE = 0>
struct PatchShape {
    static constexpr int M = K + 1;
    static constexpr int NC = 2 * K + 1, ND = 2 * K + 2;
    static constexpr int NV = NC * ND * ND;      // one velocity component
    static constexpr int NP = ND * ND * ND;      // pressure
    static constexpr int NT = NT_OVERRIDE > 0 ? NT_OVERRIDE : (K == 1 ? 64 : (K == 2 ? 128 : (K <= 4 ? 256 : 512)));
    static constexpr int NW = NT / 64;           // waves
};

// (i0, i1, i2) of entry e of velocity component c: the extents depend on c
// (2k+1 in its own direction, 2k+2 in the others), so branch on c and keep
// every divisor a compile-time constant
template <int K>
__device__ inline void vel_coords(int c, int e, int& i0, int& i1, int& i2) {
    constexpr int NC = 2 * K + 1, ND = 2 * K + 2;
    if (c == 0) {
        i0 = e % NC;
        const int t = e / NC;
        i1 = t % ND;
        i2 = t / ND;
    } else if (c == 1) {
        i0 = e % ND;
        const int t = e / ND;
        i1 = t % NC;
        i2 = t / NC;
    } else {
        i0 = e % ND;
        const int t = e / ND;
        i1 = t % ND;
        i2 = t / ND;
    }
}

// extents (x fastest) of component c: the continuous direction is c
template <int K>
__device__ constexpr int ext(int c, int d) {
    return d == c ? 2 * K + 1 : 2 * K + 2;
}

// Packed coordinates of velocity entry idx (component c, position (i0, i1, i2)
// in its box): c | i0 << 2 | i1 << 8 | i2 << 14.  A table of them sits in LDS,
// filled once per workgroup, so the passes read one word instead of redoing
// the division chain of every entry.
__device__ inline int code_c(int v) { return v & 3; }
__device__ inline int code_i(int v, int d) { return (v >> (2 + 6 * d)) & 63; }
template <int K>
__device__ inline int vel_code(int idx) {
    constexpr int NV = (2 * K + 1) * (2 * K + 2) * (2 * K + 2);
    const int c = idx / NV;
    int i0, i1, i2;
    vel_coords<K>(c, idx - c * NV, i0, i1, i2);
    return c | (i0 << 2) | (i1 << 8) | (i2 << 14);
}

// block-wide sums of one or two values per thread (NW waves; red holds 2 NW)
template <int NW, typename T>
__device__ inline T block_sum(T v, T* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if constexpr (NW == 1) return v;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    T s = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[i];
    return s;
}
template <int NW, typename T>
__device__ inline void block_sum2(T& a, T& b, T* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if constexpr (NW == 1) return;
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = a;
        red[NW + w] = b;
    }
    __syncthreads();
    a = 0;
    b = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        a += red[i];
        b += red[NW + i];
    }
}

// out[comp] = contraction of in[comp] along direction d with matrix
// S_(comp, d) (transposed if TR), for the three velocity components at once.
// one entry of contract3 for component C along direction D: every stride is a
// compile-time constant, so the LDS reads use immediate offsets
template <int K, typename T, bool TR, int C, int D>
__device__ __forceinline__ T contract_entry(const T* in, int idx, int ii, const T* S) {
    constexpr int NC = 2 * K + 1, ND = 2 * K + 2;
    constexpr int e0 = C == 0 ? NC : ND, e1 = C == 1 ? NC : ND;
    constexpr int st = D == 0 ? 1 : (D == 1 ? e0 : e0 * e1);
    constexpr int n = C == D ? NC : ND;
    const T* base = in + idx - ii * st;
    const T* row = TR ? S + ii : S + ii * n;
    T acc = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) acc += row[TR ? j * n : j] * base[j * st];
    return acc;
}

template <int K, int NTP, typename T, bool TR, int D>
__device__ __forceinline__ void contract3(const T* in, T* out, const T* const* Sdir, const int* codes) {
    using P = PatchShape<K, NTP>;
    constexpr int NV = P::NV;
    for (int idx = threadIdx.x; idx < 3 * NV; idx += P::NT) {
        const int code = codes[idx];
        const int c = code_c(code);
        const int ii = code_i(code, D);
        T acc;
        if (c == 0) acc = contract_entry<K, T, TR, 0, D>(in, idx, ii, Sdir[0 * 3 + D]);
        else if (c == 1) acc = contract_entry<K, T, TR, 1, D>(in, idx, ii, Sdir[1 * 3 + D]);
        else acc = contract_entry<K, T, TR, 2, D>(in, idx, ii, Sdir[2 * 3 + D]);
        out[idx] = acc;
    }
}

// v <- A^{-1} v for the three components (in place), work buffer w
// entries of the velocity vectors per thread: entry idx belongs to thread
// idx mod NT, as its e-th entry with e = idx div NT
template <int K, int NTP>
constexpr int entries_per_thread() {
    return (3 * PatchShape<K, NTP>::NV + PatchShape<K, NTP>::NT - 1) / PatchShape<K, NTP>::NT;
}

// rinv[e] = 1 / (lambda_0 + lambda_1 + lambda_2) of this thread's e-th entry:
// the eigenvalue sums of the fast diagonalization depend only on the patch
// type, so each thread forms its reciprocals once per patch and the scaling
// step multiplies instead of dividing
template <int K, int NTP, typename T>
__device__ inline void fd_reciprocals(T* rinv, const T* const* Ldir, const int* codes) {
    using P = PatchShape<K, NTP>;
#pragma unroll
    for (int e = 0; e < entries_per_thread<K, NTP>(); ++e) {
        const int idx = threadIdx.x + e * P::NT;
        rinv[e] = T(0);
        if (idx < 3 * P::NV) {
            const int code = codes[idx], c = code_c(code);
            rinv[e] = T(1) / (Ldir[c * 3 + 0][code_i(code, 0)] + Ldir[c * 3 + 1][code_i(code, 1)] +
                              Ldir[c * 3 + 2][code_i(code, 2)]);
        }
    }
}

template <int K, int NTP, typename T>
__device__ __forceinline__ void fd_scale(T* v, const T* rinv) {
    using P = PatchShape<K, NTP>;
#pragma unroll
    for (int e = 0; e < entries_per_thread<K, NTP>(); ++e) {
        const int idx = threadIdx.x + e * P::NT;
        if (idx < 3 * P::NV) v[idx] *= rinv[e];
    }
}

template <int K, int NTP, typename T>
__device__ __forceinline__ void fd_inverse(T* v, T* w, const T* const* Sdir, const T* rinv, const int* codes) {
    // a thread per entry: lanes read with unit stride (a thread per 1D line reads
    // fewer words but with strided, bank-conflicting lanes, and measured slower)
    contract3<K, NTP, T, true, 0>(v, w, Sdir, codes);
    __syncthreads();
    contract3<K, NTP, T, true, 1>(w, v, Sdir, codes);
    __syncthreads();
    contract3<K, NTP, T, true, 2>(v, w, Sdir, codes);
    __syncthreads();
    fd_scale<K, NTP, T>(w, rinv);
    __syncthreads();
    contract3<K, NTP, T, false, 2>(w, v, Sdir, codes);
    __syncthreads();
    contract3<K, NTP, T, false, 1>(v, w, Sdir, codes);
    __syncthreads();
    contract3<K, NTP, T, false, 0>(w, v, Sdir, codes);
    __syncthreads();
}

// ---- in-plane eigenbasis products on the matrix cores (FP32 cycle, BF16 operands)
//
// For velocity component c with extents (e0, e1, e2), the first two factors of
// the fast diagonalization form one matrix Q_c = S_0 (x) S_1 of order e0 e1,
// Q_c[j][m] = S_0[i0][i0'] S_1[i1][i1'] for j = i0 + e0 i1, m = i0' + e0 i1'.
// The in-plane products of every z-slice of the component are then one GEMM:
// forward  W[z][m] = sum_j V[z][j] Q_c[j][m],  back  V[z][j] = sum_m W[z][m] Q_c[j][m],
// on v_mfma_f32_16x16x16_bf16 (operands rounded to BF16, FP32 accumulation),
// the z-slices (e2 <= 8) as the rows of one 16-row block.  Q_c sits in LDS in
// BF16, padded with zeros to KP x KP.  The z factor and the eigenvalue scaling
// stay on the vector units.
template <int K>
struct MfShape {
    static constexpr int ND = 2 * K + 2;
    static constexpr int KP = (ND * ND + 15) / 16 * 16;   // padded order of Q_c
};

typedef short bf16x4_bits __attribute__((ext_vector_type(4)));
typedef float f32x4_mf __attribute__((ext_vector_type(4)));

__device__ inline short bf16_bits(float f) { return __builtin_bit_cast(short, __bf16(f)); }

// Q_c for the three components into Qm (3 KP x KP, BF16 bits, row j = input index)
template <int K, int NTP>
__device__ inline void build_inplane(short* Qm, const float* const* Sdir) {
    using P = PatchShape<K, NTP>;
    constexpr int KP = MfShape<K>::KP;
    for (int i = threadIdx.x; i < 3 * KP * KP; i += P::NT) {
        const int c = i / (KP * KP), jm = i - c * KP * KP, j = jm / KP, m = jm - j * KP;
        const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1);
        float v = 0.0f;
        if (j < e0 * e1 && m < e0 * e1) {
            const int i0 = j % e0, i1 = j / e0, o0 = m % e0, o1 = m / e0;
            v = Sdir[c * 3 + 0][i0 * e0 + o0] * Sdir[c * 3 + 1][i1 * e1 + o1];
        }
        Qm[i] = bf16_bits(v);
    }
}

// out_c = in_c Q_c (FWD) or in_c Q_c^T (back) for the three components, z-slices as rows
template <int K, int NTP, bool FWD>
__device__ __forceinline__ void inplane_mfma(const float* in, float* out, const short* Qm) {
    using P = PatchShape<K, NTP>;
    constexpr int NV = P::NV, KP = MfShape<K>::KP, NB = KP / 16;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int fr = lane & 15, fq = lane >> 4;
    for (int tile = w; tile < 3 * NB; tile += P::NW) {
        const int c = tile / NB, nb = tile - c * NB;
        const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1), e2 = ext<K>(c, 2), pl = e0 * e1;
        const float* src = in + c * NV;
        const short* Q = Qm + c * KP * KP;
        f32x4_mf acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < NB; ++ks) {
            const int k0 = ks * 16 + 4 * fq;
            bf16x4_bits a, b;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int kk = k0 + t;
                a[t] = bf16_bits((fr < e2 && kk < pl) ? src[fr * pl + kk] : 0.0f);
                // B[k][col]: forward Q[k][col], back Q[col][k]
                b[t] = FWD ? Q[kk * KP + nb * 16 + fr] : Q[(nb * 16 + fr) * KP + kk];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        const int col = nb * 16 + fr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int z = 4 * fq + e;
            if (z < e2 && col < pl) out[c * NV + z * pl + col] = acc[e];
        }
    }
}

// v <- A^{-1} v (FP32) with the in-plane factors on the matrix cores, work buffer w
template <int K, int NTP>
__device__ __forceinline__ void fd_inverse_mf(float* v, float* w, const float* const* Sdir, const float* rinv,
                                     const int* codes, const short* Qm) {
    inplane_mfma<K, NTP, true>(v, w, Qm);
    __syncthreads();
    contract3<K, NTP, float, true, 2>(w, v, Sdir, codes);
    __syncthreads();
    fd_scale<K, NTP, float>(v, rinv);
    __syncthreads();
    contract3<K, NTP, float, false, 2>(v, w, Sdir, codes);
    __syncthreads();
    inplane_mfma<K, NTP, false>(w, v, Qm);
    __syncthreads();
}

// vel = B^T p:  (B^T p)_c[i] = -D^T along c times the DG masses of the other directions
template <int K, int NTP, typename T>
__device__ inline void apply_BT(const T* p, T* vel, const T* Dp, const T* md, const int* codes) {
    using P = PatchShape<K, NTP>;
    constexpr int NV = P::NV, NC = P::NC, ND = P::ND;
    for (int idx = threadIdx.x; idx < 3 * NV; idx += P::NT) {
        const int code = codes[idx], c = code_c(code);
        const int i0 = code_i(code, 0), i1 = code_i(code, 1), i2 = code_i(code, 2);
        // pressure index equals i in the DG directions; the continuous one is summed
        int pbase, pst, ic;
        T mass;
        if (c == 0) {
            pbase = ND * (i1 + ND * i2), pst = 1, ic = i0, mass = md[i1] * md[i2];
        } else if (c == 1) {
            pbase = i0 + ND * ND * i2, pst = ND, ic = i1, mass = md[i0] * md[i2];
        } else {
            pbase = i0 + ND * i1, pst = ND * ND, ic = i2, mass = md[i0] * md[i1];
        }
        T acc = 0;
        for (int q = 0; q < ND; ++q) acc += Dp[q * NC + ic] * p[pbase + q * pst];
        vel[idx] = -mass * acc;
    }
}

// p = B vel (all three components summed), returns nothing; caller projects
template <int K, int NTP, typename T>
__device__ inline void apply_B(const T* vel, T* p, const T* Dp, const T* md) {
    using P = PatchShape<K, NTP>;
    constexpr int NV = P::NV, NC = P::NC, ND = P::ND;
    for (int idx = threadIdx.x; idx < P::NP; idx += P::NT) {
        const int q[3] = {idx % ND, (idx / ND) % ND, idx / (ND * ND)};
        T acc = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1);
            int vs[3] = {1, e0, e0 * e1};
            int vbase = 0;
            T mass = 1;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (d != c) {
                    vbase += q[d] * vs[d];
                    mass *= md[q[d]];
                }
            T s = 0;
            for (int j = 0; j < NC; ++j) s += Dp[q[c] * NC + j] * vel[c * NV + vbase + j * vs[c]];
            acc += mass * s;
        }
        p[idx] = -acc;
    }
}

// global index of patch-local velocity element e of component c / pressure element e
struct PatchIndex {
    int N1, bx, by, bz;   // window bases (v_d - 1)(k+1)
    size_t nc;
    template <int K>
    __device__ size_t vel(int c, int e) const {
        int i0, i1, i2;
        vel_coords<K>(c, e, i0, i1, i2);
        i0 += bx;
        i1 += by;
        i2 += bz;
        if (c == 0) return size_t(i0) + size_t(N1 - 1) * (i1 + size_t(N1) * i2);
        if (c == 1) return nc + i0 + size_t(N1) * (i1 + size_t(N1 - 1) * i2);
        return 2 * nc + i0 + size_t(N1) * (i1 + size_t(N1) * i2);
    }
    template <int K>
    __device__ size_t pres(int e) const {
        constexpr int ND = 2 * K + 2;
        const int i0 = bx + e % ND, i1 = by + (e / ND) % ND, i2 = bz + e / (ND * ND);
        return 3 * nc + i0 + size_t(N1) * (i1 + size_t(N1) * i2);
    }
};

// Warm start of the Schur CG (interior patches only): the patch pressure
// predicted by the network, normalized as in its training pairs --
// row b of y holds (U, h P) / s for the interior patch p0 + b of the colour,
// the pressure part at offset 3 NV, and s[b] the input scale.
struct PatchWarm {
    const float* y = nullptr;
    const float* s = nullptr;
    int ldy = 0, p0 = 0;
    int cnt[3] = {0, 0, 0};   // interior vertices per direction of the colour
};

template <int K, typename T, int NTP = 0, bool MF = false>
__global__ void __launch_bounds__((PatchShape<K, NTP>::NT))
patch_solve_kernel(T* __restrict__ x, const T* __restrict__ r, const T* __restrict__ tab, int n, int colour,
                   int cntx, int cnty, T cg_rtol, int cg_maxit, unsigned long long* __restrict__ counters, int boundary_only,
                   PatchWarm warm) {
    using P = PatchShape<K, NTP>;
    using PT = PatchTab<K>;
    constexpr int NV = P::NV, NP = P::NP, ND = P::ND, NW = P::NW;
    __shared__ T s_tab[PT::size];
    __shared__ T V1[3 * NV], W1[3 * NV];
    __shared__ T Pv[NP], R[NP], Dv[NP], Q[NP];
    __shared__ T red[2 * NW];
    __shared__ int codes[3 * NV];
    static_assert(!MF || (sizeof(T) == 4 && K <= 3), "matrix-core eigenbasis products: FP32 cycle, degrees 1..3");
    __shared__ short Qm[MF ? 3 * MfShape<K>::KP * MfShape<K>::KP : 1];

    const int tid = threadIdx.x;
    // vertex of this workgroup: coordinates of parity (colour bit) in 1..n-1
    const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
    // the hardware deals workgroups to the 8 XCDs round robin; the patch of this workgroup is taken so
    // that each XCD gets a contiguous eighth of the colour's patches.  With the plain order the
    // boundary-only launches put every x-boundary patch (first and last of each row of 64 patches)
    // on two XCDs and ran about 10x longer.
    const int b = xcd_contiguous(blockIdx.x, gridDim.x);
    const bool warm_start = warm.y != nullptr;
    int vx, vy, vz;
    if (warm_start) {
        // interior patch p0 + b of the colour (2 <= v_d <= n - 2), in the order of the network's batch
        const int p = warm.p0 + b;
        vx = (px ? 3 : 2) + 2 * (p % warm.cnt[0]);
        vy = (py ? 3 : 2) + 2 * ((p / warm.cnt[0]) % warm.cnt[1]);
        vz = (pz ? 3 : 2) + 2 * (p / (warm.cnt[0] * warm.cnt[1]));
    } else {
        vx = (px ? 1 : 2) + 2 * (b % cntx);
        vy = (py ? 1 : 2) + 2 * ((b / cntx) % cnty);
        vz = (pz ? 1 : 2) + 2 * (b / (cntx * cnty));
    }
    const int tx = (vx == 1 ? 1 : 0) + (vx == n - 1 ? 2 : 0);
    const int ty = (vy == 1 ? 1 : 0) + (vy == n - 1 ? 2 : 0);
    const int tz = (vz == 1 ? 1 : 0) + (vz == n - 1 ? 2 : 0);
    if (boundary_only && (tx | ty | tz) == 0) return;   // whole workgroup: no barrier reached yet
    const int N1 = n * P::M;
    PatchIndex gi{N1, (vx - 1) * P::M, (vy - 1) * P::M, (vz - 1) * P::M, size_t(N1 - 1) * N1 * N1};

    for (int i = tid; i < PT::size; i += P::NT) s_tab[i] = tab[i];
    for (int i = tid; i < 3 * NV; i += P::NT) codes[i] = vel_code<K>(i);
    // gather R_j r: F into V1 (A^{-1} F is formed in place), G into R
    for (int i = tid; i < 3 * NV; i += P::NT) {
        const int c = i / NV;
        V1[i] = r[gi.template vel<K>(c, i - c * NV)];
    }
    for (int i = tid; i < NP; i += P::NT) R[i] = r[gi.template pres<K>(i)];
    __syncthreads();

    // the eigenvector rows: at degrees 1..3 those of the continuous direction (SC) in both precisions, and in FP32
    // all of them, are read through the vector cache (relieves the LDS pipe, which bounds the kernel); the others
    // from LDS (there the vector-cache reads were slower; all measured)
    const T* St = (sizeof(T) == 4 && K <= 3) ? tab : s_tab;
    const T* SC = (K <= 3 ? tab : s_tab) + PT::SC;
    const T* LC = s_tab + PT::LC;
    const T* SDx = St + PT::SD + tx * ND * ND;
    const T* SDy = St + PT::SD + ty * ND * ND;
    const T* SDz = St + PT::SD + tz * ND * ND;
    const T* LDx = s_tab + PT::LDv + tx * ND;
    const T* LDy = s_tab + PT::LDv + ty * ND;
    const T* LDz = s_tab + PT::LDv + tz * ND;
    const T* Dp = s_tab + PT::DP;
    const T* md = s_tab + PT::MDP;
    // per component c and direction d: continuous factors on the diagonal
    const T* Sdir[9] = {SC, SDy, SDz, SDx, SC, SDz, SDx, SDy, SC};
    const T* Ldir[9] = {LC, LDy, LDz, LDx, LC, LDz, LDx, LDy, LC};
    T rinv[entries_per_thread<K, NTP>()];
    fd_reciprocals<K, NTP, T>(rinv, Ldir, codes);
    // A^{-1} by fast diagonalization: every product on the vector units, or (MF) the in-plane ones on the
    // matrix cores (inlined: the LDS arrays keep their address space)
    auto a_inverse = [&](T* vv, T* ww) __attribute__((always_inline)) {
        if constexpr (MF) fd_inverse_mf<K, NTP>(vv, ww, Sdir, rinv, codes, Qm);
        else fd_inverse<K, NTP, T>(vv, ww, Sdir, rinv, codes);
    };
    if constexpr (MF) {
        build_inplane<K, NTP>(Qm, Sdir);
        __syncthreads();
    }

    // G <- G - mean(G)
    {
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) s += R[i];
        const T mean = block_sum<NW>(s, red) / T(NP);
        for (int i = tid; i < NP; i += P::NT) R[i] -= mean;
    }
    // V1 = A^{-1} F;  rhs = B V1 - G (projected)
    a_inverse(V1, W1);
    apply_B<K, NTP, T>(V1, Q, Dp, md);
    __syncthreads();
    T rr;
    {
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) {
            Q[i] -= R[i];
            s += Q[i];
        }
        const T mean = block_sum<NW>(s, red) / T(NP);
        T s2 = 0;
        for (int i = tid; i < NP; i += P::NT) {
            const T v = Q[i] - mean;
            R[i] = v;
            Dv[i] = v;
            Pv[i] = 0;
            s2 += v * v;
        }
        rr = block_sum<NW>(s2, red);
    }
    const T rr0 = rr;   // the cold-start residual: the stopping test refers to it in both cases
    if (warm_start) {
        // P = predicted pressure (mean zero), R = rhs - S P, D = R
        const T ih = T(n);   // 1 / h
        const float sc = warm.s[b];
        const float* yrow = warm.y + size_t(b) * warm.ldy + 3 * NV;
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) {
            const T v = T(sc) * T(yrow[i]) * ih;
            Pv[i] = v;
            s += v;
        }
        const T pmean = block_sum<NW>(s, red) / T(NP);
        for (int i = tid; i < NP; i += P::NT) Pv[i] -= pmean;
        __syncthreads();
        apply_BT<K, NTP, T>(Pv, V1, Dp, md, codes);
        __syncthreads();
        a_inverse(V1, W1);
        apply_B<K, NTP, T>(V1, Q, Dp, md);
        __syncthreads();
        T sq = 0;
        for (int i = tid; i < NP; i += P::NT) sq += Q[i];
        const T qmean = block_sum<NW>(sq, red) / T(NP);
        T s2 = 0;
        for (int i = tid; i < NP; i += P::NT) {
            const T v = R[i] - (Q[i] - qmean);
            R[i] = v;
            Dv[i] = v;
            s2 += v * v;
        }
        rr = block_sum<NW>(s2, red);
    }
    // CG in precision T cannot reduce the residual much below 16 eps: a tighter request is raised
    // to that level (1.9e-6 in FP32, 3.6e-15 in FP64) instead of iterating on rounding noise
    constexpr T kFloor = T(16) * (sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7));
    const T rtol = cg_rtol > kFloor ? cg_rtol : kFloor;
    int it = 0;
    while (it < cg_maxit && rr > rtol * rtol * rr0 && rr > T(0)) {
        // Q = S Dv = B A^{-1} B^T Dv, projected to mean zero
        apply_BT<K, NTP, T>(Dv, V1, Dp, md, codes);
        __syncthreads();
        a_inverse(V1, W1);
        apply_B<K, NTP, T>(V1, Q, Dp, md);
        __syncthreads();
        T s = 0, dq = 0;
        for (int i = tid; i < NP; i += P::NT) {
            s += Q[i];
            dq += Dv[i] * Q[i];
        }
        block_sum2<NW>(s, dq, red);   // Dv has zero mean, so Dv . (Q - mean) = Dv . Q
        // S is positive definite on mean-zero vectors; d.Sd <= 0 (or not finite) only comes from
        // rounding once the iteration has stagnated at the working precision: stop there (the value
        // is uniform over the workgroup, so every thread leaves together)
        if (!(dq > T(0)) || !(dq < T(__builtin_inff()))) break;
        const T mean = s / T(NP);
        const T alpha = rr / dq;
        T s2 = 0;
        for (int i = tid; i < NP; i += P::NT) {
            Pv[i] += alpha * Dv[i];
            const T ri = R[i] - alpha * (Q[i] - mean);
            R[i] = ri;
            s2 += ri * ri;
        }
        const T rr_new = block_sum<NW>(s2, red);
        const T beta = rr_new / rr;
        for (int i = tid; i < NP; i += P::NT) Dv[i] = R[i] + beta * Dv[i];
        rr = rr_new;
        ++it;
        __syncthreads();
    }
    // U = A^{-1} (F - B^T P), F gathered again (r is not written during the colour)
    {
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) s += Pv[i];
        const T mean = block_sum<NW>(s, red) / T(NP);
        for (int i = tid; i < NP; i += P::NT) Pv[i] -= mean;
        __syncthreads();
    }
    apply_BT<K, NTP, T>(Pv, V1, Dp, md, codes);
    __syncthreads();
    for (int i = tid; i < 3 * NV; i += P::NT) {
        const int c = i / NV;
        V1[i] = r[gi.template vel<K>(c, i - c * NV)] - V1[i];
    }
    __syncthreads();
    a_inverse(V1, W1);
    // scatter x += R_j^T (U, P); the DoF sets of one colour are disjoint
    for (int i = tid; i < 3 * NV; i += P::NT) {
        const int c = i / NV;
        const size_t g = gi.template vel<K>(c, i - c * NV);
        x[g] += V1[i];
    }
    for (int i = tid; i < NP; i += P::NT) x[gi.template pres<K>(i)] += Pv[i];
    if (counters && tid == 0) {
        atomicAdd(counters, static_cast<unsigned long long>(it));
        atomicAdd(counters + 1, 1ull);
    }
}

}  // namespace smg
