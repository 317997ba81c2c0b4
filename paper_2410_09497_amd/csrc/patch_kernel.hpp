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

namespace smg {

template <int K>
struct PatchShape {
    static constexpr int M = K + 1;
    static constexpr int NC = 2 * K + 1, ND = 2 * K + 2;
    static constexpr int NV = NC * ND * ND;      // one velocity component
    static constexpr int NP = ND * ND * ND;      // pressure
    static constexpr int NT = 256;
};

// extents (x fastest) of component c: the continuous direction is c
template <int K>
__device__ constexpr int ext(int c, int d) {
    return d == c ? 2 * K + 1 : 2 * K + 2;
}

// block-wide sum of one value per thread (NT = 256: four waves)
template <typename T>
__device__ inline T block_sum(T v, T* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// out[comp] = contraction of in[comp] along direction d with matrix
// S_(comp, d) (transposed if TR), for the three velocity components at once.
template <int K, typename T, bool TR>
__device__ inline void contract3(const T* in, T* out, int d, const T* const* Sdir) {
    using P = PatchShape<K>;
    constexpr int NV = P::NV;
    for (int idx = threadIdx.x; idx < 3 * NV; idx += P::NT) {
        const int c = idx / NV, e = idx - c * NV;
        const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1), e2 = ext<K>(c, 2);
        const int i0 = e % e0, t = e / e0, i1 = t % e1, i2 = t / e1;
        const int nd = d == 0 ? e0 : (d == 1 ? e1 : e2);
        const int ii = d == 0 ? i0 : (d == 1 ? i1 : i2);
        const int st = d == 0 ? 1 : (d == 1 ? e0 : e0 * e1);
        const T* base = in + c * NV + e - ii * st;
        const T* S = Sdir[c * 3 + d];
        T acc = 0;
        for (int j = 0; j < nd; ++j) acc += (TR ? S[j * nd + ii] : S[ii * nd + j]) * base[j * st];
        out[idx] = acc;
    }
}

// v <- A^{-1} v for the three components (in place), work buffers w1, w2
template <int K, typename T>
__device__ inline void fd_inverse(T* v, T* w1, T* w2, const T* const* Sdir, const T* const* Ldir) {
    using P = PatchShape<K>;
    constexpr int NV = P::NV;
    contract3<K, T, true>(v, w1, 0, Sdir);
    __syncthreads();
    contract3<K, T, true>(w1, w2, 1, Sdir);
    __syncthreads();
    contract3<K, T, true>(w2, w1, 2, Sdir);
    __syncthreads();
    for (int idx = threadIdx.x; idx < 3 * NV; idx += P::NT) {
        const int c = idx / NV, e = idx - c * NV;
        const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1);
        const int i0 = e % e0, t = e / e0, i1 = t % e1, i2 = t / e1;
        w1[idx] /= Ldir[c * 3 + 0][i0] + Ldir[c * 3 + 1][i1] + Ldir[c * 3 + 2][i2];
    }
    __syncthreads();
    contract3<K, T, false>(w1, w2, 2, Sdir);
    __syncthreads();
    contract3<K, T, false>(w2, w1, 1, Sdir);
    __syncthreads();
    contract3<K, T, false>(w1, v, 0, Sdir);
    __syncthreads();
}

// vel = B^T p:  (B^T p)_c[i] = -D^T along c times the DG masses of the other directions
template <int K, typename T>
__device__ inline void apply_BT(const T* p, T* vel, const T* Dp, const T* md) {
    using P = PatchShape<K>;
    constexpr int NV = P::NV, NC = P::NC, ND = P::ND;
    for (int idx = threadIdx.x; idx < 3 * NV; idx += P::NT) {
        const int c = idx / NV, e = idx - c * NV;
        const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1);
        const int i[3] = {e % e0, (e / e0) % e1, e / (e0 * e1)};
        // pressure index equals i in the DG directions; the continuous one is summed
        int ps[3] = {1, ND, ND * ND};
        int pbase = 0;
        T mass = 1;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (d != c) {
                pbase += i[d] * ps[d];
                mass *= md[i[d]];
            }
        const int ic = i[c];
        T acc = 0;
        for (int q = 0; q < ND; ++q) acc += Dp[q * NC + ic] * p[pbase + q * ps[c]];
        vel[idx] = -mass * acc;
    }
}

// p = B vel (all three components summed), returns nothing; caller projects
template <int K, typename T>
__device__ inline void apply_B(const T* vel, T* p, const T* Dp, const T* md) {
    using P = PatchShape<K>;
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
        const int e0 = ext<K>(c, 0), e1 = ext<K>(c, 1);
        const int i0 = bx + e % e0, i1 = by + (e / e0) % e1, i2 = bz + e / (e0 * e1);
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

template <int K, typename T>
__global__ void __launch_bounds__(256)
patch_solve_kernel(T* __restrict__ x, const T* __restrict__ r, const T* __restrict__ tab, int n, int colour,
                   int cntx, int cnty, T cg_rtol, int cg_maxit, int* __restrict__ counters, int boundary_only) {
    using P = PatchShape<K>;
    using PT = PatchTab<K>;
    constexpr int NV = P::NV, NP = P::NP, NC = P::NC, ND = P::ND;
    __shared__ T s_tab[PT::size];
    __shared__ T F[3 * NV], V1[3 * NV], W1[3 * NV], W2[3 * NV];
    __shared__ T Pv[NP], R[NP], Dv[NP], Q[NP];
    __shared__ T red[4];

    const int tid = threadIdx.x;
    // vertex of this workgroup: coordinates of parity (colour bit) in 1..n-1
    const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
    const int b = blockIdx.x;
    const int vx = (px ? 1 : 2) + 2 * (b % cntx);
    const int vy = (py ? 1 : 2) + 2 * ((b / cntx) % cnty);
    const int vz = (pz ? 1 : 2) + 2 * (b / (cntx * cnty));
    const int tx = (vx == 1 ? 1 : 0) + (vx == n - 1 ? 2 : 0);
    const int ty = (vy == 1 ? 1 : 0) + (vy == n - 1 ? 2 : 0);
    const int tz = (vz == 1 ? 1 : 0) + (vz == n - 1 ? 2 : 0);
    if (boundary_only && (tx | ty | tz) == 0) return;   // whole workgroup: no barrier reached yet
    const int N1 = n * P::M;
    PatchIndex gi{N1, (vx - 1) * P::M, (vy - 1) * P::M, (vz - 1) * P::M, size_t(N1 - 1) * N1 * N1};

    for (int i = tid; i < PT::size; i += P::NT) s_tab[i] = tab[i];
    // gather R_j r
    for (int i = tid; i < 3 * NV; i += P::NT) {
        const int c = i / NV;
        F[i] = r[gi.template vel<K>(c, i - c * NV)];
    }
    for (int i = tid; i < NP; i += P::NT) R[i] = r[gi.template pres<K>(i)];
    __syncthreads();

    const T* SC = s_tab + PT::SC;
    const T* LC = s_tab + PT::LC;
    const T* SDx = s_tab + PT::SD + tx * ND * ND;
    const T* SDy = s_tab + PT::SD + ty * ND * ND;
    const T* SDz = s_tab + PT::SD + tz * ND * ND;
    const T* LDx = s_tab + PT::LDv + tx * ND;
    const T* LDy = s_tab + PT::LDv + ty * ND;
    const T* LDz = s_tab + PT::LDv + tz * ND;
    const T* Dp = s_tab + PT::DP;
    const T* md = s_tab + PT::MDP;
    // per component c and direction d: continuous factors on the diagonal
    const T* Sdir[9] = {SC, SDy, SDz, SDx, SC, SDz, SDx, SDy, SC};
    const T* Ldir[9] = {LC, LDy, LDz, LDx, LC, LDz, LDx, LDy, LC};

    // G <- G - mean(G)
    {
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) s += R[i];
        const T mean = block_sum(s, red) / T(NP);
        for (int i = tid; i < NP; i += P::NT) R[i] -= mean;
    }
    // V1 = A^{-1} F;  rhs = B V1 - G (projected)
    for (int i = tid; i < 3 * NV; i += P::NT) V1[i] = F[i];
    __syncthreads();
    fd_inverse<K, T>(V1, W1, W2, Sdir, Ldir);
    apply_B<K, T>(V1, Q, Dp, md);
    __syncthreads();
    T rr;
    {
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) {
            Q[i] -= R[i];
            s += Q[i];
        }
        const T mean = block_sum(s, red) / T(NP);
        T s2 = 0;
        for (int i = tid; i < NP; i += P::NT) {
            const T v = Q[i] - mean;
            R[i] = v;
            Dv[i] = v;
            Pv[i] = 0;
            s2 += v * v;
        }
        rr = block_sum(s2, red);
    }
    const T rr0 = rr;
    int it = 0;
    while (it < cg_maxit && rr > cg_rtol * cg_rtol * rr0 && rr > T(0)) {
        // Q = S Dv = B A^{-1} B^T Dv, projected to mean zero
        apply_BT<K, T>(Dv, V1, Dp, md);
        __syncthreads();
        fd_inverse<K, T>(V1, W1, W2, Sdir, Ldir);
        apply_B<K, T>(V1, Q, Dp, md);
        __syncthreads();
        T s = 0, dq = 0;
        for (int i = tid; i < NP; i += P::NT) {
            s += Q[i];
            dq += Dv[i] * Q[i];
        }
        s = block_sum(s, red);
        dq = block_sum(dq, red);   // Dv has zero mean, so Dv . (Q - mean) = Dv . Q
        const T mean = s / T(NP);
        const T alpha = rr / dq;
        T s2 = 0;
        for (int i = tid; i < NP; i += P::NT) {
            Pv[i] += alpha * Dv[i];
            const T ri = R[i] - alpha * (Q[i] - mean);
            R[i] = ri;
            s2 += ri * ri;
        }
        const T rr_new = block_sum(s2, red);
        const T beta = rr_new / rr;
        for (int i = tid; i < NP; i += P::NT) Dv[i] = R[i] + beta * Dv[i];
        rr = rr_new;
        ++it;
        __syncthreads();
    }
    // U = A^{-1} (F - B^T P)
    {
        T s = 0;
        for (int i = tid; i < NP; i += P::NT) s += Pv[i];
        const T mean = block_sum(s, red) / T(NP);
        for (int i = tid; i < NP; i += P::NT) Pv[i] -= mean;
        __syncthreads();
    }
    apply_BT<K, T>(Pv, V1, Dp, md);
    __syncthreads();
    for (int i = tid; i < 3 * NV; i += P::NT) V1[i] = F[i] - V1[i];
    __syncthreads();
    fd_inverse<K, T>(V1, W1, W2, Sdir, Ldir);
    // scatter x += R_j^T (U, P); the DoF sets of one colour are disjoint
    for (int i = tid; i < 3 * NV; i += P::NT) {
        const int c = i / NV;
        const size_t g = gi.template vel<K>(c, i - c * NV);
        x[g] += V1[i];
    }
    for (int i = tid; i < NP; i += P::NT) x[gi.template pres<K>(i)] += Pv[i];
    if (counters && tid == 0) {
        atomicAdd(counters, it);
        atomicAdd(counters + 1, 1);
    }
}

}  // namespace smg
