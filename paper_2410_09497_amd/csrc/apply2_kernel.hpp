// Fused operator y = K x / residual r = b - K x for degrees k = 1..3 (gfx950).
//
// Same separable form as the generic kernel (Sec. 2.2; Kronecker factors of
// Eqs. block_A and b extended to 3D), reorganised so that every stencil
// coefficient is a compile-time constant:
//
//  * a workgroup owns a tile of 8 x 8 cells in xy and marches through a chunk
//    of cell layers in z; it has one wave per in-cell position (A, B) in the
//    xy plane, (k+1)^2 waves, and lane l of every wave owns cell
//    (l mod 8, l div 8) of the tile.  A wave's position in the cell is
//    uniform, so its x and y rows of every 1D matrix are fixed at compile time
//    (one instantiation per (A, B), selected by a wave-uniform branch);
//  * each z-plane of the four fields is loaded with coalesced row reads into
//    LDS in a cell-strided layout [b][a][cell y][cell x], so the neighbours a
//    lane needs are at compile-time offsets from its own address;
//  * the z direction streams through registers: the discontinuous z coupling
//    of the interior-penalty terms needs only two face traces per
//    neighbouring layer, the continuous z direction only the shared node, so
//    a lane keeps ~7(k+1)+14 accumulators; the next plane is prefetched into
//    registers while the current one is computed.
//
// Reference scaling (h = 1 tables, penalty gamma h = 2 (k+1)^2): with
// v = Mc_x u_x, s = w_b Ld_x u_z + w_a Ld_y u_z,
//   y_x = h [w_b w_c Kc u_x + w_c Ld_y v + w_b Ld_z v - h w_b w_c D^T p]
//   y_z = h [Mc_z s + w_a w_b Kc_z u_z - h w_a w_b D^T_z p]
//   y_p = -h^2 [w_b w_c D_x u_x + w_a w_c D_y u_y + w_a w_b D_z u_z].
// Rows of the first/last cell in a direction (domain boundary faces of
// Eq. bilinear) are the interior row plus the rank-two boundary correction;
// neighbour values outside the domain read as zero.
#pragma once

#include <hip/hip_runtime.h>

#include "ref_tables_gen.hpp"

namespace smg {

template <int K>
struct Ap2 {
    static constexpr int M = K + 1;
    static constexpr int C = 8;              // cells per tile side
    static constexpr int H = C + 2;          // with a one-cell halo
    static constexpr int PX = H;             // cell stride in x inside LDS
    static constexpr int NW = M * M;         // waves per workgroup
    static constexpr int NT = 64 * NW;       // threads
    static constexpr int UC = M * M * H * PX;  // one field plane: [b][a][cy][cx]
    static constexpr int VXN = M * M * H * C;  // Mc_x u_x: [b][a][cy (halo)][cx]
    static constexpr int VYN = M * M * C * PX; // Mc_y u_y: [b][a][cy][cx (halo)]
    static constexpr int REG = 10 * M * 10 * M;  // loaded region of one field
    static constexpr int NLOAD = (REG + NT - 1) / NT;
    // occupancy target (waves per SIMD) that the register budget is sized for
    static constexpr int WPE = (K == 2) ? 3 : 4;
};

__device__ inline int xcd_remap2(int bid, int G) {
    const int xcd = bid & 7, local = bid >> 3;
    const int per = G >> 3, extra = G & 7;
    return xcd * per + (xcd < extra ? xcd : extra) + local;
}

// Raw buffer access: a uniform descriptor per z-plane (base = plane start,
// size = plane bytes) and a 32-bit per-lane byte offset.  The hardware range
// check makes out-of-domain offsets read zero and drops their stores.
constexpr int kBufFlags = 0x00020000;
constexpr int kOOB = 0x7ffffff0;      // a lane offset beyond any plane

__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, size_t off_elems, int elem, size_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(static_cast<const char*>(base)) + off_elems * elem, 0, int(nbytes), kBufFlags);
}

template <typename T>
__device__ inline T buf_ld(__amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <typename T>
__device__ inline void buf_st(__amdgpu_buffer_rsrc_t r, int off, T v) {
    if constexpr (sizeof(T) == 8) {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, off, 0, 0);
    } else {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, v), r, off, 0, 0);
    }
}

template <int K, typename T>
struct Ap2Ctx {
    const T* __restrict__ x;
    const T* __restrict__ bv;
    T* __restrict__ y;
    T* U;         // [4][UC]
    T* VX;
    T* VY;
    int n, N1, L0, L1, gcx, gcy, lane;
    size_t nc;
    T h;
    // loader: LDS element index (-1: none) and byte offsets inside a plane
    int lidx[Ap2<K>::NLOAD];
    int ox[Ap2<K>::NLOAD], oy[Ap2<K>::NLOAD], ozp[Ap2<K>::NLOAD];
};

template <int K, int A, int B, typename T, bool RESID>
__device__ __forceinline__ void apply2_body(const Ap2Ctx<K, T>& cx_) {
    using R = ref::R<K>;
    using S = Ap2<K>;
    constexpr int M = S::M, H = S::H, PX = S::PX, UC = S::UC, NL = S::NLOAD;
    const int n = cx_.n, N1 = cx_.N1, L0 = cx_.L0, L1 = cx_.L1;
    const T h = cx_.h;
    const int lane = cx_.lane;
    const int cx = lane & 7, cy = lane >> 3;
    const bool own_ok = cx_.gcx + cx < n && cx_.gcy + cy < n;
    const int gcx = cx_.gcx + cx, gcy = cx_.gcy + cy;
    const size_t nc = cx_.nc;
    const size_t sxy = size_t(N1 - 1) * N1, szp = size_t(N1) * N1;
    constexpr int E = sizeof(T);

    // element (field f, position (a', b'), halo cell (cyh, cxh)) of an LDS plane
    auto ui = [](int f, int bb, int aa, int cyh, int cxh) { return (((f * M + bb) * M + aa) * H + cyh) * PX + cxh; };

    // -------------------------------------------------------------- state
    // ax/ay: rows of layers Lin-1 (cur) and Lin (new); az_new: continuous-z
    // rows of layer Lin (the last one is the node shared with Lin+1), az_sh:
    // the shared node of layer Lin-1, still open
    T ax_cur[M], ax_new[M], ay_cur[M], ay_new[M], az_new[M], ap_new[M];
    T az_sh = 0;
#pragma unroll
    for (int i = 0; i < M; ++i) ax_cur[i] = ax_new[i] = ay_cur[i] = ay_new[i] = az_new[i] = ap_new[i] = T(0);
    T tx_eL = 0, tx_dL = 0, tx_eR = 0, tx_dR = 0, ty_eL = 0, ty_dL = 0, ty_eR = 0, ty_dR = 0;
    T tx_eRp = 0, tx_dRp = 0, ty_eRp = 0, ty_dRp = 0;
    T s_prev = 0, uz_prev = 0, s_last = 0, uz_last = 0;

    constexpr T gp = T(R::gp);
    constexpr T wA = T(R::w[A]), wB = T(R::w[B]);

    T pre[4][NL];
    const int zfirst = (L0 > 0 ? L0 - 1 : 0) * M;
    const int zlast = (L1 < n ? L1 : n - 1) * M + M - 1;

    auto load_plane = [&](int Z) {
        const auto rx = plane_rsrc(cx_.x, sxy * Z, E, sxy * E);
        const auto ry = plane_rsrc(cx_.x, nc + sxy * Z, E, sxy * E);
        const auto rz = plane_rsrc(cx_.x, 2 * nc + szp * Z, E, Z < N1 - 1 ? szp * E : 0);
        const auto rp = plane_rsrc(cx_.x, 3 * nc + szp * Z, E, szp * E);
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            pre[0][r] = buf_ld<T>(rx, cx_.ox[r]);
            pre[1][r] = buf_ld<T>(ry, cx_.oy[r]);
            pre[2][r] = buf_ld<T>(rz, cx_.ozp[r]);
            pre[3][r] = buf_ld<T>(rp, cx_.ozp[r]);
        }
    };
    load_plane(zfirst);

    for (int Lin = L0 - 1; Lin <= L1; ++Lin) {
        const bool have = Lin >= 0 && Lin < n;
        if (have) {
            // start of layer: coupling from layer Lin-1 (its top traces), node 0 of the cell
#pragma unroll
            for (int c = 0; c < M; ++c) {
                ax_new[c] = wB * (T(R::eL[c]) * (-gp * tx_eRp + T(0.5) * tx_dRp) - T(R::dL[c]) * T(0.5) * tx_eRp);
                ay_new[c] = wA * (T(R::eL[c]) * (-gp * ty_eRp + T(0.5) * ty_dRp) - T(R::dL[c]) * T(0.5) * ty_eRp);
                ap_new[c] = -wA * wB * T(R::D[c][0]) * uz_prev;
            }
            az_sh += T(R::Mc[0][0]) * s_prev + wA * wB * T(R::Kc[0][0]) * uz_prev;
#pragma unroll
            for (int j = 1; j <= M; ++j) az_new[j - 1] = T(R::Mc[j][0]) * s_prev + wA * wB * T(R::Kc[j][0]) * uz_prev;
            tx_eL = tx_dL = tx_eR = tx_dR = ty_eL = ty_dL = ty_eR = ty_dR = T(0);

#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int Z = Lin * M + c;
                T* Ub = cx_.U;
                // 1) prefetched plane -> LDS (single buffer: the previous plane's readers are done)
                __syncthreads();
#pragma unroll
                for (int r = 0; r < NL; ++r) {
                    const int li = cx_.lidx[r];
                    if (li >= 0) {
                        Ub[li] = pre[0][r];
                        Ub[UC + li] = pre[1][r];
                        Ub[2 * UC + li] = pre[2][r];
                        Ub[3 * UC + li] = pre[3][r];
                    }
                }
                __syncthreads();
                if (Z < zlast) load_plane(Z + 1);
                const T* Ux = Ub;
                const T* Uy = Ub + UC;
                const T* Uz = Ub + 2 * UC;
                const T* Pp = Ub + 3 * UC;

                // 2) v = Mc_x u_x at (A, B) on tile columns x all halo rows; Mc_y u_y on all halo columns x tile rows
                auto mcx = [&](int cyh, int cxh) {       // node j of cell (cxh) on row (cyh, B)
                    T acc = 0;
#pragma unroll
                    for (int j = 0; j <= M; ++j) {
                        const T v = (j == 0) ? Ux[ui(0, B, M - 1, cyh, cxh - 1)] : Ux[ui(0, B, j - 1, cyh, cxh)];
                        acc += T(R::Mc[A + 1][j]) * v;
                    }
                    if constexpr (A == M - 1) {
#pragma unroll
                        for (int j = 1; j <= M; ++j) acc += T(R::Mc[0][j]) * Ux[ui(0, B, j - 1, cyh, cxh + 1)];
                        acc += T(R::Mc[0][0]) * Ux[ui(0, B, M - 1, cyh, cxh)];
                    }
                    return acc;
                };
                auto mcy = [&](int cyh, int cxh) {
                    T acc = 0;
#pragma unroll
                    for (int j = 0; j <= M; ++j) {
                        const T v = (j == 0) ? Uy[ui(0, M - 1, A, cyh - 1, cxh)] : Uy[ui(0, j - 1, A, cyh, cxh)];
                        acc += T(R::Mc[B + 1][j]) * v;
                    }
                    if constexpr (B == M - 1) {
#pragma unroll
                        for (int j = 1; j <= M; ++j) acc += T(R::Mc[0][j]) * Uy[ui(0, j - 1, A, cyh + 1, cxh)];
                        acc += T(R::Mc[0][0]) * Uy[ui(0, M - 1, A, cyh, cxh)];
                    }
                    return acc;
                };
                // VX[b][a][cyh][cx], VY[b][a][cy][cxh]
                cx_.VX[((B * M + A) * H + cy + 1) * S::C + cx] = mcx(cy + 1, cx + 1);
                cx_.VY[((B * M + A) * S::C + cy) * PX + cx + 1] = mcy(cy + 1, cx + 1);
                if (lane < 16) {
                    const int e = lane & 7, side = (lane >> 3) ? H - 1 : 0;
                    cx_.VX[((B * M + A) * H + side) * S::C + e] = mcx(side, e + 1);
                    cx_.VY[((B * M + A) * S::C + e) * PX + side] = mcy(e + 1, side);
                }
                __syncthreads();

                // 3) in-plane rows at (A, B) of this lane's cell
                const int cyh = cy + 1, cxh = cx + 1;
                auto uxn = [&](int j, int dcx) {          // u_x at node j of cell cx+dcx, row (cy, B)
                    return (j == 0) ? Ux[ui(0, B, M - 1, cyh, cxh + dcx - 1)] : Ux[ui(0, B, j - 1, cyh, cxh + dcx)];
                };
                auto uyn = [&](int j, int dcy) {
                    return (j == 0) ? Uy[ui(0, M - 1, A, cyh + dcy - 1, cxh)] : Uy[ui(0, j - 1, A, cyh + dcy, cxh)];
                };
                T lcx = 0, dtx = 0, dxux = 0, lcy = 0, dty = 0, dyuy = 0;
#pragma unroll
                for (int j = 0; j <= M; ++j) {
                    const T vx0 = uxn(j, 0), vy0 = uyn(j, 0);
                    lcx += T(R::Kc[A + 1][j]) * vx0;
                    dxux += T(R::D[A][j]) * vx0;
                    lcy += T(R::Kc[B + 1][j]) * vy0;
                    dyuy += T(R::D[B][j]) * vy0;
                }
                if constexpr (A == M - 1) {
#pragma unroll
                    for (int j = 0; j <= M; ++j) lcx += T(R::Kc[0][j]) * uxn(j, 1);
                }
                if constexpr (B == M - 1) {
#pragma unroll
                    for (int j = 0; j <= M; ++j) lcy += T(R::Kc[0][j]) * uyn(j, 1);
                }
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    dtx += T(R::D[q][A + 1]) * Pp[ui(0, B, q, cyh, cxh)];
                    dty += T(R::D[q][B + 1]) * Pp[ui(0, q, A, cyh, cxh)];
                    if constexpr (A == M - 1) dtx += T(R::D[q][0]) * Pp[ui(0, B, q, cyh, cxh + 1)];
                    if constexpr (B == M - 1) dty += T(R::D[q][0]) * Pp[ui(0, q, A, cyh + 1, cxh)];
                }
                // keep the scheduler from hoisting every LDS read of the plane at once
                __builtin_amdgcn_sched_barrier(0);
                // discontinuous rows: Ld_x on Mc_y u_y and on u_z, Ld_y on Mc_x u_x and on u_z
                T ldx_vy = 0, ldx_uz = 0, ldy_vx = 0, ldy_uz = 0;
#pragma unroll
                for (int d = -1; d <= 1; ++d) {
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const T cxr = T(R::Ld[A][(d + 1) * M + q]);
                        const T cyr = T(R::Ld[B][(d + 1) * M + q]);
                        ldx_vy += cxr * cx_.VY[((B * M + q) * S::C + cy) * PX + cxh + d];
                        ldx_uz += cxr * Uz[ui(0, B, q, cyh, cxh + d)];
                        ldy_vx += cyr * cx_.VX[((q * M + A) * H + cyh + d) * S::C + cx];
                        ldy_uz += cyr * Uz[ui(0, q, A, cyh + d, cxh)];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                // boundary rows (first / last cell of the mesh in x or y)
                if (gcx == 0 || gcx == n - 1) {
                    T tvL = 0, tvD = 0, tuL = 0, tuD = 0, tvR = 0, tvDR = 0, tuR = 0, tuDR = 0;
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const T vv = cx_.VY[((B * M + q) * S::C + cy) * PX + cxh];
                        const T uu = Uz[ui(0, B, q, cyh, cxh)];
                        tvL += T(R::eL[q]) * vv; tvD += T(R::dL[q]) * vv;
                        tuL += T(R::eL[q]) * uu; tuD += T(R::dL[q]) * uu;
                        tvR += T(R::eR[q]) * vv; tvDR += T(R::dR[q]) * vv;
                        tuR += T(R::eR[q]) * uu; tuDR += T(R::dR[q]) * uu;
                    }
                    if (gcx == 0) {
                        ldx_vy += T(R::eL[A]) * (gp * tvL + T(0.5) * tvD) + T(R::dL[A]) * T(0.5) * tvL;
                        ldx_uz += T(R::eL[A]) * (gp * tuL + T(0.5) * tuD) + T(R::dL[A]) * T(0.5) * tuL;
                    }
                    if (gcx == n - 1) {
                        ldx_vy += T(R::eR[A]) * (gp * tvR - T(0.5) * tvDR) - T(R::dR[A]) * T(0.5) * tvR;
                        ldx_uz += T(R::eR[A]) * (gp * tuR - T(0.5) * tuDR) - T(R::dR[A]) * T(0.5) * tuR;
                    }
                }
                if (gcy == 0 || gcy == n - 1) {
                    T tvL = 0, tvD = 0, tuL = 0, tuD = 0, tvR = 0, tvDR = 0, tuR = 0, tuDR = 0;
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const T vv = cx_.VX[((q * M + A) * H + cyh) * S::C + cx];
                        const T uu = Uz[ui(0, q, A, cyh, cxh)];
                        tvL += T(R::eL[q]) * vv; tvD += T(R::dL[q]) * vv;
                        tuL += T(R::eL[q]) * uu; tuD += T(R::dL[q]) * uu;
                        tvR += T(R::eR[q]) * vv; tvDR += T(R::dR[q]) * vv;
                        tuR += T(R::eR[q]) * uu; tuDR += T(R::dR[q]) * uu;
                    }
                    if (gcy == 0) {
                        ldy_vx += T(R::eL[B]) * (gp * tvL + T(0.5) * tvD) + T(R::dL[B]) * T(0.5) * tvL;
                        ldy_uz += T(R::eL[B]) * (gp * tuL + T(0.5) * tuD) + T(R::dL[B]) * T(0.5) * tuL;
                    }
                    if (gcy == n - 1) {
                        ldy_vx += T(R::eR[B]) * (gp * tvR - T(0.5) * tvDR) - T(R::dR[B]) * T(0.5) * tvR;
                        ldy_uz += T(R::eR[B]) * (gp * tuR - T(0.5) * tuDR) - T(R::dR[B]) * T(0.5) * tuR;
                    }
                }
                const T vxo = cx_.VX[((B * M + A) * H + cyh) * S::C + cx];
                const T vyo = cx_.VY[((B * M + A) * S::C + cy) * PX + cxh];
                const T uzo = Uz[ui(0, B, A, cyh, cxh)];
                const T po = Pp[ui(0, B, A, cyh, cxh)];

                // 4) in-plane parts of the rows of plane c
                const T wc = T(R::w[c]);
                ax_new[c] += wB * wc * lcx + wc * ldy_vx - h * wB * wc * dtx;
                ay_new[c] += wA * wc * lcy + wc * ldx_vy - h * wA * wc * dty;
                ap_new[c] += -(wB * wc * dxux + wA * wc * dyuy);
                const T s = wB * ldx_uz + wA * ldy_uz;

                // 5) z direction, streamed: own block of Ld_z, face traces, Mc_z / Kc_z / D_z columns
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    ax_new[q] += wB * T(R::Ld[q][M + c]) * vxo;
                    ay_new[q] += wA * T(R::Ld[q][M + c]) * vyo;
                    ap_new[q] += -wA * wB * T(R::D[q][c + 1]) * uzo;
                }
                tx_eL += T(R::eL[c]) * vxo; tx_dL += T(R::dL[c]) * vxo;
                tx_eR += T(R::eR[c]) * vxo; tx_dR += T(R::dR[c]) * vxo;
                ty_eL += T(R::eL[c]) * vyo; ty_dL += T(R::dL[c]) * vyo;
                ty_eR += T(R::eR[c]) * vyo; ty_dR += T(R::dR[c]) * vyo;
                az_sh += T(R::Mc[0][c + 1]) * s + wA * wB * T(R::Kc[0][c + 1]) * uzo - h * wA * wB * T(R::D[c][0]) * po;
#pragma unroll
                for (int j = 1; j <= M; ++j)
                    az_new[j - 1] += T(R::Mc[j][c + 1]) * s + wA * wB * T(R::Kc[j][c + 1]) * uzo -
                                     h * wA * wB * T(R::D[c][j]) * po;
                if (c == M - 1) {
                    s_last = s;
                    uz_last = uzo;
                }
            }

            // end of layer: coupling Lin -> Lin-1, boundary corrections of layer Lin
#pragma unroll
            for (int c = 0; c < M; ++c) {
                ax_cur[c] += wB * (T(R::eR[c]) * (-gp * tx_eL - T(0.5) * tx_dL) + T(R::dR[c]) * T(0.5) * tx_eL);
                ay_cur[c] += wA * (T(R::eR[c]) * (-gp * ty_eL - T(0.5) * ty_dL) + T(R::dR[c]) * T(0.5) * ty_eL);
            }
            if (Lin == 0) {
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    ax_new[c] += wB * (T(R::eL[c]) * (gp * tx_eL + T(0.5) * tx_dL) + T(R::dL[c]) * T(0.5) * tx_eL);
                    ay_new[c] += wA * (T(R::eL[c]) * (gp * ty_eL + T(0.5) * ty_dL) + T(R::dL[c]) * T(0.5) * ty_eL);
                }
            }
            if (Lin == n - 1) {
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    ax_new[c] += wB * (T(R::eR[c]) * (gp * tx_eR - T(0.5) * tx_dR) - T(R::dR[c]) * T(0.5) * tx_eR);
                    ay_new[c] += wA * (T(R::eR[c]) * (gp * ty_eR - T(0.5) * ty_dR) - T(R::dR[c]) * T(0.5) * ty_eR);
                }
            }
            // pressure rows and the first M-1 continuous-z rows of layer Lin are complete,
            // and so is the shared z node of layer Lin-1
            {
                const int X = gcx * M + A, Y = gcy * M + B;
                const int oz = own_ok ? (X + N1 * Y) * E : kOOB;
                if (Lin >= L0 && Lin < L1) {
#pragma unroll
                    for (int c = 0; c < M; ++c) {
                        const size_t po = 3 * nc + szp * (Lin * M + c);
                        T v = h * h * ap_new[c];
                        if constexpr (RESID) v = buf_ld<T>(plane_rsrc(cx_.bv, po, E, szp * E), oz) - v;
                        buf_st<T>(plane_rsrc(cx_.y, po, E, szp * E), oz, v);
                    }
#pragma unroll
                    for (int c = 0; c < M - 1; ++c) {
                        const int Z = Lin * M + c;
                        const size_t bz = 2 * nc + szp * Z;
                        const size_t nzb = Z < N1 - 1 ? szp * E : 0;
                        T v = h * az_new[c];
                        if constexpr (RESID) v = buf_ld<T>(plane_rsrc(cx_.bv, bz, E, nzb), oz) - v;
                        buf_st<T>(plane_rsrc(cx_.y, bz, E, nzb), oz, v);
                    }
                }
                if (Lin - 1 >= L0 && Lin - 1 < L1) {
                    const int Z = (Lin - 1) * M + M - 1;
                    const size_t bz = 2 * nc + szp * Z;
                    const size_t nzb = Z < N1 - 1 ? szp * E : 0;
                    T v = h * az_sh;
                    if constexpr (RESID) v = buf_ld<T>(plane_rsrc(cx_.bv, bz, E, nzb), oz) - v;
                    buf_st<T>(plane_rsrc(cx_.y, bz, E, nzb), oz, v);
                }
                az_sh = az_new[M - 1];
            }
        }
        // velocity rows of layer Lin-1 are complete
        const int L = Lin - 1;
        if (L >= L0 && L < L1) {
            const int X = gcx * M + A, Y = gcy * M + B;
            const int ox = (own_ok && X < N1 - 1) ? (X + (N1 - 1) * Y) * E : kOOB;
            const int oy = (own_ok && Y < N1 - 1) ? (X + N1 * Y) * E : kOOB;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int Z = L * M + c;
                const size_t bx = sxy * Z, by = nc + sxy * Z;
                T vx = h * ax_cur[c], vy = h * ay_cur[c];
                if constexpr (RESID) {
                    vx = buf_ld<T>(plane_rsrc(cx_.bv, bx, E, sxy * E), ox) - vx;
                    vy = buf_ld<T>(plane_rsrc(cx_.bv, by, E, sxy * E), oy) - vy;
                }
                buf_st<T>(plane_rsrc(cx_.y, bx, E, sxy * E), ox, vx);
                buf_st<T>(plane_rsrc(cx_.y, by, E, sxy * E), oy, vy);
            }
        }
        // slide by one layer
#pragma unroll
        for (int c = 0; c < M; ++c) {
            ax_cur[c] = have ? ax_new[c] : T(0);
            ay_cur[c] = have ? ay_new[c] : T(0);
        }
        tx_eRp = have ? tx_eR : T(0);
        tx_dRp = have ? tx_dR : T(0);
        ty_eRp = have ? ty_eR : T(0);
        ty_dRp = have ? ty_dR : T(0);
        s_prev = have ? s_last : T(0);
        uz_prev = have ? uz_last : T(0);
    }
}

template <int K, typename T, bool RESID, int W>
__device__ __forceinline__ void apply2_dispatch(int wave, const Ap2Ctx<K, T>& c) {
    constexpr int M = K + 1;
    if constexpr (W < M * M) {
        if (wave == W)
            apply2_body<K, W % M, W / M, T, RESID>(c);
        else
            apply2_dispatch<K, T, RESID, W + 1>(wave, c);
    }
}

template <int K, typename T, bool RESID>
__global__ void __launch_bounds__(64 * (K + 1) * (K + 1)) __attribute__((amdgpu_waves_per_eu(Ap2<K>::WPE, 8)))
apply2_kernel(const T* __restrict__ x, const T* __restrict__ bv, T* __restrict__ y, int n, int cz, int tiles,
              T h) {
    using S = Ap2<K>;
    constexpr int M = S::M;
    __shared__ T U[4 * S::UC];
    __shared__ T VX[S::VXN];
    __shared__ T VY[S::VYN];
    const int tid = threadIdx.x;
    const int lin = xcd_remap2(blockIdx.x, gridDim.x);
    const int tile_x = lin % tiles, rest = lin / tiles;
    const int tile_y = rest % tiles, zc = rest / tiles;
    Ap2Ctx<K, T> c;
    c.x = x;
    c.bv = bv;
    c.y = y;
    c.U = U;
    c.VX = VX;
    c.VY = VY;
    c.n = n;
    c.N1 = n * M;
    c.L0 = zc * cz;
    c.L1 = (c.L0 + cz < n) ? c.L0 + cz : n;
    c.gcx = tile_x * S::C;
    c.gcy = tile_y * S::C;
    c.lane = tid & 63;
    c.nc = size_t(c.N1 - 1) * c.N1 * c.N1;
    c.h = h;
    const int X0 = c.gcx * M, Y0 = c.gcy * M, N1 = c.N1;
#pragma unroll
    for (int r = 0; r < S::NLOAD; ++r) {
        const int e = tid + S::NT * r;
        c.lidx[r] = -1;
        c.ox[r] = c.oy[r] = c.ozp[r] = kOOB;
        if (e < S::REG) {
            const int Yr = e / (10 * M), Xr = e % (10 * M);
            const int X = X0 - M + Xr, Y = Y0 - M + Yr;
            c.lidx[r] = (((Yr % M) * M + Xr % M) * S::H + Yr / M) * S::PX + Xr / M;
            const bool in = X >= 0 && X < N1 && Y >= 0 && Y < N1;
            constexpr int E = sizeof(T);
            if (in && X < N1 - 1) c.ox[r] = (X + (N1 - 1) * Y) * E;
            if (in && Y < N1 - 1) c.oy[r] = (X + N1 * Y) * E;
            if (in) c.ozp[r] = (X + N1 * Y) * E;
        }
    }
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    apply2_dispatch<K, T, RESID, 0>(wave, c);
}

}  // namespace smg
