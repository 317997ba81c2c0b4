// Fused matrix-free operator y = K x (or residual r = b - K x) for the
// H(div)-DG Stokes discretization (Alg. 1), gfx950.
//
// Every term of K is a Kronecker product with at most two non-diagonal 1D
// factors (stencil_tables.hpp).  Per component c (continuous direction c):
//   y_c = mm (Lc_c u_c - D^T_c p) + sum_{d != c} m_e Ld_d (Mc_c u_c)
//   y_p = -sum_c mm D_c u_c
// with mm the two diagonal DG masses of the other directions and m_e the one
// of the third direction.  Each face of Eq. bilinear is inside an Ld row, so
// the cell, interior-face and boundary-face loops of Alg. 1 are all carried
// by the rows: every face is evaluated once, by the owner of each output.
//
// Work decomposition (2.5D): one workgroup owns a tile of CX x CY cells in
// the xy plane and marches through a chunk of cell layers in z.  One thread
// owns one xy position (one DoF column) of the tile.
//  * in-plane (x, y) stencils read one z-plane of all four fields, with a
//    one-cell halo, from LDS; the halo comes from L2 (neighbouring tiles of
//    one XCD read it too);
//  * z stencils are evaluated in registers from a sliding window of three
//    cell layers per thread: no z halo except one layer at each chunk end.
// Each input element is read from HBM once per chunk and each output written
// once: 2 words per unknown (apply), 3 (residual).
#pragma once

#include <hip/hip_runtime.h>

#include "stencil_tables.hpp"

namespace smg {

template <int K, int CX, int CY>
struct ApplyShape {
    static constexpr int M = K + 1;
    static constexpr int TX = CX * M, TY = CY * M;   // tile positions
    static constexpr int NT = TX * TY;               // threads
    static constexpr int RX = TX + 2 * M, RY = TY + 2 * M;
    static constexpr int RS = RX * RY;               // LDS plane with halo
};

// blockIdx -> tile so that consecutive tiles sit on the same XCD (the
// hardware deals workgroups to the 8 XCDs round robin).
__device__ inline int xcd_remap(int bid, int G) {
    const int xcd = bid & 7, local = bid >> 3;
    const int per = G >> 3, extra = G & 7;
    return xcd * per + (xcd < extra ? xcd : extra) + local;
}

// PF: the next plane's global loads are issued into registers before the
// current plane is computed (software pipelining), and stored to LDS at the
// start of the next plane; otherwise each plane is loaded, then computed.
template <int K, typename T, int CX, int CY, bool RESID, bool PF>
__global__ void __launch_bounds__(CX * CY * (K + 1) * (K + 1))
stokes_apply_kernel(const T* __restrict__ x, const T* __restrict__ bvec, T* __restrict__ y,
                    const T* __restrict__ tab, int n, int cz, int tiles_x, int tiles_y) {
    using S = ApplyShape<K, CX, CY>;
    constexpr int M = S::M, TX = S::TX, TY = S::TY, NT = S::NT, RX = S::RX, RY = S::RY, RS = S::RS;
    constexpr int NL = (RS + NT - 1) / NT;   // plane elements per thread and field
    using TB = Tab<K>;

    __shared__ T s_tab[TB::size];
    __shared__ T s_u[2][4][RS];      // ux, uy, uz, p planes (double buffered)
    __shared__ T s_vx[TX * RY];      // Mc_x ux over tile columns x all region rows
    __shared__ T s_vy[RX * TY];      // Mc_y uy over all region columns x tile rows

    const int tid = threadIdx.x;
    for (int i = tid; i < TB::size; i += NT) s_tab[i] = tab[i];

    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_x = lin % tiles_x;
    const int rest = lin / tiles_x;
    const int tile_y = rest % tiles_y;
    const int zc = rest / tiles_y;
    const int N1 = n * M;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int tx = tid % TX, ty = tid / TX;
    const int X = X0 + tx, Y = Y0 + ty;
    const int a = tx % M, b = ty % M;                 // position in cell (tiles are cell aligned)
    const int vxv = ld_variant(X / M, n), vyv = ld_variant(Y / M, n);
    const int L0 = zc * cz;
    const int L1 = (L0 + cz < n) ? L0 + cz : n;

    const size_t nc = size_t(N1 - 1) * N1 * N1;
    const T* __restrict__ gx = x;
    const T* __restrict__ gy = x + nc;
    const T* __restrict__ gz = x + 2 * nc;
    const T* __restrict__ gp = x + 3 * nc;

    // sliding windows over three layers (prev | cur | next), M planes each
    T wvx[3 * M], wvy[3 * M], ws[3 * M], wuz[3 * M], wp[3 * M];
    T pix[2][M], piy[2][M], pip[2][M];               // in-plane partials (cur, next)
#pragma unroll
    for (int i = 0; i < 3 * M; ++i) wvx[i] = wvy[i] = ws[i] = wuz[i] = wp[i] = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) pix[0][i] = piy[0][i] = pip[0][i] = pix[1][i] = piy[1][i] = pip[1][i] = T(0);

    __syncthreads();
    const T* __restrict__ MC = s_tab + TB::MC;
    const T* __restrict__ LC = s_tab + TB::LC;
    const T* __restrict__ DT = s_tab + TB::DT;
    const T* __restrict__ DD = s_tab + TB::DD;
    const T* __restrict__ LD = s_tab + TB::LD;
    const T* __restrict__ MD = s_tab + TB::MDg;
    const T mda = MD[a], mdb = MD[b];

    // plane Z of the four fields, tile + halo, zero outside the domain
    auto load_plane = [&](int Z, T (&v)[4][NL]) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int i = tid + t * NT;
            const int gxp = X0 - M + i % RX, gyp = Y0 - M + i / RX;
            const bool in = i < RS && gxp >= 0 && gxp < N1 && gyp >= 0 && gyp < N1;
            T vux = 0, vuy = 0, vuz = 0, vp = 0;
            if (in) {
                if (gxp < N1 - 1) vux = gx[gxp + size_t(N1 - 1) * (gyp + size_t(N1) * Z)];
                if (gyp < N1 - 1) vuy = gy[gxp + size_t(N1) * (gyp + size_t(N1 - 1) * Z)];
                if (Z < N1 - 1) vuz = gz[gxp + size_t(N1) * (gyp + size_t(N1) * Z)];
                vp = gp[gxp + size_t(N1) * (gyp + size_t(N1) * Z)];
            }
            v[0][t] = vux;
            v[1][t] = vuy;
            v[2][t] = vuz;
            v[3][t] = vp;
        }
    };
    T pf[4][NL];
    const int Zfirst = (L0 > 0 ? L0 - 1 : 0) * M;
    const int Zlast = (L1 < n ? L1 + 1 : n) * M - 1;
    if constexpr (PF) load_plane(Zfirst, pf);

    int buf = 0;
    for (int Lin = L0 - 1; Lin <= L1; ++Lin) {
        const bool have = (Lin >= 0) && (Lin < n);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T ix = 0, iy = 0, ip = 0, s = 0, vxo = 0, vyo = 0, uzo = 0, po = 0;
            if (have) {
                const int Z = Lin * M + c;
                T* su = &s_u[buf][0][0];
                // 1) plane Z of the four fields into LDS
                if constexpr (PF) {
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        const int i = tid + t * NT;
                        if (i < RS) {
#pragma unroll
                            for (int f = 0; f < 4; ++f) su[f * RS + i] = pf[f][t];
                        }
                    }
                    if (Z < Zlast) load_plane(Z + 1, pf);   // in flight during this plane's work
                } else {
                    T v[4][NL];
                    load_plane(Z, v);
#pragma unroll
                    for (int t = 0; t < NL; ++t) {
                        const int i = tid + t * NT;
                        if (i < RS) {
#pragma unroll
                            for (int f = 0; f < 4; ++f) su[f * RS + i] = v[f][t];
                        }
                    }
                }
                __syncthreads();
                const T* sux = su;
                const T* suy = su + RS;
                const T* suz = su + 2 * RS;
                const T* sp = su + 3 * RS;
                // 2) Mc along x for the rows the y stencil needs, Mc along y for the columns
                for (int i = tid; i < TX * RY; i += NT) {
                    const int qx = i % TX, ry = i / TX;
                    const int aa = qx % M;
                    const T* row = MC + aa * (2 * M + 1);
                    const T* src = sux + ry * RX + qx;        // region col qx + M - M
                    T acc = 0;
#pragma unroll
                    for (int o = 0; o < 2 * M + 1; ++o) acc += row[o] * src[o];
                    s_vx[i] = acc;
                }
                for (int i = tid; i < RX * TY; i += NT) {
                    const int rx = i % RX, qy = i / RX;
                    const int bb = qy % M;
                    const T* row = MC + bb * (2 * M + 1);
                    const T* src = suy + qy * RX + rx;        // region row qy + M - M
                    T acc = 0;
#pragma unroll
                    for (int o = 0; o < 2 * M + 1; ++o) acc += row[o] * src[o * RX];
                    s_vy[i] = acc;
                }
                __syncthreads();
                // 3) in-plane terms at this thread's position
                const int rx = tx + M, ry = ty + M;
                const T* rux = sux + ry * RX;               // row Y of ux
                T lcx = 0, dtx = 0, ldyvx = 0, lcy = 0, dty = 0, ldxvy = 0, ldxuz = 0, ldyuz = 0, dxux = 0, dyuy = 0;
#pragma unroll
                for (int o = 0; o < 2 * M + 1; ++o) {
                    lcx += LC[a * (2 * M + 1) + o] * rux[rx + o - M];
                    lcy += LC[b * (2 * M + 1) + o] * suy[(ry + o - M) * RX + rx];
                }
#pragma unroll
                for (int o = 0; o < 2 * M; ++o) {
                    dtx += DT[a * 2 * M + o] * sp[ry * RX + tx - a + M + o];
                    dty += DT[b * 2 * M + o] * sp[(ty - b + M + o) * RX + rx];
                }
#pragma unroll
                for (int o = 0; o < 3 * M; ++o) {
                    const T cy = LD[vyv * 3 * M * M + b * 3 * M + o];
                    const T cx = LD[vxv * 3 * M * M + a * 3 * M + o];
                    ldyvx += cy * s_vx[(ty - b + o) * TX + tx];
                    ldxvy += cx * s_vy[ty * RX + tx - a + o];
                    ldxuz += cx * suz[ry * RX + tx - a + o];
                    ldyuz += cy * suz[(ty - b + o) * RX + rx];
                }
#pragma unroll
                for (int j = 0; j < M + 1; ++j) {
                    dxux += DD[a * (M + 1) + j] * rux[tx - a + M + j - 1];
                    dyuy += DD[b * (M + 1) + j] * suy[(ty - b + M + j - 1) * RX + rx];
                }
                const T mdc = MD[c];
                ix = mdb * mdc * (lcx - dtx) + mdc * ldyvx;
                iy = mda * mdc * (lcy - dty) + mdc * ldxvy;
                s = mdb * ldxuz + mda * ldyuz;
                ip = -mdc * (mdb * dxux + mda * dyuy);
                vxo = s_vx[ry * TX + tx];
                vyo = s_vy[ty * RX + rx];
                uzo = suz[ry * RX + rx];
                po = sp[ry * RX + rx];
                buf ^= 1;
            }
            wvx[2 * M + c] = vxo;
            wvy[2 * M + c] = vyo;
            ws[2 * M + c] = s;
            wuz[2 * M + c] = uzo;
            wp[2 * M + c] = po;
            pix[1][c] = ix;
            piy[1][c] = iy;
            pip[1][c] = ip;
        }

        // 4) layer Lin-1 is complete: z stencils from the windows, write it
        const int L = Lin - 1;
        if (L >= L0) {
            const int vz = ld_variant(L, n);
            const T* LDz = LD + vz * 3 * M * M;
            const bool okxy = X < N1 && Y < N1;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int Z = L * M + c;
                T zx = 0, zy = 0, zp = 0, zms = 0, zlc = 0, zdt = 0;
#pragma unroll
                for (int o = 0; o < 3 * M; ++o) {
                    zx += LDz[c * 3 * M + o] * wvx[o];
                    zy += LDz[c * 3 * M + o] * wvy[o];
                }
#pragma unroll
                for (int j = 0; j < M + 1; ++j) zp += DD[c * (M + 1) + j] * wuz[M + j - 1];
#pragma unroll
                for (int o = 0; o < 2 * M + 1; ++o) {
                    zms += MC[c * (2 * M + 1) + o] * ws[c + o];
                    zlc += LC[c * (2 * M + 1) + o] * wuz[c + o];
                }
#pragma unroll
                for (int o = 0; o < 2 * M; ++o) zdt += DT[c * 2 * M + o] * wp[M + o];
                const T yx = pix[0][c] + mdb * zx;
                const T yy = piy[0][c] + mda * zy;
                const T yp = pip[0][c] - mda * mdb * zp;
                const T yz = zms + mda * mdb * (zlc - zdt);
                if (okxy) {
                    const size_t ox = X + size_t(N1 - 1) * (Y + size_t(N1) * Z);
                    const size_t oy = X + size_t(N1) * (Y + size_t(N1 - 1) * Z);
                    const size_t oz = X + size_t(N1) * (Y + size_t(N1) * Z);
                    if (X < N1 - 1) y[ox] = RESID ? bvec[ox] - yx : yx;
                    if (Y < N1 - 1) y[nc + oy] = RESID ? bvec[nc + oy] - yy : yy;
                    if (Z < N1 - 1) y[2 * nc + oz] = RESID ? bvec[2 * nc + oz] - yz : yz;
                    y[3 * nc + oz] = RESID ? bvec[3 * nc + oz] - yp : yp;
                }
            }
        }
        // 5) slide the windows by one layer
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) {
            wvx[i] = wvx[i + M];
            wvy[i] = wvy[i + M];
            ws[i] = ws[i + M];
            wuz[i] = wuz[i + M];
            wp[i] = wp[i + M];
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            pix[0][i] = pix[1][i];
            piy[0][i] = piy[1][i];
            pip[0][i] = pip[1][i];
        }
    }
}

}  // namespace smg
