// Fused operator y = K x (or r = b - K x), 2.5D tile kernel with the work of
// every xy position split between two wave groups (Alg. 1 in the separable
// form of stencil_tables.hpp; same arithmetic as apply_kernel.hpp).
//
// Group A (the first NA threads, whole waves) owns y_x and y_y of its
// position: the in-plane rows Lc, D^T and Ld on Mc u, and the z stencil Ld_z
// on Mc_x u_x and Mc_y u_y from its register windows (or forward sums, ZP).
// Group B owns y_z and y_p: the in-plane Ld rows on u_z, the divergence rows
// D u, and the z stencils Mc_z, Lc_z, D^T_z, D_z; it also forms the shared
// Mc_x u_x plane (and the Mc_y u_y plane, unless group A forms it first: AVY)
// while group A evaluates its first in-plane terms.  Each group runs its own
// copy of the layer loop, so a thread keeps only its group's windows live
// (about half the registers of one thread per position), and a CU holds twice
// as many waves.  Both copies pass the same barriers in the same order.
//
// The kernel is bound by LDS issue, so the per-degree options (apply_launch.hpp)
// move work off LDS: the z rows are scalar loads, each group's in-plane rows
// sit in registers, LDS or the vector cache, and the two groups' LDS reads
// are evened out.
#pragma once

#include <hip/hip_runtime.h>

#include "apply_kernel.hpp"
#include "stencil_tables.hpp"

namespace smg {

template <int K, int CX, int CY, bool PAD = false>
struct SplitShape {
    static constexpr int M = K + 1;
    static constexpr int TX = CX * M, TY = CY * M;
    static constexpr int NP = TX * TY;                  // positions
    static constexpr int NA = (NP + 63) / 64 * 64;      // threads per group (whole waves)
    static constexpr int NT = 2 * NA;
    static constexpr int RX = TX + 2 * M, RY = TY + 2 * M;
    static constexpr int RS = RX * RY;
    static constexpr int NL = (RS + NT - 1) / NT;       // plane elements per thread and field
    // LDS row pitch of the planes and of Mc_y u_y; PAD: congruent to the tile
    // width modulo 16 elements, so the 16 lanes of one LDS cycle that straddle a
    // tile row end still hit distinct banks (pays only for FP64 at degree 2)
    static constexpr int PX = PAD ? RX + ((TX - RX) % 16 + 16) % 16 : RX;
    static constexpr int PS = PX * RY;
};

// GT: the group's in-plane stencil rows (which differ from lane to lane) are
// read from global memory through the vector cache instead of from LDS.  The
// z rows are the same for every lane of a plane and are always read from
// global memory, which makes them scalar loads.  Splitting the reads between
// the LDS and the vector-memory pipe by group balances the two (measured).
// HOLD: the group's rows that do not change along the plane loop are loaded
// once into registers (group A: Lc, D^T and Ld in x and y; group B: Ld and D
// in x and y).
// AVY: group A forms the Mc_y u_y plane (before its own first rows) and group
// B only the Mc_x u_x plane, which evens out their LDS reads.
// ZP: the z stencils are accumulated forward instead of evaluated from
// register windows: each plane adds its terms to the rows of the three cell
// layers it couples to (its own, the one below, the one above), and a layer's
// rows are written once the plane loop has passed the layer above it.  Three
// layers of accumulators per output field replace the windows of Mc u, u_z, p
// and the in-plane partials (about half the registers at high degree).
template <int K, typename T, int CX, int CY, bool RESID, int ROLE, bool GT, bool HOLD, bool AVY, bool PAD, bool ZP>
__device__ inline void split_loop(const T* __restrict__ x, const T* __restrict__ bvec, T* __restrict__ y,
                                  const T* __restrict__ s_tab, const T* __restrict__ g_tab,
                                  T (*s_u)[4][SplitShape<K, CX, CY, PAD>::PS], T* s_vx, T* s_vy, int n, int L0, int L1,
                                  int X0, int Y0) {
    using S = SplitShape<K, CX, CY, PAD>;
    constexpr int M = S::M, TX = S::TX, TY = S::TY, NP = S::NP, NA = S::NA, NT = S::NT, RX = S::RX, RY = S::RY,
                  RS = S::RS, NL = S::NL, PX = S::PX, PS = S::PS;
    using TB = Tab<K>;
    const int tid = threadIdx.x;
    const int p = tid - ROLE * NA;                 // position of this thread in its group
    const bool act = p < NP;
    const int tx = act ? p % TX : 0, ty = act ? p / TX : 0;
    const int X = X0 + tx, Y = Y0 + ty;
    const int a = tx % M, b = ty % M;
    const int N1 = n * M;
    const int vxv = ld_variant(X / M, n), vyv = ld_variant(Y / M, n);
    const size_t nc = size_t(N1 - 1) * N1 * N1;
    const T* __restrict__ gx = x;
    const T* __restrict__ gy = x + nc;
    const T* __restrict__ gz = x + 2 * nc;
    const T* __restrict__ gp = x + 3 * nc;
    const T mda = s_tab[TB::MDg + a], mdb = s_tab[TB::MDg + b];
    // The stencil rows are re-read where they are used: the table base goes
    // through an SGPR move the compiler cannot see through, so the rows are
    // not hoisted out of the layer loop into registers.
    auto tables = [&]() {
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        return (GT ? g_tab : s_tab) + z;
    };
    auto ztables = [&]() {
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        return g_tab + z;
    };
    constexpr int HW = HOLD ? 1 : 0;
    T hlca[HW * (2 * M + 1) + 1], hlcb[HW * (2 * M + 1) + 1], hdta[HW * 2 * M + 1], hdtb[HW * 2 * M + 1],
        hlda[HW * 3 * M + 1], hldb[HW * 3 * M + 1];
    if constexpr (HOLD && ROLE == 0) {
#pragma unroll
        for (int o = 0; o < 2 * M + 1; ++o) {
            hlca[o] = g_tab[TB::LC + a * (2 * M + 1) + o];
            hlcb[o] = g_tab[TB::LC + b * (2 * M + 1) + o];
        }
#pragma unroll
        for (int o = 0; o < 2 * M; ++o) {
            hdta[o] = g_tab[TB::DT + a * 2 * M + o];
            hdtb[o] = g_tab[TB::DT + b * 2 * M + o];
        }
    }
    if constexpr (HOLD) {
#pragma unroll
        for (int o = 0; o < 3 * M; ++o) {
            hlda[o] = g_tab[TB::LD + vxv * 3 * M * M + a * 3 * M + o];
            hldb[o] = g_tab[TB::LD + vyv * 3 * M * M + b * 3 * M + o];
        }
    }
    constexpr int HB = (HOLD && ROLE == 1) ? 1 : 0;
    T hdda[HB * (M + 1) + 1], hddb[HB * (M + 1) + 1];
    if constexpr (HB) {
#pragma unroll
        for (int j = 0; j < M + 1; ++j) {
            hdda[j] = g_tab[TB::DD + a * (M + 1) + j];
            hddb[j] = g_tab[TB::DD + b * (M + 1) + j];
        }
    }

    // plane Z of the four fields, tile + halo, zero outside the domain (all threads share the loads)
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

    // group A: windows of Mc_x u_x, Mc_y u_y and the in-plane partials of y_x, y_y;
    // group B: windows of the in-plane Ld u_z, of u_z and of p, and the partial of y_p
    constexpr int W = 3 * M;
    T w0[W], w1[W], w2[ROLE == 1 ? W : 1];
    T q0[2][M], q1[ROLE == 0 ? 2 : 1][M];
#pragma unroll
    for (int i = 0; i < W; ++i) w0[i] = w1[i] = T(0);
#pragma unroll
    for (int i = 0; i < (ROLE == 1 ? W : 1); ++i) w2[i] = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        q0[0][i] = q0[1][i] = T(0);
        q1[0][i] = T(0);
        q1[ROLE == 0 ? 1 : 0][i] = T(0);
    }

    // ZP accumulators: [0] layer Lin-1, [1] layer Lin, [2] layer Lin+1;
    // group A: y_x, y_y; group B: y_z, y_p
    T acc0[ZP ? 3 : 1][M], acc1[ZP ? 3 : 1][M];
#pragma unroll
    for (int l = 0; l < (ZP ? 3 : 1); ++l)
#pragma unroll
        for (int i = 0; i < M; ++i) acc0[l][i] = acc1[l][i] = T(0);

    T pf[4][NL];
    const int Zlast = (L1 < n ? L1 + 1 : n) * M - 1;
    load_plane((L0 > 0 ? L0 - 1 : 0) * M, pf);

    int buf = 0;
    for (int Lin = L0 - 1; Lin <= L1; ++Lin) {
        const bool have = (Lin >= 0) && (Lin < n);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            T r0 = 0, r1 = 0, r2 = 0, r3 = 0;
            if (have) {
                const int Z = Lin * M + c;
                T* su = &s_u[buf][0][0];
                // 1) the prefetched plane into LDS, the next plane's loads in flight
#pragma unroll
                for (int t = 0; t < NL; ++t) {
                    const int i = tid + t * NT;
                    if (i < RS) {
                        const int li = (i / RX) * PX + i % RX;
#pragma unroll
                        for (int f = 0; f < 4; ++f) su[f * PS + li] = pf[f][t];
                    }
                }
                if (Z < Zlast) load_plane(Z + 1, pf);
                __syncthreads();
                const T* sux = su;
                const T* suy = su + PS;
                const T* suz = su + 2 * PS;
                const T* sp = su + 3 * PS;
                const int rx = tx + M, ry = ty + M;
                const T* tb = tables();
                const T* __restrict__ MC = tb + TB::MC;
                const T* __restrict__ LC = tb + TB::LC;
                const T* __restrict__ DT = tb + TB::DT;
                const T* __restrict__ DD = tb + TB::DD;
                const T* __restrict__ LD = tb + TB::LD;
                const T mdc = tb[TB::MDg + c];
                T lcx = 0, dtx = 0, lcy = 0, dty = 0;
                if constexpr (ROLE == 1) {
                    // 2B) Mc along x for the rows the y stencil needs (and, unless group A does it,
                    // Mc along y for the columns the x stencil needs)
                    for (int i = p; i < TX * RY; i += NA) {
                        const int qx = i % TX, qy = i / TX;
                        const T* row = MC + (qx % M) * (2 * M + 1);
                        const T* src = sux + qy * PX + qx;
                        T acc = 0;
#pragma unroll
                        for (int o = 0; o < 2 * M + 1; ++o) acc += row[o] * src[o];
                        s_vx[i] = acc;
                    }
                }
                if constexpr (ROLE == (AVY ? 0 : 1)) {
                    for (int i = p; i < RX * TY; i += NA) {
                        const int qx = i % RX, qy = i / RX;
                        const T* row = MC + (qy % M) * (2 * M + 1);
                        const T* src = suy + qy * PX + qx;
                        T acc = 0;
#pragma unroll
                        for (int o = 0; o < 2 * M + 1; ++o) acc += row[o] * src[o * PX];
                        s_vy[qy * PX + qx] = acc;
                    }
                }
                if (ROLE == 0 && act) {
                    // 2A) the in-plane rows that need only the raw plane
                    const T* rux = sux + ry * PX;
#pragma unroll
                    for (int o = 0; o < 2 * M + 1; ++o) {
                        const T ca = HOLD ? hlca[o * HW] : LC[a * (2 * M + 1) + o];
                        const T cb = HOLD ? hlcb[o * HW] : LC[b * (2 * M + 1) + o];
                        lcx += ca * rux[rx + o - M];
                        lcy += cb * suy[(ry + o - M) * PX + rx];
                    }
#pragma unroll
                    for (int o = 0; o < 2 * M; ++o) {
                        const T ca = HOLD ? hdta[o * HW] : DT[a * 2 * M + o];
                        const T cb = HOLD ? hdtb[o * HW] : DT[b * 2 * M + o];
                        dtx += ca * sp[ry * PX + tx - a + M + o];
                        dty += cb * sp[(ty - b + M + o) * PX + rx];
                    }
                }
                __syncthreads();
                // 3) the remaining in-plane terms at this thread's position
                if (act) {
                    if constexpr (ROLE == 0) {
                        T ldyvx = 0, ldxvy = 0;
#pragma unroll
                        for (int o = 0; o < 3 * M; ++o) {
                            const T cb = HOLD ? hldb[o * HW] : LD[vyv * 3 * M * M + b * 3 * M + o];
                            const T ca = HOLD ? hlda[o * HW] : LD[vxv * 3 * M * M + a * 3 * M + o];
                            ldyvx += cb * s_vx[(ty - b + o) * TX + tx];
                            ldxvy += ca * s_vy[ty * PX + tx - a + o];
                        }
                        r0 = mdb * mdc * (lcx - dtx) + mdc * ldyvx;   // in-plane part of y_x
                        r1 = mda * mdc * (lcy - dty) + mdc * ldxvy;   // in-plane part of y_y
                        r2 = s_vx[ry * TX + tx];                      // Mc_x u_x at this position
                        r3 = s_vy[ty * PX + rx];                      // Mc_y u_y
                    } else {
                        T ldxuz = 0, ldyuz = 0, dxux = 0, dyuy = 0;
#pragma unroll
                        for (int o = 0; o < 3 * M; ++o) {
                            const T ca = HOLD ? hlda[o * HW] : LD[vxv * 3 * M * M + a * 3 * M + o];
                            const T cb = HOLD ? hldb[o * HW] : LD[vyv * 3 * M * M + b * 3 * M + o];
                            ldxuz += ca * suz[ry * PX + tx - a + o];
                            ldyuz += cb * suz[(ty - b + o) * PX + rx];
                        }
                        const T* rux = sux + ry * PX;
#pragma unroll
                        for (int j = 0; j < M + 1; ++j) {
                            const T ca = HB ? hdda[j * HB] : DD[a * (M + 1) + j];
                            const T cb = HB ? hddb[j * HB] : DD[b * (M + 1) + j];
                            dxux += ca * rux[tx - a + M + j - 1];
                            dyuy += cb * suy[(ty - b + M + j - 1) * PX + rx];
                        }
                        r0 = mdb * ldxuz + mda * ldyuz;                // in-plane Ld on u_z
                        r1 = suz[ry * PX + rx];                        // u_z
                        r2 = sp[ry * PX + rx];                         // p
                        r3 = -mdc * (mdb * dxux + mda * dyuy);         // in-plane part of y_p
                    }
                }
                buf ^= 1;
            }
            if constexpr (ZP) {
                if (have) {
                    // plane c of layer Lin into the rows of layers Lin-1+t, t = 0, 1, 2
                    const T* zt = ztables();
                    if constexpr (ROLE == 0) {
                        acc0[1][c] += r0;
                        acc1[1][c] += r1;
                        const T gxv = mdb * r2, gyv = mda * r3;
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
                            const T* LDt = zt + TB::LD + ld_variant(Lin - 1 + t, n) * 3 * M * M;
#pragma unroll
                            for (int cc = 0; cc < M; ++cc) {
                                const T co = LDt[cc * 3 * M + (2 - t) * M + c];
                                acc0[t][cc] += co * gxv;
                                acc1[t][cc] += co * gyv;
                            }
                        }
                    } else {
                        acc1[1][c] += r3;
                        const T mab = mda * mdb;
                        const T uzs = mab * r1, ps = mab * r2;
#pragma unroll
                        for (int t = 0; t < 3; ++t) {
#pragma unroll
                            for (int cc = 0; cc < M; ++cc) {
                                const int o = (2 - t) * M + c - cc;      // Mc_z, Lc_z column
                                if (o >= 0 && o <= 2 * M)
                                    acc0[t][cc] += zt[TB::MC + cc * (2 * M + 1) + o] * r0 +
                                                   zt[TB::LC + cc * (2 * M + 1) + o] * uzs;
                                const int od = (1 - t) * M + c;          // D^T_z column
                                if (od >= 0 && od < 2 * M) acc0[t][cc] -= zt[TB::DT + cc * 2 * M + od] * ps;
                                const int j = (1 - t) * M + c + 1;       // D_z column
                                if (j >= 0 && j <= M) acc1[t][cc] -= zt[TB::DD + cc * (M + 1) + j] * uzs;
                            }
                        }
                    }
                }
            } else if constexpr (ROLE == 0) {
                w0[2 * M + c] = r2;
                w1[2 * M + c] = r3;
                q0[1][c] = r0;
                q1[1][c] = r1;
            } else {
                w0[2 * M + c] = r0;
                w1[2 * M + c] = r1;
                w2[2 * M + c] = r2;
                q0[1][c] = r3;
            }
        }

        // 4) layer Lin-1 is complete: z stencils from the windows, write it
        const int L = Lin - 1;
        if (L >= L0) {
            const bool okxy = act && X < N1 && Y < N1;
            const T* tb = ztables();
            const T* __restrict__ MC = tb + TB::MC;
            const T* __restrict__ LC = tb + TB::LC;
            const T* __restrict__ DT = tb + TB::DT;
            const T* __restrict__ DD = tb + TB::DD;
            const T* __restrict__ LD = tb + TB::LD;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int Z = L * M + c;
                const size_t oz = X + size_t(N1) * (Y + size_t(N1) * Z);
                if constexpr (ZP) {
                    const T v0 = acc0[0][c], v1 = acc1[0][c];
                    if (okxy) {
                        if constexpr (ROLE == 0) {
                            const size_t ox = X + size_t(N1 - 1) * (Y + size_t(N1) * Z);
                            const size_t oy = X + size_t(N1) * (Y + size_t(N1 - 1) * Z);
                            if (X < N1 - 1) y[ox] = RESID ? bvec[ox] - v0 : v0;
                            if (Y < N1 - 1) y[nc + oy] = RESID ? bvec[nc + oy] - v1 : v1;
                        } else {
                            if (Z < N1 - 1) y[2 * nc + oz] = RESID ? bvec[2 * nc + oz] - v0 : v0;
                            y[3 * nc + oz] = RESID ? bvec[3 * nc + oz] - v1 : v1;
                        }
                    }
                } else if constexpr (ROLE == 0) {
                    const T* LDz = LD + ld_variant(L, n) * 3 * M * M;
                    T zx = 0, zy = 0;
#pragma unroll
                    for (int o = 0; o < 3 * M; ++o) {
                        zx += LDz[c * 3 * M + o] * w0[o];
                        zy += LDz[c * 3 * M + o] * w1[o];
                    }
                    const T yx = q0[0][c] + mdb * zx;
                    const T yy = q1[0][c] + mda * zy;
                    if (okxy) {
                        const size_t ox = X + size_t(N1 - 1) * (Y + size_t(N1) * Z);
                        const size_t oy = X + size_t(N1) * (Y + size_t(N1 - 1) * Z);
                        if (X < N1 - 1) y[ox] = RESID ? bvec[ox] - yx : yx;
                        if (Y < N1 - 1) y[nc + oy] = RESID ? bvec[nc + oy] - yy : yy;
                    }
                } else {
                    T zp = 0, zms = 0, zlc = 0, zdt = 0;
#pragma unroll
                    for (int j = 0; j < M + 1; ++j) zp += DD[c * (M + 1) + j] * w1[M + j - 1];
#pragma unroll
                    for (int o = 0; o < 2 * M + 1; ++o) {
                        zms += MC[c * (2 * M + 1) + o] * w0[c + o];
                        zlc += LC[c * (2 * M + 1) + o] * w1[c + o];
                    }
#pragma unroll
                    for (int o = 0; o < 2 * M; ++o) zdt += DT[c * 2 * M + o] * w2[M + o];
                    const T yp = q0[0][c] - mda * mdb * zp;
                    const T yz = zms + mda * mdb * (zlc - zdt);
                    if (okxy) {
                        if (Z < N1 - 1) y[2 * nc + oz] = RESID ? bvec[2 * nc + oz] - yz : yz;
                        y[3 * nc + oz] = RESID ? bvec[3 * nc + oz] - yp : yp;
                    }
                }
            }
        }
        // 5) slide the windows (accumulators) by one layer
        if constexpr (ZP) {
#pragma unroll
            for (int i = 0; i < M; ++i) {
                acc0[0][i] = acc0[1][i];
                acc0[1][i] = acc0[2][i];
                acc0[2][i] = T(0);
                acc1[0][i] = acc1[1][i];
                acc1[1][i] = acc1[2][i];
                acc1[2][i] = T(0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 2 * M; ++i) {
                w0[i] = w0[i + M];
                w1[i] = w1[i + M];
                if constexpr (ROLE == 1) w2[i] = w2[i + M];
            }
#pragma unroll
            for (int i = 0; i < M; ++i) {
                q0[0][i] = q0[1][i];
                if constexpr (ROLE == 0) q1[0][i] = q1[1][i];
            }
        }
    }
}

// FP32 at degrees 1 and 2: at least four waves per SIMD (two 8-wave
// workgroups per CU), so the rows held in registers do not cost occupancy
template <int K, typename T, int CX, int CY, bool RESID, bool GA, bool GB, bool HA, bool HB, bool AVY, bool PAD, bool ZP>
__global__ void __launch_bounds__((SplitShape<K, CX, CY, PAD>::NT), (sizeof(T) == 4 && K <= 2) ? 4 : 1)
stokes_apply_split_kernel(const T* __restrict__ x, const T* __restrict__ bvec, T* __restrict__ y,
                          const T* __restrict__ tab, int n, int cz, int tiles_x, int tiles_y) {
    using S = SplitShape<K, CX, CY, PAD>;
    using TB = Tab<K>;
    __shared__ T s_tab[TB::size];
    __shared__ T s_u[2][4][S::PS];        // ux, uy, uz, p planes (double buffered)
    __shared__ T s_vx[S::TX * S::RY];     // Mc_x ux over tile columns x all region rows
    __shared__ T s_vy[S::PX * S::TY];     // Mc_y uy over all region columns x tile rows
    for (int i = threadIdx.x; i < TB::size; i += S::NT) s_tab[i] = tab[i];
    const int lin = xcd_remap(blockIdx.x, gridDim.x);
    const int tile_x = lin % tiles_x;
    const int rest = lin / tiles_x;
    const int tile_y = rest % tiles_y;
    const int zc = rest / tiles_y;
    const int L0 = zc * cz;
    const int L1 = (L0 + cz < n) ? L0 + cz : n;
    const int X0 = tile_x * S::TX, Y0 = tile_y * S::TY;
    __syncthreads();
    // the groups are whole waves; each runs its copy of the layer loop (same barriers, same order)
    if (threadIdx.x < S::NA)
        split_loop<K, T, CX, CY, RESID, 0, GA, HA, AVY, PAD, ZP>(x, bvec, y, s_tab, tab, s_u, s_vx, s_vy, n, L0, L1, X0, Y0);
    else
        split_loop<K, T, CX, CY, RESID, 1, GB, HB, AVY, PAD, ZP>(x, bvec, y, s_tab, tab, s_u, s_vx, s_vy, n, L0, L1, X0, Y0);
}

}  // namespace smg
