// Multigrid and Krylov vector kernels (gfx950): tensor-product transfers,
// the coarse pseudo-inverse GEMV, precision conversion, multi-dot and
// multi-axpy for the Arnoldi process, pressure-mean normalization.
#include "mg_kernels.hpp"

namespace smg {

namespace {

constexpr int NT = 256;

// level geometry for the layout [u_x | u_y | u_z | p]
struct Geo {
    int N1;
    size_t nc;
    __device__ void decode(size_t i, int& comp, int& X, int& Y, int& Z) const {
        const size_t np = size_t(N1) * N1 * N1;
        (void)np;
        if (i < 3 * nc) {
            comp = int(i / nc);
            size_t e = i - size_t(comp) * nc;
            const int ex = comp == 0 ? N1 - 1 : N1, ey = comp == 1 ? N1 - 1 : N1;
            X = int(e % ex);
            e /= ex;
            Y = int(e % ey);
            Z = int(e / ey);
        } else {
            comp = 3;
            size_t e = i - 3 * nc;
            X = int(e % N1);
            e /= N1;
            Y = int(e % N1);
            Z = int(e / N1);
        }
    }
    __device__ size_t encode(int comp, int X, int Y, int Z) const {
        if (comp == 3) return 3 * nc + X + size_t(N1) * (Y + size_t(N1) * Z);
        const int ex = comp == 0 ? N1 - 1 : N1, ey = comp == 1 ? N1 - 1 : N1;
        return size_t(comp) * nc + X + size_t(ex) * (Y + size_t(ey) * Z);
    }
};

// out[i] (+)= sum over the tensor product of three 1D row lists of in[...]
// dg / cn: row lists of the DG and continuous directions (idx, weight), widths wd / wc
template <typename T, bool ACC>
__global__ void __launch_bounds__(NT)
tensor_transfer(const T* __restrict__ in, T* __restrict__ out, Geo go, Geo gi, const int* __restrict__ dgi,
                const double* __restrict__ dgw, int wd, const int* __restrict__ cni, const double* __restrict__ cnw,
                int wc, size_t total) {
    const size_t i = size_t(blockIdx.x) * NT + threadIdx.x;
    if (i >= total) return;
    int comp, X, Y, Z;
    go.decode(i, comp, X, Y, Z);
    const int P[3] = {X, Y, Z};
    const int* li[3];
    const double* lw[3];
    int wdt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool cont = d == comp;
        li[d] = cont ? cni + size_t(P[d]) * wc : dgi + size_t(P[d]) * wd;
        lw[d] = cont ? cnw + size_t(P[d]) * wc : dgw + size_t(P[d]) * wd;
        wdt[d] = cont ? wc : wd;
    }
    double acc = 0.0;
    for (int c = 0; c < wdt[2]; ++c) {
        const int iz = li[2][c];
        if (iz < 0) continue;
        const double wz = lw[2][c];
        for (int b = 0; b < wdt[1]; ++b) {
            const int iy = li[1][b];
            if (iy < 0) continue;
            const double wzy = wz * lw[1][b];
            for (int a = 0; a < wdt[0]; ++a) {
                const int ix = li[0][a];
                if (ix < 0) continue;
                acc += wzy * lw[0][a] * double(in[gi.encode(comp, ix, iy, iz)]);
            }
        }
    }
    if (ACC)
        out[i] += T(acc);
    else
        out[i] = T(acc);
}

// x = K0^+ b with the FP64 matrix (row-major n x n); vectors in T
template <typename T>
__global__ void __launch_bounds__(NT) coarse_gemv(const double* __restrict__ A, const T* __restrict__ b, T* __restrict__ x,
                                                   int n) {
    const int row = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += NT) s += A[size_t(row) * n + j] * double(b[j]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double red[NT / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[w];
        x[row] = T(t);
    }
}

template <typename S, typename D>
__global__ void __launch_bounds__(NT) convert(const S* __restrict__ a, D* __restrict__ b, size_t n) {
    const size_t i = size_t(blockIdx.x) * NT + threadIdx.x;
    if (i < n) b[i] = D(a[i]);
}

template <typename T>
__global__ void __launch_bounds__(NT) fill(T* __restrict__ a, T v, size_t n) {
    const size_t i = size_t(blockIdx.x) * NT + threadIdx.x;
    if (i < n) a[i] = v;
}

// partial[block][j] = sum over this block's range of V_j . w, j < nv
__global__ void __launch_bounds__(NT) multidot_partial(const double* __restrict__ V, size_t ld, const double* __restrict__ w,
                                                       int nv, size_t n, double* __restrict__ partial) {
    __shared__ double red[NT / 64];
    const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const size_t lo = size_t(blockIdx.x) * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (int j = 0; j < nv; ++j) {
        const double* v = V + size_t(j) * ld;
        double s = 0.0;
        for (size_t i = lo + threadIdx.x; i < hi; i += NT) s += v[i] * w[i];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int q = 0; q < NT / 64; ++q) t += red[q];
            partial[size_t(blockIdx.x) * nv + j] = t;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(NT) multidot_final(const double* __restrict__ partial, int nblocks, int nv,
                                                     double* __restrict__ out) {
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NT) s += partial[size_t(b) * nv + j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double red[NT / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < NT / 64; ++q) t += red[q];
        out[j] = t;
    }
}

// w = alpha w + sum_j c_j V_j (coefficients on the device)
__global__ void __launch_bounds__(NT) multiaxpy(const double* __restrict__ V, size_t ld, const double* __restrict__ c, int nv,
                                                double csign, double alpha, double* __restrict__ w, size_t n) {
    const size_t i = size_t(blockIdx.x) * NT + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += c[j] * V[size_t(j) * ld + i];
    w[i] = alpha * w[i] + csign * s;
}

// pressure integral mean: sum_i p_i h^3 w_a w_b w_c with the DG weights of the index
template <typename T>
__global__ void __launch_bounds__(NT) pressure_moment(const T* __restrict__ p, int N1, int m, const double* __restrict__ wg,
                                                      double h3, double* __restrict__ partial) {
    const size_t np = size_t(N1) * N1 * N1;
    double s = 0.0;
    for (size_t i = size_t(blockIdx.x) * NT + threadIdx.x; i < np; i += size_t(gridDim.x) * NT) {
        const int X = int(i % N1), Y = int((i / N1) % N1), Z = int(i / (size_t(N1) * N1));
        s += double(p[i]) * wg[X % m] * wg[Y % m] * wg[Z % m];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double red[NT / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < NT / 64; ++q) t += red[q];
        partial[blockIdx.x] = t * h3;
    }
}

template <typename T>
__global__ void __launch_bounds__(NT) shift_pressure(T* __restrict__ p, const double* __restrict__ mean, size_t np) {
    const size_t i = size_t(blockIdx.x) * NT + threadIdx.x;
    if (i < np) p[i] = T(double(p[i]) - *mean);
}

unsigned blocks_for(size_t n) { return unsigned((n + NT - 1) / NT); }

}  // namespace

hipError_t launch_transfer(bool f64, bool acc, const void* in, void* out, int N1_out, int N1_in, const int* dgi,
                           const double* dgw, int wd, const int* cni, const double* cnw, int wc, hipStream_t st) {
    Geo go{N1_out, size_t(N1_out - 1) * N1_out * N1_out};
    Geo gi{N1_in, size_t(N1_in - 1) * N1_in * N1_in};
    const size_t total = 3 * go.nc + size_t(N1_out) * N1_out * N1_out;
    const unsigned g = blocks_for(total);
    if (f64) {
        if (acc)
            hipLaunchKernelGGL((tensor_transfer<double, true>), dim3(g), dim3(NT), 0, st, static_cast<const double*>(in),
                               static_cast<double*>(out), go, gi, dgi, dgw, wd, cni, cnw, wc, total);
        else
            hipLaunchKernelGGL((tensor_transfer<double, false>), dim3(g), dim3(NT), 0, st, static_cast<const double*>(in),
                               static_cast<double*>(out), go, gi, dgi, dgw, wd, cni, cnw, wc, total);
    } else {
        if (acc)
            hipLaunchKernelGGL((tensor_transfer<float, true>), dim3(g), dim3(NT), 0, st, static_cast<const float*>(in),
                               static_cast<float*>(out), go, gi, dgi, dgw, wd, cni, cnw, wc, total);
        else
            hipLaunchKernelGGL((tensor_transfer<float, false>), dim3(g), dim3(NT), 0, st, static_cast<const float*>(in),
                               static_cast<float*>(out), go, gi, dgi, dgw, wd, cni, cnw, wc, total);
    }
    return hipGetLastError();
}

hipError_t launch_coarse_gemv(bool f64, const double* A, const void* b, void* x, int n, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL((coarse_gemv<double>), dim3(n), dim3(NT), 0, st, A, static_cast<const double*>(b),
                           static_cast<double*>(x), n);
    else
        hipLaunchKernelGGL((coarse_gemv<float>), dim3(n), dim3(NT), 0, st, A, static_cast<const float*>(b),
                           static_cast<float*>(x), n);
    return hipGetLastError();
}

hipError_t launch_convert(bool from_f64, const void* a, void* b, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (from_f64)
        hipLaunchKernelGGL((convert<double, float>), dim3(blocks_for(n)), dim3(NT), 0, st, static_cast<const double*>(a),
                           static_cast<float*>(b), n);
    else
        hipLaunchKernelGGL((convert<float, double>), dim3(blocks_for(n)), dim3(NT), 0, st, static_cast<const float*>(a),
                           static_cast<double*>(b), n);
    return hipGetLastError();
}

hipError_t launch_zero(bool f64, void* a, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL((fill<double>), dim3(blocks_for(n)), dim3(NT), 0, st, static_cast<double*>(a), 0.0, n);
    else
        hipLaunchKernelGGL((fill<float>), dim3(blocks_for(n)), dim3(NT), 0, st, static_cast<float*>(a), 0.0f, n);
    return hipGetLastError();
}

hipError_t launch_multidot(const double* V, size_t ld, const double* w, int nv, size_t n, double* partial, int nblocks,
                           double* out, hipStream_t st) {
    hipLaunchKernelGGL(multidot_partial, dim3(nblocks), dim3(NT), 0, st, V, ld, w, nv, n, partial);
    hipLaunchKernelGGL(multidot_final, dim3(nv), dim3(NT), 0, st, partial, nblocks, nv, out);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(const double* V, size_t ld, const double* c, int nv, double csign, double alpha, double* w,
                            size_t n, hipStream_t st) {
    hipLaunchKernelGGL(multiaxpy, dim3(blocks_for(n)), dim3(NT), 0, st, V, ld, c, nv, csign, alpha, w, n);
    return hipGetLastError();
}

hipError_t launch_normalize_pressure(bool f64, void* x, int N1, int m, const double* wg, double h, double* scratch,
                                     hipStream_t st) {
    const size_t nc = size_t(N1 - 1) * N1 * N1, np = size_t(N1) * N1 * N1;
    // scratch: [0] the mean, [1 .. g] per-block partial moments (fixed-order sum: deterministic)
    const unsigned g = unsigned(std::min<size_t>(kMomentBlocks, blocks_for(np)));
    if (f64) {
        double* p = static_cast<double*>(x) + 3 * nc;
        hipLaunchKernelGGL((pressure_moment<double>), dim3(g), dim3(NT), 0, st, p, N1, m, wg, h * h * h, scratch + 1);
        hipLaunchKernelGGL(multidot_final, dim3(1), dim3(NT), 0, st, scratch + 1, int(g), 1, scratch);
        hipLaunchKernelGGL((shift_pressure<double>), dim3(blocks_for(np)), dim3(NT), 0, st, p, scratch, np);
    } else {
        float* p = static_cast<float*>(x) + 3 * nc;
        hipLaunchKernelGGL((pressure_moment<float>), dim3(g), dim3(NT), 0, st, p, N1, m, wg, h * h * h, scratch + 1);
        hipLaunchKernelGGL(multidot_final, dim3(1), dim3(NT), 0, st, scratch + 1, int(g), 1, scratch);
        hipLaunchKernelGGL((shift_pressure<float>), dim3(blocks_for(np)), dim3(NT), 0, st, p, scratch, np);
    }
    return hipGetLastError();
}

}  // namespace smg
