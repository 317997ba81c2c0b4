// Multigrid and Krylov vector kernels (gfx950): tensor-product transfers,
// the coarse pseudo-inverse GEMV, precision conversion, multi-dot and
// multi-axpy for the Arnoldi process, pressure-mean normalization.
#include "mg_kernels.hpp"

namespace smg {

namespace {

constexpr int NT = 256;

// One 1D pass of a tensor-product transfer: for every component c, along
// `axis`, out_c(..., P, ...) (+)= sum_a w[P][a] in_c(..., idx[P][a], ...), with
// the continuous-direction lists when axis == c and the DG lists otherwise.
// Arrays [Z][Y][X] per component, X fastest, components one after another.
struct Pass {
    int ein[4][3], eout[4][3];
    size_t oin[4], oout[4];
    int axis;
    const int* li[2];       // [0]: DG lists, [1]: continuous lists (idx; -1 = unused)
    const double* lw[2];
    int w[2];
};

constexpr int PX = 128, PY = 2;

// block (PX, PY): rows Y = blockIdx.x PY + threadIdx.y, plane Z = blockIdx.y, component blockIdx.z
template <typename T, bool ACC>
__global__ void __launch_bounds__(PX * PY) transfer_pass(const T* __restrict__ in, T* __restrict__ out, Pass p) {
    const int c = blockIdx.z;
    const int ex = p.eout[c][0], ey = p.eout[c][1], ez = p.eout[c][2];
    const int Y = blockIdx.x * PY + threadIdx.y, Z = blockIdx.y;
    if (Y >= ey || Z >= ez) return;
    const int kind = p.axis == c ? 1 : 0;
    const int* __restrict__ li = p.li[kind];
    const double* __restrict__ lw = p.lw[kind];
    const int w = p.w[kind];
    const int ix = p.ein[c][0], iy = p.ein[c][1];
    const T* src = in + p.oin[c];
    T* dst = out + p.oout[c] + size_t(ex) * (Y + size_t(ey) * Z);
    for (int X = threadIdx.x; X < ex; X += PX) {
        const int P = p.axis == 0 ? X : (p.axis == 1 ? Y : Z);
        double acc = 0.0;
        for (int a = 0; a < w; ++a) {
            const int j = li[P * w + a];
            if (j < 0) continue;
            const int xi = p.axis == 0 ? j : X, yi = p.axis == 1 ? j : Y, zi = p.axis == 2 ? j : Z;
            acc += lw[P * w + a] * double(src[xi + size_t(ix) * (yi + size_t(iy) * zi)]);
        }
        if (ACC)
            dst[X] += T(acc);
        else
            dst[X] = T(acc);
    }
}

template <typename T>
hipError_t run_pass(const void* in, void* out, const Pass& p, bool acc, hipStream_t st) {
    int my = 0, mz = 0;
    for (int c = 0; c < 4; ++c) {
        my = my > p.eout[c][1] ? my : p.eout[c][1];
        mz = mz > p.eout[c][2] ? mz : p.eout[c][2];
    }
    const dim3 grid((my + PY - 1) / PY, mz, 4), block(PX, PY);
    if (acc)
        hipLaunchKernelGGL((transfer_pass<T, true>), grid, block, 0, st, static_cast<const T*>(in), static_cast<T*>(out),
                           p);
    else
        hipLaunchKernelGGL((transfer_pass<T, false>), grid, block, 0, st, static_cast<const T*>(in),
                           static_cast<T*>(out), p);
    return hipGetLastError();
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
                           const double* dgw, int wd, const int* cni, const double* cnw, int wc, void* tmp,
                           hipStream_t st) {
    // extents per component along x, y, z: N1 - 1 in the component's own (continuous) direction, else N1
    auto ext = [](int N1, int c, int d) { return c == d ? N1 - 1 : N1; };
    int cur[4][3];
    for (int c = 0; c < 4; ++c)
        for (int d = 0; d < 3; ++d) cur[c][d] = ext(N1_in, c, d);
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    char* bufs[2] = {static_cast<char*>(tmp), nullptr};
    const void* src = in;
    for (int axis = 0; axis < 3; ++axis) {
        Pass p{};
        p.axis = axis;
        p.li[0] = dgi;
        p.lw[0] = dgw;
        p.w[0] = wd;
        p.li[1] = cni;
        p.lw[1] = cnw;
        p.w[1] = wc;
        size_t oi = 0, oo = 0;
        for (int c = 0; c < 4; ++c) {
            for (int d = 0; d < 3; ++d) {
                p.ein[c][d] = cur[c][d];
                p.eout[c][d] = d == axis ? ext(N1_out, c, d) : cur[c][d];
            }
            p.oin[c] = oi;
            p.oout[c] = oo;
            oi += size_t(p.ein[c][0]) * p.ein[c][1] * p.ein[c][2];
            oo += size_t(p.eout[c][0]) * p.eout[c][1] * p.eout[c][2];
        }
        // passes 0 and 1 write the temporaries (the second right after the first), pass 2 the output
        void* dst = out;
        if (axis < 2) {
            if (axis == 1) bufs[1] = bufs[0] + (oi * esz + 255) / 256 * 256;
            dst = bufs[axis];
        }
        const hipError_t e = f64 ? run_pass<double>(src, dst, p, axis == 2 && acc, st)
                                 : run_pass<float>(src, dst, p, axis == 2 && acc, st);
        if (e != hipSuccess) return e;
        for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 3; ++d) cur[c][d] = p.eout[c][d];
        src = dst;
    }
    return hipSuccess;
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
