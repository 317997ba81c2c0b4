// Kernels of the per-patch MLP local solver (launchers; asynchronous on `st`).
//
// Network x -> GELU(x W1 + b1) -> GELU(. W2 + b2) -> . W3 + b3, weights
// row-major [in x out], activations row-major [rows x features], FP32 in
// memory.  Products run on the matrix cores with FP32 accumulation; the
// operands are rounded to BF16 (production) or kept in FP32 (checks).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace smg {

enum class Epi : int {
    Store = 0,      // C = acc
    Bias = 1,       // C = acc + bias[col]
    BiasGelu = 2,   // Z = acc + bias[col] (if Z != null), C = gelu(acc + bias[col])
    GeluGrad = 3,   // C = acc * gelu'(Z[row][col])
};

// C[M x N] = op(A) op(B) with the epilogue `epi`.
//   A: ta = false -> element (m, k) at A[row(m) lda + k] with row(m) = arows ? arows[m] : m;
//      ta = true  -> element (m, k) at A[k lda + m]
//   B: tb = false -> element (k, n) at B[k ldb + n];  tb = true -> B[n ldb + k]
//   arows (optional) maps A's storage rows: row m (ta = false) or row k (ta = true)
// lda, ldb, ldc, ldz multiples of 4 and every pointer 16-byte aligned
// (checked by the caller).  bf16: operands rounded to BF16 on the way to LDS.
// Epi::Store with few output tiles and a long K splits K over partial tiles
// in split_ws (split_ws_floats floats; the split is skipped if too small).
hipError_t launch_gemm(bool bf16, Epi epi, bool ta, bool tb, int M, int N, int K, const float* A, int lda,
                       const int* arows, const float* B, int ldb, float* C, int ldc, const float* bias, float* Z,
                       int ldz, float* split_ws, size_t split_ws_floats, hipStream_t st);

// dY = 2 (Y - T[trows]) / (rows cols); partial[b] = block b's sum of squares
// (nblocks = kLossBlocks), loss_out = mean of squares (second stage).
constexpr int kLossBlocks = 512;
hipError_t launch_mse_grad(const float* Y, const float* T, const int* trows, int rows, int cols, float* dY,
                           double* partial, float* loss_out, hipStream_t st);

// out[n] = sum_m G[m ldg + n] for m < rows (two stages through `partial`,
// kColsumSplit x cols floats).
constexpr int kColsumSplit = 32;
hipError_t launch_colsum(const float* G, int ldg, int rows, int cols, float* partial, float* out, hipStream_t st);

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr mhat / (sqrt(vhat) + eps) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
hipError_t launch_adam(float* p, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);

// The vertex patches of one colour in groups, one patch type per group: group
// g holds the vertices (first[g][0] + 2 a, first[g][1] + 2 b, first[g][2] + 2 c),
// a < cnt[g][0], b < cnt[g][1], c < cnt[g][2], in lexicographic order (a
// fastest), as rows start[g] .. start[g] + count - 1 of a row space; mat[g] is
// the type index t_0 + 3 t_1 + 9 t_2 (t_d = 1: vertex 1, 2: vertex n - 1,
// 0: neither; 27: the single patch of n = 2).  all_types = false: the interior
// patches only, one group from row 0 (rows p0 .. of the interior launchers).
// all_types = true: every patch of the colour, each group padded to a
// multiple of kGroupAlign rows (padding rows belong to no patch).
constexpr int kMaxGroups = 27;
constexpr int kGroupAlign = 128;
struct PatchGroups {
    int ng;
    int start[kMaxGroups + 1];
    int first[kMaxGroups][3];
    int cnt[kMaxGroups][3];
    int mat[kMaxGroups];
};
PatchGroups colour_groups(int n, int colour, bool all_types);

// The Direct solver on every patch of one colour (colour_groups with
// all_types), in one launch: x[R_j] += M_type (R_j r scaled by 1/h (velocity)
// and 1/h^2 (pressure)), the output's pressure rows scaled by 1/h, for each
// patch j.  Bt holds per type the map M padded with zeros to dn x dk
// (direct_dims), row-major [out][in], BF16 (bf16) or FP32, types dn dk
// elements apart; every pointer 16-byte aligned.  Products on the matrix
// cores with FP32 accumulation.  r and x: level vectors (double if f64, else
// float), distinct.
void direct_dims(int d, int* dk, int* dn);
hipError_t launch_direct_patch(bool f64, bool bf16, const void* r, void* x, int n, int k, const PatchGroups& pg,
                               const void* Bt, hipStream_t st);

// Interior patches p0 .. p0+np-1 of one colour: patch-local vectors of a
// level vector (row q of X / Y / T belongs to patch p0 + q).
//   gather:  X[q] = (R_j r scaled by 1/h (velocity) and 1/h^2 (pressure)) / s_q,
//            s_q = its Euclidean norm (X[q] = 0 and s_q = 0 for a zero residual)
//   scatter: x[R_j] += omega s_q (Y[q] velocity rows, (Y[q] pressure rows - their mean) / h)
//   gather_diff (pair capture): T[q] = (x_new - x_old)[R_j] scaled to (U, h P) / s_q
// Patches of a colour are its interior vertices in lexicographic order (x
// fastest).  The level vectors are double (f64) or float.
hipError_t launch_patch_gather(bool f64, const void* r, int n, int k, int colour, int p0, int np, float* X, int ldx,
                               float* s, hipStream_t st);
hipError_t launch_patch_scatter(bool f64, void* x, int n, int k, int colour, int p0, int np, const float* Y, int ldy,
                                const float* s, double omega, hipStream_t st);
hipError_t launch_patch_gather_diff(bool f64, const void* xnew, const void* xold, int n, int k, int colour, int p0,
                                    int np, float* T, int ldt, const float* s, hipStream_t st);

// rows[i] = pi(start + i) for a keyed pseudo-random permutation pi of [0, n)
// (balanced Feistel bijection of the next even power of two, cycle-walked).
hipError_t launch_batch_rows(int* rows, int64_t start, int count, int64_t n, uint64_t key, hipStream_t st);

// x += c (n entries, double or float)
hipError_t launch_add(bool f64, void* x, const void* c, size_t n, hipStream_t st);

// *acc += *v (one device scalar into a double accumulator)
hipError_t launch_accumulate(const float* v, double* acc, hipStream_t st);

// interior vertices of colour c on an n^3 mesh (2 <= v_d <= n-2, v_d = c_d mod 2)
inline int interior_count_1d(int n, int parity) {
    int c = 0;
    for (int v = 2; v <= n - 2; ++v) c += (v & 1) == parity;
    return c;
}
inline int64_t interior_count(int n, int colour) {
    return int64_t(interior_count_1d(n, colour & 1)) * interior_count_1d(n, (colour >> 1) & 1) *
           interior_count_1d(n, (colour >> 2) & 1);
}

}  // namespace smg
