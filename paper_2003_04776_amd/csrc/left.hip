// Left eigenvectors u of the Schur pencil, u^H (beta S - alpha T) = 0, by the right-
// eigenvector path on the flipped transposed pencil.  With J the exchange matrix,
// (S', T') = (J S^T J, J T^T J) is again a real Schur pencil (its 2 x 2 block at
// (m-2-p, m-1-p) comes from the block of S at (p, p+1)), and u^H (beta S - alpha T) = 0
// iff (beta S' - alpha T') (J conj(u)) = 0.  So u = conj(J z') with z' the right
// eigenvector of (S', T') for the same eigenvalue: the right solve's output Y' turned by
// 180 degrees (rows and columns reversed, the scales reversed), and for every complex pair
// (p, p+1) of S the two columns swapped with the imaginary part negated.  The robust
// bounds of the right solve on (S', T') are those of a left solve on (S, T): its
// infinity norms of tiles of S' are the 1-norms of tiles of S (the conclusion, Section 7,
// names left eigenvectors with the 1-norm in place of the infinity norm as the extension).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rgev {

constexpr int kFlipTile = 64;

// B = J A^T J (B[i][j] = A[m-1-j][m-1-i]), B column-major with leading dimension m; one
// 64 x 64 tile of B per workgroup through LDS, reads and writes along columns
__global__ __launch_bounds__(256) void left_flip_kernel(int64_t m, const double* __restrict__ A, int64_t lda,
                                                        double* __restrict__ B) {
  __shared__ double t[kFlipTile][kFlipTile + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kFlipTile, j0 = (int64_t)blockIdx.y * kFlipTile;
  const int tid = threadIdx.x;
  // element (a, b) of the tile: B[i0 + a][j0 + b] = A[m-1-j0-b][m-1-i0-a]
  for (int a = tid / kFlipTile; a < kFlipTile; a += 256 / kFlipTile) {
    const int b = tid % kFlipTile;
    const int64_t i = i0 + a, j = j0 + b;
    if (i < m && j < m) t[a][b] = A[(m - 1 - j) + (m - 1 - i) * lda];
  }
  __syncthreads();
  for (int b = tid / kFlipTile; b < kFlipTile; b += 256 / kFlipTile) {
    const int a = tid % kFlipTile;
    const int64_t i = i0 + a, j = j0 + b;
    if (i < m && j < m) B[i + j * m] = t[a][b];
  }
}

__global__ void left_select_kernel(int64_t m, const int32_t* __restrict__ sel, int32_t* __restrict__ out) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c < m) out[c] = sel[m - 1 - c];
}

// 180-degree turn of Y in place (element k of the first half swaps with element
// m^2 - 1 - k) and the scales reversed
__global__ void left_rotate_kernel(int64_t m, double* Y, int64_t ldy, int32_t* scales) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < m * m / 2) {
    const int64_t i = k % m, c = k / m;
    double* p = Y + i + c * ldy;
    double* q = Y + (m - 1 - i) + (m - 1 - c) * ldy;
    const double x = *p, y = *q;
    *p = y;
    *q = x;
  }
  if (scales && k < m / 2) {
    const int32_t x = scales[k], y = scales[m - 1 - k];
    scales[k] = y;
    scales[m - 1 - k] = x;
  }
}

// for a complex pair (c, c+1) of S (block (m-2-c, m-1-c) of S', blkp[m-1-c] == 2):
// column c <- column c+1 (the real part), column c+1 <- -column c (the imaginary part)
__global__ void left_pair_kernel(int64_t m, const int8_t* __restrict__ blkp, double* Y, int64_t ldy) {
  const int64_t c = blockIdx.x;
  if (c + 1 >= m || blkp[m - 1 - c] != 2) return;
  const int64_t i = blockIdx.y * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  double* x = Y + i + c * ldy;
  const double re = x[ldy], im = x[0];
  x[0] = re;
  x[ldy] = -im;
}

void launch_left_flip(int64_t m, const double* A, int64_t lda, double* B, hipStream_t s) {
  const unsigned n = (unsigned)((m + kFlipTile - 1) / kFlipTile);
  left_flip_kernel<<<dim3(n, n), 256, 0, s>>>(m, A, lda, B);
}

void launch_left_select(int64_t m, const int32_t* sel, int32_t* out, hipStream_t s) {
  left_select_kernel<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, sel, out);
}

void launch_left_finish(int64_t m, const int8_t* blkp, double* Y, int64_t ldy, int32_t* scales, hipStream_t s) {
  const int64_t half = m * m / 2 > m / 2 ? m * m / 2 : m / 2;
  if (half > 0) left_rotate_kernel<<<(unsigned)((half + 255) / 256), 256, 0, s>>>(m, Y, ldy, scales);
  left_pair_kernel<<<dim3((unsigned)m, (unsigned)((m + 255) / 256)), 256, 0, s>>>(m, blkp, Y, ldy);
}

}  // namespace rgev
