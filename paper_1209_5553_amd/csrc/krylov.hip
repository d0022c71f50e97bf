// Arnoldi process on the device for the Krylov evaluation of phi1 (Sec. 4.1,
// Alg. alg:al2: modified Gram-Schmidt).  Every inner product is reduced in a
// fixed order by a one-workgroup kernel that writes the Hessenberg entry into
// device memory, where the next pass reads it: the host does not sync inside
// the process and reads H once at the end.
#include "device.h"
#include "krylov.h"

namespace erem {

namespace {

constexpr int kRedThreads = 1024;

__device__ inline int block_id() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }

__device__ inline double block_sum256(double v) {
  __shared__ double sh[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int t = threadIdx.x + threadIdx.y * kBX;
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  return t == 0 ? sh[0] + sh[1] + sh[2] + sh[3] : 0.0;
}

// partial sums of a . b
__global__ __launch_bounds__(kThreads) void k_dot(Dims d, const double* __restrict__ a, const double* __restrict__ b,
                                        double* __restrict__ part) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s = 0.0;
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    s = a[i] * b[i];
  }
  s = block_sum256(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = s;
}

// w = J v (stencil), partial sums of w . v1
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_spmv_dot(Dims d, const double* __restrict__ coef,
                                             const double* __restrict__ v, double* __restrict__ w,
                                             const double* __restrict__ v1, double* __restrict__ part) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s = 0.0;
  if (x < d.nx && y < d.ny) {
    const int N = d.N;
    const int i = x + d.nx * (y + d.ny * z);
    double jv = coef[i] * v[i];
    jv += coef[N + i] * v[x > 0 ? i - 1 : i];
    jv += coef[2 * N + i] * v[x + 1 < d.nx ? i + 1 : i];
    jv += coef[3 * N + i] * v[y > 0 ? i - d.nx : i];
    jv += coef[4 * N + i] * v[y + 1 < d.ny ? i + d.nx : i];
    if (DIM == 3) {
      const int pl = d.nx * d.ny;
      jv += coef[5 * N + i] * v[z > 0 ? i - pl : i];
      jv += coef[6 * N + i] * v[z + 1 < d.nz ? i + pl : i];
    }
    w[i] = jv;
    s = jv * v1[i];
  }
  s = block_sum256(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = s;
}

// w -= h v_i (h read from device memory), then partial sums of w . next
// (next = v_{i+1}, or w itself for the norm).
__global__ __launch_bounds__(kThreads) void k_axpy_dot(Dims d, double* w, const double* __restrict__ vi,
                                             const double* __restrict__ hptr, const double* next,
                                             double* __restrict__ part) {
  const double h = *hptr;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  double s = 0.0;
  if (x < d.nx && y < d.ny) {
    const int i = x + d.nx * (y + d.ny * z);
    const double wi = w[i] - h * vi[i];
    w[i] = wi;
    s = wi * (next == w ? wi : next[i]);
  }
  s = block_sum256(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[block_id()] = s;
}

// out = sum of the block partials (fixed order); sqrt_out: out = sqrt(sum)
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ part, int nb,
                                              double* __restrict__ out, int sqrt_out) {
  __shared__ double sh[kRedThreads / 64];
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) v += part[b];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kRedThreads / 64; ++k) s += sh[k];
    *out = sqrt_out ? sqrt(s) : s;
  }
}

// vout = w / h (zero if h == 0: happy breakdown, the host truncates there)
__global__ __launch_bounds__(kThreads) void k_scale(Dims d, const double* w, const double* __restrict__ hptr,
                                          double* vout) {
  const double h = *hptr;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  vout[i] = w[i] * inv;
}

// u = (first ? 0 : u) + sum_k c_k V_k  (c from device memory)
__global__ __launch_bounds__(kThreads) void k_combine(Dims d, const double* __restrict__ V, int nvec,
                                            const double* __restrict__ c, double* __restrict__ u, int first) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * z);
  const size_t N = d.N;
  double acc = first ? 0.0 : u[i];
  for (int k = 0; k < nvec; ++k) acc += c[k] * V[k * N + i];
  u[i] = acc;
}

}  // namespace

int kry_num_blocks(const Dims& d) {
  const dim3 g = cell_grid(d);
  return static_cast<int>(g.x * g.y * g.z);
}

// Arnoldi with modified Gram-Schmidt (Alg. alg:al2) on v (already in V[0],
// unnormalised): beta = ||v||, V[0] = v / beta, then for j = 0..m-1:
// w = J V[j]; h_ij = w . V[i], w -= h_ij V[i] (i = 0..j); h_{j+1,j} = ||w||;
// V[j+1] = w / h_{j+1,j}.  H (row-major (m+1) x m) and beta stay on the device.
hipError_t arnoldi_mgs(const Dims& d, const double* coef, double* V, double* w, double* H, double* beta,
                       double* part, int m, hipStream_t s) {
  const size_t N = d.N;
  const int nb = kry_num_blocks(d);
  const dim3 g = cell_grid(d), b = cell_block();
  hipLaunchKernelGGL(k_dot, g, b, 0, s, d, V, V, part);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, part, nb, beta, 1);
  hipLaunchKernelGGL(k_scale, g, b, 0, s, d, V, beta, V);
  for (int j = 0; j < m; ++j) {
    const double* vj = V + j * N;
    if (d.dim == 3)
      hipLaunchKernelGGL(k_spmv_dot<3>, g, b, 0, s, d, coef, vj, w, V, part);
    else
      hipLaunchKernelGGL(k_spmv_dot<2>, g, b, 0, s, d, coef, vj, w, V, part);
    for (int i = 0; i <= j; ++i) {
      double* hij = H + i * m + j;
      hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, part, nb, hij, 0);
      const double* next = (i < j) ? V + (i + 1) * N : w;
      hipLaunchKernelGGL(k_axpy_dot, g, b, 0, s, d, w, V + i * N, hij, next, part);
    }
    double* hnext = H + (j + 1) * m + j;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, part, nb, hnext, 1);
    hipLaunchKernelGGL(k_scale, g, b, 0, s, d, w, hnext, V + (j + 1) * N);
  }
  return hipGetLastError();
}

hipError_t krylov_combine(const Dims& d, const double* V, int nvec, const double* c, double* u, int first,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_combine, cell_grid(d), cell_block(), 0, s, d, V, nvec, c, u, first);
  return hipGetLastError();
}

}  // namespace erem
