// Arnoldi process on the device for the Krylov evaluation of phi1 (Sec. 4.1,
// Alg. alg:al2).  Each new column is orthogonalised against the basis by
// classical Gram-Schmidt applied twice (CGS2) rather than by the algorithm's
// modified Gram-Schmidt: both give the same Hessenberg matrix in exact
// arithmetic, and the second pass keeps the computed basis orthogonal to
// working precision, while each projection becomes one pass over the basis
// with all its inner products at once.  Column j therefore costs three
// streaming passes and three reductions whatever j is:
//   1. w = J v_j, with the partial sums of v_i . w (i <= j);
//   2. w -= sum_i g_i v_i, with the partial sums of v_i . w again;
//   3. w -= sum_i g'_i v_i, with the partial sum of w . w;
// each followed by a one-launch reduction of its partials in a fixed order
// (wave_part_sum) that writes the Hessenberg entries h_ij = g_i + g'_i and
// h_{j+1,j} = ||w|| into device memory.  v_{j+1} = w / h_{j+1,j} is formed
// inside pass 1 of the next column, which reads w and the norm.  The host
// does not sync inside the process and reads H once at the end.
#include "device.h"
#include "krylov.h"

namespace erem {

namespace {

constexpr int kRedThreads = 64;  // one wavefront per reduced value

__device__ inline int band_id() { return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z); }

// Block sum of one value per thread; thread 0 gets the result.
__device__ inline double block_sum256(double v) {
  __shared__ double sh[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int t = threadIdx.x + threadIdx.y * kBX;
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  return t == 0 ? sh[0] + sh[1] + sh[2] + sh[3] : 0.0;
}

// Wavefront sum of v into sh[i * waves + wave] (lane 0 writes).
__device__ inline void wave_store(double v, double* sh, int i) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if (threadIdx.x == 0) sh[i * kBY + threadIdx.y] = v;
}

// wave_store of V_k[i] * a for k < n; the loads go eight at a time ahead of
// the (convergent) shuffle trees.
__device__ inline void wave_dots(const double* __restrict__ V, size_t N, int i, bool in, double a, int n,
                                 double* sh) {
  constexpr int kBatch = 8;
  for (int k0 = 0; k0 < n; k0 += kBatch) {
    double t[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) t[u] = in && k0 + u < n ? V[(k0 + u) * N + i] * a : 0.0;
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (k0 + u < n) wave_store(t[u], sh, k0 + u);
  }
}

// After wave_store of n values: thread t < n writes the block's partial of
// value t to part[t * nb + band], adding the wavefronts in order.
__device__ inline void block_flush(const double* sh, int n, double* __restrict__ part, int nb) {
  __syncthreads();
  const int t = threadIdx.x + threadIdx.y * kBX;
  for (int i = t; i < n; i += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBY; ++w) s += sh[i * kBY + w];
    part[static_cast<size_t>(i) * nb + band_id()] = s;
  }
}

// partial sums of a . a
__global__ __launch_bounds__(kThreads) void k_norm_part(Dims d, const double* __restrict__ a,
                                                        double* __restrict__ part) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  double s = 0.0;
  if (x < d.nx && y < d.ny) {
    const double v = a[x + d.nx * (y + d.ny * static_cast<int>(blockIdx.z))];
    s = v * v;
  }
  s = block_sum256(s);
  if (threadIdx.x == 0 && threadIdx.y == 0) part[band_id()] = s;
}

// Pass 1 of column j: v_j = src / *nrm is written to vj, w = J v_j (stencil,
// neighbours of v_j read from src and scaled), and the partials of
// v_i . w for i = 0..j (V holds v_0..v_{j-1}; v_j comes from registers).
// src and w are different buffers: the neighbour reads of src must not see
// this pass's stores.
template <int DIM>
__global__ __launch_bounds__(kThreads) void k_kry_spmv(Dims d, const double* __restrict__ coef,
                                                       const double* __restrict__ src,
                                                       const double* __restrict__ nrm, double* __restrict__ vj,
                                                       double* __restrict__ w, const double* __restrict__ V, int j,
                                                       double* __restrict__ part, int nb) {
  __shared__ double sh[(kMaxKrylov + 1) * kBY];
  const double h = *nrm;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;  // zero: happy breakdown, the host truncates there
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int z = blockIdx.z;
  const bool in = x < d.nx && y < d.ny;
  const int N = d.N;
  const int i = in ? x + d.nx * (y + d.ny * z) : 0;
  double vc = 0.0, jv = 0.0;
  if (in) {
    vc = src[i] * inv;
    jv = coef[i] * vc;
    jv += coef[N + i] * (src[x > 0 ? i - 1 : i] * inv);
    jv += coef[2 * N + i] * (src[x + 1 < d.nx ? i + 1 : i] * inv);
    jv += coef[3 * N + i] * (src[y > 0 ? i - d.nx : i] * inv);
    jv += coef[4 * N + i] * (src[y + 1 < d.ny ? i + d.nx : i] * inv);
    if (DIM == 3) {
      const int pl = d.nx * d.ny;
      jv += coef[5 * N + i] * (src[z > 0 ? i - pl : i] * inv);
      jv += coef[6 * N + i] * (src[z + 1 < d.nz ? i + pl : i] * inv);
    }
    vj[i] = vc;
    w[i] = jv;
  }
  wave_dots(V, N, i, in, jv, j, sh);
  wave_store(vc * jv, sh, j);
  block_flush(sh, j + 1, part, nb);
}

// Passes 2 and 3: w -= sum_{k < nv} g_k v_k, then the partials of v_k . w
// for k < nv (pass 2) or of w . w (pass 3, NORM).
template <bool NORM>
__global__ __launch_bounds__(kThreads) void k_kry_update(Dims d, double* __restrict__ w,
                                                         const double* __restrict__ V, int nv,
                                                         const double* __restrict__ g,
                                                         double* __restrict__ part, int nb) {
  __shared__ double sh[(kMaxKrylov + 1) * kBY];
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const bool in = x < d.nx && y < d.ny;
  const size_t N = d.N;
  const int i = in ? x + d.nx * (y + d.ny * static_cast<int>(blockIdx.z)) : 0;
  double acc = 0.0;
  if (in) {
    acc = w[i];
#pragma unroll 4
    for (int k = 0; k < nv; ++k) acc -= g[k] * V[k * N + i];
    w[i] = acc;
  }
  if (NORM) {
    wave_store(acc * acc, sh, 0);
    block_flush(sh, 1, part, nb);
  } else {
    wave_dots(V, N, i, in, acc, nv, sh);
    block_flush(sh, nv, part, nb);
  }
}

enum RedMode : int { kRedStore = 0, kRedAdd = 1, kRedSqrt = 2 };

// Workgroup k sums the nb partials part[k * nb ..] in a fixed order.
// kRedStore: g[k] = s, H[k * hs] = s; kRedAdd: g[k] = s, H[k * hs] += s;
// kRedSqrt: H[k * hs] = sqrt(s).
__global__ __launch_bounds__(kRedThreads) void k_kry_reduce(const double* __restrict__ part, int nb,
                                                            double* __restrict__ H, int hs,
                                                            double* __restrict__ g, int mode) {
  const int k = blockIdx.x;
  const double s = wave_part_sum(part + static_cast<size_t>(k) * nb, nb);
  if (threadIdx.x != 0) return;
  double* hk = H + static_cast<size_t>(k) * hs;
  if (mode == kRedSqrt) {
    *hk = sqrt(s);
  } else {
    g[k] = s;
    *hk = mode == kRedAdd ? *hk + s : s;
  }
}

// vout = w / *nrm (zero if the norm is zero)
__global__ __launch_bounds__(kThreads) void k_scale(Dims d, const double* __restrict__ w,
                                                    const double* __restrict__ nrm, double* __restrict__ vout) {
  const double h = *nrm;
  const double inv = h > 0.0 ? 1.0 / h : 0.0;
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * static_cast<int>(blockIdx.z));
  vout[i] = w[i] * inv;
}

// u = (first ? 0 : u) + sum_k c_k V_k  (c from device memory)
__global__ __launch_bounds__(kThreads) void k_combine(Dims d, const double* __restrict__ V, int nvec,
                                                      const double* __restrict__ c, double* __restrict__ u,
                                                      int first) {
  const int x = blockIdx.x * kBX + threadIdx.x;
  const int y = blockIdx.y * kBY + threadIdx.y;
  if (x >= d.nx || y >= d.ny) return;
  const int i = x + d.nx * (y + d.ny * static_cast<int>(blockIdx.z));
  const size_t N = d.N;
  double acc = first ? 0.0 : u[i];
  for (int k = 0; k < nvec; ++k) acc += c[k] * V[k * N + i];
  u[i] = acc;
}

}  // namespace

int kry_num_blocks(const Dims& d) { return cell_bands(d); }

// Arnoldi on the start vector in w[0 .. N) (unnormalised; the second half of
// w is the other buffer of the pair): beta = ||w||, then for j = 0..m-1 the
// three passes above, and V[m] = w / h_{m,m-1} at the end.  H (row-major
// (m+1) x m) and beta stay on the device; g holds m + 1 doubles of scratch
// and part (m + 1) * kry_num_blocks(d).
hipError_t arnoldi_cgs2(const Dims& d, const double* coef, double* V, double* w, double* H, double* beta,
                        double* g, double* part, int m, hipStream_t s) {
  const size_t N = d.N;
  const int nb = kry_num_blocks(d);
  const dim3 gr = cell_grid(d), b = cell_block();
  hipLaunchKernelGGL(k_norm_part, gr, b, 0, s, d, w, part);
  hipLaunchKernelGGL(k_kry_reduce, dim3(1), dim3(kRedThreads), 0, s, part, nb, beta, 0, g, kRedSqrt);
  const double* nrm = beta;
  for (int j = 0; j < m; ++j) {
    double* src = w + (j & 1) * N;
    double* wj = w + ((j + 1) & 1) * N;
    if (d.dim == 3)
      hipLaunchKernelGGL(k_kry_spmv<3>, gr, b, 0, s, d, coef, src, nrm, V + j * N, wj, V, j, part, nb);
    else
      hipLaunchKernelGGL(k_kry_spmv<2>, gr, b, 0, s, d, coef, src, nrm, V + j * N, wj, V, j, part, nb);
    hipLaunchKernelGGL(k_kry_reduce, dim3(j + 1), dim3(kRedThreads), 0, s, part, nb, H + j, m, g, kRedStore);
    hipLaunchKernelGGL(k_kry_update<false>, gr, b, 0, s, d, wj, V, j + 1, g, part, nb);
    hipLaunchKernelGGL(k_kry_reduce, dim3(j + 1), dim3(kRedThreads), 0, s, part, nb, H + j, m, g, kRedAdd);
    hipLaunchKernelGGL(k_kry_update<true>, gr, b, 0, s, d, wj, V, j + 1, g, part, nb);
    double* hnext = H + (j + 1) * m + j;
    hipLaunchKernelGGL(k_kry_reduce, dim3(1), dim3(kRedThreads), 0, s, part, nb, hnext, 0, g, kRedSqrt);
    nrm = hnext;
  }
  hipLaunchKernelGGL(k_scale, gr, b, 0, s, d, w + (m & 1) * N, nrm, V + m * N);
  return hipGetLastError();
}

hipError_t krylov_combine(const Dims& d, const double* V, int nvec, const double* c, double* u, int first,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_combine, cell_grid(d), cell_block(), 0, s, d, V, nvec, c, u, first);
  return hipGetLastError();
}

}  // namespace erem
