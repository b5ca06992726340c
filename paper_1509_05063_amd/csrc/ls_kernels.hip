// Device kernels of the operator apply (HIP, gfx950).
//
// Data layout (all vector-major, [rhs][...]):
//   u, v        [nrhs][N] complex, operator order (sorted by cell)
//   sigma       [nrhs][ncell][U] equivalent-source strengths per cell
//   lattice     [nrhs][2 sets][2 kinds][Pa][Pb] zero-padded face lattices
//   after the spectral product the field of set s sits in kind 0.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "ls_kernels.hpp"

namespace lsx {

template <typename T> struct C2;
template <> struct C2<double> { using t = double2; };
template <> struct C2<float> { using t = float2; };

template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename V> __device__ __forceinline__ V cfma(V a, V b, V c) {   // c + a*b
  c.x = fma(a.x, b.x, c.x);
  c.x = fma(-a.y, b.y, c.x);
  c.y = fma(a.x, b.y, c.y);
  c.y = fma(a.y, b.x, c.y);
  return c;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { a.x += b.x; a.y += b.y; return a; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(a.x) s) { a.x *= s; a.y *= s; return a; }
template <typename V> __device__ __forceinline__ V czero() { V r; r.x = 0; r.y = 0; return r; }

// Matrix-core products (16x16x4 tiles).  Operand A: row lane%16, k lane/16;
// operand B: k lane/16, column lane%16.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element held by (lane, r): row lane/16 + 4r, column lane%16
  static __device__ __forceinline__ int row(int lane, int r) { return lane / 16 + 4 * r; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element held by (lane, r): row 4(lane/16) + r, column lane%16
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

// ---------------------------------------------------------------------------
// a1: projection onto equivalent sources.  One workgroup per occupied cell
// and right-hand side; sigma_c = Psh phi_slots + sum_b Pbd_b phi_b with
// phi = c u (plain quadrature weight times density).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_project(const typename C2<T>::t* __restrict__ u,
                                                 typename C2<T>::t* __restrict__ sigma,
                                                 const typename C2<T>::t* __restrict__ Psh,
                                                 const typename C2<T>::t* __restrict__ Pbd,
                                                 const T* __restrict__ cw, const int32_t* __restrict__ slot_map,
                                                 const int32_t* __restrict__ cell_start,
                                                 const int32_t* __restrict__ cell_nint,
                                                 const int32_t* __restrict__ cell_nb,
                                                 const int32_t* __restrict__ cell_boff, int S, int U,
                                                 int64_t N, int ncell) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* phi = reinterpret_cast<V*>(smem_raw);
  const int c = blockIdx.x;
  const int r = blockIdx.y;
  const V* ur = u + (int64_t)r * N;
  const int nb = cell_nb[c];
  const int b0 = cell_start[c] + cell_nint[c];
  for (int a = threadIdx.x; a < S + nb; a += blockDim.x) {
    int64_t j = a < S ? slot_map[(int64_t)c * S + a] : (int64_t)(b0 + a - S);
    phi[a] = j >= 0 ? cscale(ur[j], cw[j]) : czero<V>();
  }
  __syncthreads();
  const int64_t boff = cell_boff[c];
  for (int t = threadIdx.x; t < U; t += blockDim.x) {
    V acc = czero<V>();
    const V* prow = Psh + (int64_t)t * S;
    for (int a = 0; a < S; ++a) acc = cfma(prow[a], phi[a], acc);
    for (int b = 0; b < nb; ++b) acc = cfma(Pbd[(boff + b) * U + t], phi[S + b], acc);
    sigma[((int64_t)r * ncell + c) * U + t] = acc;
  }
}

// Projection, one workgroup of 2 x 96 threads per cell (q = 12: U = 96
// sources, S = 64 slots): thread (g, t) sums half of the slots (PshT, the
// transposed slot matrix [S][U], read coalesced over t) and every other band
// node; the two halves are added through LDS.
template <typename T>
__global__ void __launch_bounds__(192) k_project2(const typename C2<T>::t* __restrict__ u,
                                                  typename C2<T>::t* __restrict__ sigma,
                                                  const typename C2<T>::t* __restrict__ PshT,
                                                  const typename C2<T>::t* __restrict__ Pbd,
                                                  const T* __restrict__ cw, const int32_t* __restrict__ slot_map,
                                                  const int32_t* __restrict__ cell_start,
                                                  const int32_t* __restrict__ cell_nint,
                                                  const int32_t* __restrict__ cell_nb,
                                                  const int32_t* __restrict__ cell_boff, int64_t N, int ncell) {
  using V = typename C2<T>::t;
  constexpr int U = 96, S = 64;
  extern __shared__ unsigned char smem_raw[];
  V* red = reinterpret_cast<V*>(smem_raw);   // [U] second half's sums
  V* phi = red + U;                          // [S + nb]
  const int c = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const V* ur = u + (int64_t)r * N;
  const int nb = cell_nb[c];
  const int64_t b0 = cell_start[c] + cell_nint[c];
  for (int a = tid; a < S + nb; a += blockDim.x) {
    const int64_t j = a < S ? slot_map[(int64_t)c * S + a] : b0 + a - S;
    phi[a] = j >= 0 ? cscale(ur[j], cw[j]) : czero<V>();
  }
  __syncthreads();
  const int t = tid % U, g = tid / U;
  V acc = czero<V>();
#pragma unroll 8
  for (int a = 32 * g; a < 32 * g + 32; ++a) acc = cfma(PshT[a * U + t], phi[a], acc);
  const V* prow = Pbd + (int64_t)cell_boff[c] * U + t;
#pragma unroll 4
  for (int b = g; b < nb; b += 2) acc = cfma(prow[(int64_t)b * U], phi[S + b], acc);
  if (g == 1) red[t] = acc;
  __syncthreads();
  if (g == 0) sigma[((int64_t)r * ncell + c) * U + t] = cadd(acc, red[t]);
}

// a1 for RB right-hand sides per workgroup (batched applies): the weighted
// densities of the cell's nodes for RB right-hand sides are staged in LDS
// ([node][rhs]); each projection value is loaded once and applied to all
// RB of them (per right-hand side the band columns would be re-read from
// L2 every time).  Thread (t, g): output t, half g of the node range.
template <typename T, int RB>
__global__ void __launch_bounds__(192) k_project_rb(const typename C2<T>::t* __restrict__ u,
                                                    typename C2<T>::t* __restrict__ sigma,
                                                    const typename C2<T>::t* __restrict__ PshT,
                                                    const typename C2<T>::t* __restrict__ Pbd,
                                                    const T* __restrict__ cw, const int32_t* __restrict__ slot_map,
                                                    const int32_t* __restrict__ cell_start,
                                                    const int32_t* __restrict__ cell_nint,
                                                    const int32_t* __restrict__ cell_nb,
                                                    const int32_t* __restrict__ cell_boff, int64_t N, int ncell,
                                                    int nrhs) {
  using V = typename C2<T>::t;
  constexpr int U = 96, S = 64;
  extern __shared__ unsigned char smem_raw[];
  const int c = blockIdx.x, r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int nb = cell_nb[c], K = S + nb;
  V* phi = reinterpret_cast<V*>(smem_raw);   // [K][RB]
  V* red = phi + (size_t)K * RB;             // [RB][U] second half's sums
  const int64_t b0 = cell_start[c] + cell_nint[c];
  for (int i = tid; i < K * RB; i += blockDim.x) {
    const int a = i % K, q = i / K, r = r0 + q;    // consecutive threads: consecutive nodes
    const int64_t j = a < S ? slot_map[(int64_t)c * S + a] : b0 + a - S;
    phi[a * RB + q] = (j >= 0 && r < nrhs) ? cscale(u[(int64_t)r * N + j], cw[j]) : czero<V>();
  }
  __syncthreads();
  const int t = tid % U, g = tid / U;
  V acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = czero<V>();
  for (int a = 32 * g; a < 32 * g + 32; ++a) {
    const V p = PshT[a * U + t];
    const V* ph = phi + a * RB;
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = cfma(p, ph[q], acc[q]);
  }
  const V* prow = Pbd + (int64_t)cell_boff[c] * U + t;
  for (int b = g; b < nb; b += 2) {
    const V p = prow[(int64_t)b * U];
    const V* ph = phi + (S + b) * RB;
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = cfma(p, ph[q], acc[q]);
  }
  if (g == 1) {
#pragma unroll
    for (int q = 0; q < RB; ++q) red[q * U + t] = acc[q];
  }
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (r0 + q < nrhs) sigma[((int64_t)(r0 + q) * ncell + c) * U + t] = cadd(acc[q], red[q * U + t]);
  }
}

// a1 on the matrix cores, interior slots (q = 12: U = 96 sources, S = 64
// slots).  The slot projection Psh is the same for every cell, so the
// interior part of all cells and right-hand sides is one product
// Sigma^T [(cells x rhs) x 96] = Phi^T [(cells x rhs) x 64] Psh^T [64 x 96]:
// a row of Phi^T is one (interior cell, right-hand side) pair, phi = c u
// gathered through the slot map.  Psh^T sits in LDS (one copy per
// workgroup); a wave takes tiles of 16 pairs (MFMA A operand: pair
// lane % 16, slots 4 kk + lane / 16), 6 column tiles of 16 sources, 16
// steps of 4 slots.  Output element (pair, source): the 16 lanes of a group
// write 16 consecutive sources of one pair.  G3 (single precision): complex
// products as three real products (Gauss), else four.  Every pair's sums
// run in one fixed order, so a vector's strengths do not depend on the
// other pairs of its launch (alone or in a batch).
//
// One tile of 16 pairs: the products against Psh^T in LDS (the 96 sources
// in two halves of 3 column tiles) and the stores; a[kk]: this lane's
// densities (pair lane % 16, slot 4 kk + lane / 16); lane m < 16 holds
// pair m's right-hand side r (< 0: no pair) and cell c.
template <typename T, bool G3>
__device__ __forceinline__ void proj_tile(const typename C2<T>::t* B, const typename C2<T>::t* a, int r, int c,
                                          int lane, typename C2<T>::t* __restrict__ sigma, int ncell) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int U = 96, KS = 16, RH = U / 32;
  const int kl = lane >> 4, col = lane & 15;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    v4 re[RH], im[RH], p3[G3 ? RH : 1];
#pragma unroll
    for (int rt = 0; rt < RH; ++rt) {
      re[rt] = v4{0, 0, 0, 0};
      im[rt] = v4{0, 0, 0, 0};
      if (G3) p3[rt] = v4{0, 0, 0, 0};
    }
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const V x = a[kk];
      const V* brow = B + (4 * kk + kl) * U + 48 * h + col;
      if (G3) {
        const T xs = x.x + x.y;
#pragma unroll
        for (int rt = 0; rt < RH; ++rt) {
          const V w = brow[16 * rt];
          re[rt] = M::op(xs, w.x, re[rt]);
          im[rt] = M::op(x.y, w.x + w.y, im[rt]);
          p3[rt] = M::op(x.x, w.y - w.x, p3[rt]);
        }
      } else {
#pragma unroll
        for (int rt = 0; rt < RH; ++rt) {
          const V w = brow[16 * rt];
          re[rt] = M::op(x.x, w.x, re[rt]);
          re[rt] = M::op(-x.y, w.y, re[rt]);
          im[rt] = M::op(x.x, w.y, im[rt]);
          im[rt] = M::op(x.y, w.x, im[rt]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int m = M::row(lane, q);
      const int rq = __shfl(r, m, 64), cq = __shfl(c, m, 64);
      if (rq < 0) continue;
      V* out = sigma + ((int64_t)rq * ncell + cq) * U + 48 * h + col;
#pragma unroll
      for (int rt = 0; rt < RH; ++rt) {
        V o;
        if (G3) {
          o.x = re[rt][q] - im[rt][q];
          o.y = re[rt][q] + p3[rt][q];
        } else {
          o.x = re[rt][q];
          o.y = im[rt][q];
        }
        out[16 * rt] = o;
      }
    }
  }
}

// One tile of 16 pairs per wave, 4 waves per workgroup (each workgroup
// copies Psh^T to LDS).
template <typename T, bool G3>
__global__ void __launch_bounds__(256) k_project_int(const typename C2<T>::t* __restrict__ u,
                                                     typename C2<T>::t* __restrict__ sigma,
                                                     const typename C2<T>::t* __restrict__ PshT,
                                                     const T* __restrict__ cw, const int32_t* __restrict__ slot_map,
                                                     const int32_t* __restrict__ icells, int nicell, int ncell,
                                                     int64_t N, int nrhs) {
  using V = typename C2<T>::t;
  constexpr int U = 96, S = 64, KS = S / 4;
  extern __shared__ unsigned char smem_raw[];
  V* B = reinterpret_cast<V*>(smem_raw);      // PshT [S][U]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kl = lane >> 4, col = lane & 15;
  for (int i = tid; i < S * U; i += blockDim.x) B[i] = PshT[i];
  const int64_t ncols = (int64_t)nicell * nrhs;
  const int64_t gc = ((int64_t)blockIdx.x * 4 + wave) * 16 + col;
  const int r = gc < ncols ? (int)(gc / nicell) : -1;
  const int c = gc < ncols ? icells[gc % nicell] : 0;
  V a[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    a[kk] = czero<V>();
    if (r >= 0) {
      const int j = slot_map[(int64_t)c * S + 4 * kk + kl];
      if (j >= 0) a[kk] = cscale(u[(int64_t)r * N + j], cw[j]);
    }
  }
  __syncthreads();
  proj_tile<T, G3>(B, a, r, c, lane, sigma, ncell);
}

// The same for large batches as a persistent kernel: 8 waves per workgroup
// and one workgroup per compute unit (one copy of Psh^T each); each wave
// walks tiles with a stride of the whole grid, three tiles in flight: while
// tile t's products run, the densities of t + 1 (raw values, scaled after
// the products), the slot indices of t + 2 and the cells of t + 3 are being
// loaded.  The products of a pair are those of k_project_int.
template <typename T, bool G3>
__global__ void __launch_bounds__(512) k_project_int_walk(const typename C2<T>::t* __restrict__ u,
                                                          typename C2<T>::t* __restrict__ sigma,
                                                          const typename C2<T>::t* __restrict__ PshT,
                                                          const T* __restrict__ cw,
                                                          const int32_t* __restrict__ slot_map,
                                                          const int32_t* __restrict__ icells, int nicell, int ncell,
                                                          int64_t N, int nrhs) {
  using V = typename C2<T>::t;
  constexpr int U = 96, S = 64, KS = S / 4, NW = 8;
  extern __shared__ unsigned char smem_raw[];
  V* B = reinterpret_cast<V*>(smem_raw);      // PshT [S][U]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kl = lane >> 4, col = lane & 15;
  for (int i = tid; i < S * U; i += blockDim.x) B[i] = PshT[i];
  __syncthreads();
  const int64_t ncols = (int64_t)nicell * nrhs;
  const int64_t ntiles = (ncols + 15) / 16, stride = (int64_t)gridDim.x * NW;
  auto pair_of = [&](int64_t t, int& r, int& c) {
    const int64_t gc = t * 16 + col;
    r = gc < ncols ? (int)(gc / nicell) : -1;
    c = gc < ncols ? icells[gc % nicell] : 0;
  };
  auto slots = [&](int r, int c, int* j) {
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) j[kk] = r >= 0 ? slot_map[(int64_t)c * S + 4 * kk + kl] : -1;
  };
  auto raw = [&](int r, const int* j, V* x, T* w) {
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      x[kk] = j[kk] >= 0 ? u[(int64_t)r * N + j[kk]] : czero<V>();
      w[kk] = j[kk] >= 0 ? cw[j[kk]] : (T)0;
    }
  };
  int64_t t = (int64_t)blockIdx.x * NW + wave;
  if (t >= ntiles) return;
  int r, c, r1, c1, r2, c2;
  int j1[KS];
  V a[KS];
  {
    int j[KS];
    V x[KS];
    T w[KS];
    pair_of(t, r, c);
    slots(r, c, j);
    raw(r, j, x, w);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) a[kk] = cscale(x[kk], w[kk]);
  }
  pair_of(t + stride, r1, c1);
  slots(r1, c1, j1);
  pair_of(t + 2 * stride, r2, c2);
  for (; t < ntiles; t += stride) {
    // keeps the Psh reads from LDS inside the loop (hoisted out of it they
    // would hold the whole matrix in registers)
    asm volatile("" ::: "memory");
    V xn[KS];
    T wn[KS];
    raw(r1, j1, xn, wn);             // densities of t + 1 (r1 < 0: none)
    int j2[KS];
    slots(r2, c2, j2);               // slot indices of t + 2
    int r3, c3;
    pair_of(t + 3 * stride, r3, c3); // cells of t + 3
    proj_tile<T, G3>(B, a, r, c, lane, sigma, ncell);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      a[kk] = cscale(xn[kk], wn[kk]);
      j1[kk] = j2[kk];
    }
    r = r1;
    c = c1;
    r1 = r2;
    c1 = c2;
    r2 = r3;
    c2 = c3;
  }
}

// a1, boundary-patch nodes of a cell (their projection columns Pbd differ
// node by node): sigma[r][c] += sum_b Pbd_b phi_b for RB right-hand sides
// per workgroup, added to the interior part k_project_int wrote (cells with
// interior nodes) or started from zero.  Thread (t, g): source t, the nodes
// b = g mod 2; the odd half is added to the even one through LDS.  The sums
// of one output run in the same order for every RB, so results do not
// depend on the batch.
template <typename T, int RB>
__global__ void __launch_bounds__(192) k_project_band(const typename C2<T>::t* __restrict__ u,
                                                      typename C2<T>::t* __restrict__ sigma,
                                                      const typename C2<T>::t* __restrict__ Pbd,
                                                      const T* __restrict__ cw, const int32_t* __restrict__ bcells,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ cell_nint,
                                                      const int32_t* __restrict__ cell_nb,
                                                      const int32_t* __restrict__ cell_boff, int64_t N, int ncell,
                                                      int nrhs) {
  using V = typename C2<T>::t;
  constexpr int U = 96;
  extern __shared__ unsigned char smem_raw[];
  const int c = bcells[blockIdx.x], r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int nb = cell_nb[c];
  V* phi = reinterpret_cast<V*>(smem_raw);   // [nb][RB]
  V* red = phi + (size_t)nb * RB;            // [RB][U] odd half's sums
  const int64_t b0 = cell_start[c] + cell_nint[c];
  for (int i = tid; i < nb * RB; i += blockDim.x) {
    const int bb = i % nb, q = i / nb, r = r0 + q;    // consecutive threads: consecutive nodes
    const int64_t j = b0 + bb;
    phi[bb * RB + q] = r < nrhs ? cscale(u[(int64_t)r * N + j], cw[j]) : czero<V>();
  }
  __syncthreads();
  const int t = tid % U, g = tid / U;
  const bool has_int = cell_nint[c] > 0;
  V acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q)
    acc[q] = (g == 0 && has_int && r0 + q < nrhs) ? sigma[((int64_t)(r0 + q) * ncell + c) * U + t] : czero<V>();
  const V* prow = Pbd + (int64_t)cell_boff[c] * U + t;
  for (int bb = g; bb < nb; bb += 2) {
    const V p = prow[(int64_t)bb * U];
    const V* ph = phi + bb * RB;
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = cfma(p, ph[q], acc[q]);
  }
  if (g == 1) {
#pragma unroll
    for (int q = 0; q < RB; ++q) red[q * U + t] = acc[q];
  }
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (r0 + q < nrhs) sigma[((int64_t)(r0 + q) * ncell + c) * U + t] = cadd(acc[q], red[q * U + t]);
  }
}

// a1 on the matrix cores for large batches, boundary-patch nodes of a cell
// (their projection columns Pbd differ node by node):
// Sigma^T [rhs x 96] += Phi^T [rhs x nb] Pbd^T [nb x 96] for the cell's nb
// nodes, added to the interior part k_project_int wrote (cells with
// interior nodes) or started from zero.
// One workgroup per (cell, 16 right-hand sides), wave w on sources
// 16 w .. 16 w + 15 (MFMA A operand: right-hand side lane % 16, nodes
// 4 kk + lane / 16; B operand: 16 consecutive sources of Pbd).  Each
// right-hand side's sums run in one fixed order whatever the batch.
template <typename T, bool G3>
__global__ void __launch_bounds__(384) k_project_band_mfma(const typename C2<T>::t* __restrict__ u,
                                                      typename C2<T>::t* __restrict__ sigma,
                                                      const typename C2<T>::t* __restrict__ Pbd,
                                                      const T* __restrict__ cw, const int32_t* __restrict__ bcells,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ cell_nint,
                                                      const int32_t* __restrict__ cell_nb,
                                                      const int32_t* __restrict__ cell_boff, int64_t N, int ncell,
                                                      int nrhs) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int U = 96;
  const int lane = threadIdx.x & 63, kl = lane >> 4, col = lane & 15, rt = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 16;
  const int c = bcells[blockIdx.x];
  const int nb = cell_nb[c];
  const int64_t b0 = cell_start[c] + cell_nint[c];
  const bool rv = r0 + col < nrhs;
  const typename C2<T>::t* __restrict__ ur = u + (int64_t)(rv ? r0 + col : r0) * N + b0;
  const T* __restrict__ cwb = cw + b0;
  const V* __restrict__ prow = Pbd + (int64_t)cell_boff[c] * U + 16 * rt + col;
  v4 re = v4{0, 0, 0, 0}, im = v4{0, 0, 0, 0}, p3 = v4{0, 0, 0, 0};
  // steps of 4 nodes in groups of D = 4 steps; the next group's operands
  // (raw densities and weights) are loaded while the current group's
  // products run
  constexpr int D = 4;
  const int ngroups = (nb + 4 * D - 1) / (4 * D);
  auto load = [&](int g, V* x, T* wc, V* w) {
#pragma unroll
    for (int z = 0; z < D; ++z) {
      const int node = 4 * (D * g + z) + kl;
      const bool ok = node < nb;
      x[z] = ok && rv ? ur[node] : czero<V>();
      wc[z] = ok && rv ? cwb[node] : (T)0;
      w[z] = ok ? prow[(int64_t)node * U] : czero<V>();
    }
  };
  V xn[D], wn[D];
  T cn[D];
  if (ngroups > 0) load(0, xn, cn, wn);
  for (int g = 0; g < ngroups; ++g) {
    V x[D], w[D];
#pragma unroll
    for (int z = 0; z < D; ++z) {
      x[z] = cscale(xn[z], cn[z]);
      w[z] = wn[z];
    }
    if (g + 1 < ngroups) load(g + 1, xn, cn, wn);
#pragma unroll
    for (int z = 0; z < D; ++z) {
      if (G3) {
        re = M::op(x[z].x + x[z].y, w[z].x, re);
        im = M::op(x[z].y, w[z].x + w[z].y, im);
        p3 = M::op(x[z].x, w[z].y - w[z].x, p3);
      } else {
        re = M::op(x[z].x, w[z].x, re);
        re = M::op(-x[z].y, w[z].y, re);
        im = M::op(x[z].x, w[z].y, im);
        im = M::op(x[z].y, w[z].x, im);
      }
    }
  }
  const bool has_int = cell_nint[c] > 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + M::row(lane, q);
    if (r >= nrhs) continue;
    V* out = sigma + ((int64_t)r * ncell + c) * U + 16 * rt + col;
    V o;
    if (G3) {
      o.x = re[q] - im[q];
      o.y = re[q] + p3[q];
    } else {
      o.x = re[q];
      o.y = im[q];
    }
    *out = has_int ? cadd(*out, o) : o;
  }
}

// ---------------------------------------------------------------------------
// Lattice fill: node (a, b) of set s gathers face 0 of the cell whose
// normal index is a and face 1 of the cell a-1 (at most two cells, no
// atomics); zero padding elsewhere.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(const typename C2<T>::t* __restrict__ sigma, typename C2<T>::t* __restrict__ lat,
                       const int32_t* __restrict__ cell_map, int L, int q, int U, int ncell, int na,
                       int nb, int Pa, int Pb) {
  using V = typename C2<T>::t;
  // only the a < na, b < nb corner is written; the transforms treat the
  // rest of the plane as zero without reading it
  const int64_t plane = (int64_t)Pa * Pb;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)na * nb) return;
  const int s = blockIdx.y;       // set
  const int r = blockIdx.z;       // rhs
  const int a = (int)(idx / nb), b = (int)(idx % nb);
  V mono = czero<V>(), dip = czero<V>();
  {
    const int t = b / q, j = b % q;
    for (int f = 0; f < 2; ++f) {
      int cn = a - f;            // cell index along the set's normal axis
      if (cn < 0 || cn >= L) continue;
      int cx = s == 0 ? cn : t, cy = s == 0 ? t : cn;
      int c = cell_map[cy * L + cx];
      if (c < 0) continue;
      const V* sg = sigma + ((int64_t)r * ncell + c) * U + s * 4 * q;
      mono = cadd(mono, sg[f * q + j]);
      dip = cadd(dip, sg[2 * q + f * q + j]);
    }
  }
  V* base = lat + ((int64_t)(r * 2 + s) * 2) * plane + (int64_t)a * Pb + b;
  base[0] = mono;
  base[plane] = dip;
}

// ---------------------------------------------------------------------------
// FFT: Stockham autosort (mixed radix 2/3/4/5), one transform per workgroup
// held in LDS, twiddles from a table W_n^k = exp(-2 pi i k / n).  Pass with
// radix R and current sub-length Ns: butterfly j reads x[j + m n/R],
// multiplies by W^{(j mod Ns) m n/(Ns R)}, applies the R-point DFT and writes
// y[(j / Ns) Ns R + (j mod Ns) + m Ns].
// ---------------------------------------------------------------------------
template <typename V, int DIR>
__device__ __forceinline__ void dft_small(V* v, int R) {
  using T = decltype(v[0].x);
  if (R == 2) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (R == 4) {
    V a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    V b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    // b1 * (-i DIR)
    V rb1;
    rb1.x = DIR > 0 ? b1.y : -b1.y;
    rb1.y = DIR > 0 ? -b1.x : b1.x;
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, rb1);
    v[3] = csub(a1, rb1);
  } else if (R == 3) {
    const T c1 = (T)-0.5, s1 = (T)(DIR > 0 ? -0.86602540378443864676 : 0.86602540378443864676);
    V t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    V y0 = cadd(v[0], t1);
    V m1;
    m1.x = v[0].x + c1 * t1.x;
    m1.y = v[0].y + c1 * t1.y;
    V m2;                         // i s1 t2
    m2.x = -s1 * t2.y;
    m2.y = s1 * t2.x;
    v[0] = y0;
    v[1] = cadd(m1, m2);
    v[2] = csub(m1, m2);
  } else {   // R == 5
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)(DIR > 0 ? -0.95105651629515357212 : 0.95105651629515357212);
    const T s2 = (T)(DIR > 0 ? -0.58778525229247312917 : 0.58778525229247312917);
    V a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    V a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    V y0 = cadd(v[0], cadd(a1, a2));
    V p1, p2;
    p1.x = v[0].x + c1 * a1.x + c2 * a2.x;
    p1.y = v[0].y + c1 * a1.y + c2 * a2.y;
    p2.x = v[0].x + c2 * a1.x + c1 * a2.x;
    p2.y = v[0].y + c2 * a1.y + c1 * a2.y;
    V q1, q2;   // i (s1 b1 + s2 b2), i (s2 b1 - s1 b2)
    q1.x = -(s1 * b1.y + s2 * b2.y);
    q1.y = s1 * b1.x + s2 * b2.x;
    q2.x = -(s2 * b1.y - s1 * b2.y);
    q2.y = s2 * b1.x - s1 * b2.x;
    v[0] = y0;
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
  }
}

// Composite radices R = A B (A the smallest factor) in registers, by one
// Cooley–Tukey step: x[B n1 + n2] -> A-point DFTs over n1, twiddle by
// W_R^{n2 k1}, B-point DFTs over n2 -> X[k1 + A k2].  Twiddles are
// compile-time constants (cosine / sine of 2 pi p / R by a Taylor series on
// [-pi, pi]), so the whole R-point DFT is straight-line code.
constexpr double ce_pi = 3.14159265358979323846264338327950288;
constexpr double ce_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k < 30; ++k) {
    t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    s += t;
  }
  return s;
}
constexpr double ce_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 30; ++k) {
    t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}
// angle of W^p with p folded into (-R/2, R/2]
constexpr double ce_angle(int p, int R) { return 2.0 * ce_pi * (double)(p * 2 > R ? p - R : p) / (double)R; }

template <int R> struct RadixSplit {
  static constexpr int A = R % 2 == 0 ? 2 : R % 3 == 0 ? 3 : 5;
  static constexpr int B = R / A;
};

template <int... I, typename Fn>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, I...>, Fn&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename Fn> __device__ __forceinline__ void sfor(Fn&& f) {
  sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

template <typename V, int DIR, int R>
__device__ __forceinline__ void dft_r(V* x) {
  if constexpr (R == 2 || R == 3 || R == 4 || R == 5) {
    dft_small<V, DIR>(x, R);
  } else {
    using T = decltype(x[0].x);
    constexpr int A = RadixSplit<R>::A, B = RadixSplit<R>::B;
    V y[R];
    sfor<B>([&](auto n2c) {
      constexpr int n2 = decltype(n2c)::value;
      V t[A];
      sfor<A>([&](auto n1c) { t[decltype(n1c)::value] = x[B * decltype(n1c)::value + n2]; });
      dft_r<V, DIR, A>(t);
      sfor<A>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        constexpr int p = (n2 * k1) % R;
        if constexpr (p == 0) {
          y[n2 * A + k1] = t[k1];
        } else {
          // W_R^p = exp(-2 pi i p / R) forward, conjugate inverse
          constexpr double c = ce_cos(ce_angle(p, R)), sn = ce_sin(ce_angle(p, R));
          V w;
          w.x = (T)c;
          w.y = (T)(DIR > 0 ? -sn : sn);
          y[n2 * A + k1] = cmul(t[k1], w);
        }
      });
    });
    sfor<A>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      V t[B];
      sfor<B>([&](auto n2c) { t[decltype(n2c)::value] = y[decltype(n2c)::value * A + k1]; });
      dft_r<V, DIR, B>(t);
      sfor<B>([&](auto k2c) { x[k1 + A * decltype(k2c)::value] = t[decltype(k2c)::value]; });
    });
  }
}

// Division by a divisor d >= 1 fixed at run time, without the integer
// divide sequence: q = floor(x m / 2^32) with m = floor((2^32 - 1) / d) + 1,
// exact for 0 <= x with x d < 2^32 (the error x (m d - 2^32) / (d 2^32)
// stays below 1/d), which every index here satisfies (x < 2^20, d < 2^12).
struct FastDiv {
  uint64_t m;
  int d;
  __device__ __forceinline__ explicit FastDiv(int d_) : m((uint64_t)(0xFFFFFFFFu / (unsigned)d_) + 1), d(d_) {}
  __device__ __forceinline__ int div(int x) const { return (int)(((uint64_t)(unsigned)x * m) >> 32); }
};

template <typename V, int DIR, int R>
__device__ __forceinline__ void stockham_pass(const V* __restrict__ src, V* __restrict__ dst, const V* __restrict__ tw,
                                              int n, int Ns, const FastDiv& fs, int tid, int nthr) {
  const int stride = fs.d;
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  const FastDiv fn(Ns);
  for (int w = tid; w < nb * stride; w += nthr) {
    const int j = fs.div(w), lane = w - j * stride;
    const int jq = fn.div(j), jm = j - jq * Ns;
    V v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      V x = src[(j + m * nb) * stride + lane];
      if (m > 0 && jm > 0) {
        V t = tw[jm * m * twstep];     // jm m < Ns R, so the index stays below n
        if (DIR < 0) t.y = -t.y;
        x = cmul(x, t);
      }
      v[m] = x;
    }
    dft_r<V, DIR, R>(v);
    const int o = jq * Ns * R + jm;
#pragma unroll
    for (int m = 0; m < R; ++m) dst[(o + m * Ns) * stride + lane] = v[m];
  }
}

// Stage nvalid values into LDS: value i = load(i) (a global load) goes to
// dst[slot(i)].  A thread issues the loads of U strides before it waits on
// any: no load sits under a branch (the last strip's indices past nvalid are
// clamped to nvalid - 1, loaded and dropped), so U loads per thread are in
// flight at once.  zero_lds fills slots that stand for zero padding.
template <int U, typename V, typename Ld, typename Sl>
__device__ __forceinline__ void stage_lds(V* dst, int nvalid, Ld&& load, Sl&& slot) {
  for (int base = threadIdx.x; base < nvalid; base += U * (int)blockDim.x) {
    V r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = load(min(base + u * (int)blockDim.x, nvalid - 1));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * (int)blockDim.x;
      if (i < nvalid) dst[slot(i)] = r[u];
    }
  }
}
template <typename V, typename Sl>
__device__ __forceinline__ void zero_lds(V* dst, int count, Sl&& slot) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) dst[slot(i)] = czero<V>();
}

template <typename V, int DIR>
__device__ void stockham_lds(V* buf0, V* buf1, const V* __restrict__ tw, int n, const int8_t* radix,
                             int npass, int stride, int tid, int nthr, V** result) {
  // stride: distance between consecutive elements of one transform in LDS
  // (1 for rows; >1 when several columns are interleaved).
  V* src = buf0;
  V* dst = buf1;
  int Ns = 1;
  const FastDiv fs(stride);
  for (int p = 0; p < npass; ++p) {
    const int R = radix[p];
    switch (R) {
      case 2: stockham_pass<V, DIR, 2>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 3: stockham_pass<V, DIR, 3>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 4: stockham_pass<V, DIR, 4>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 5: stockham_pass<V, DIR, 5>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 6: stockham_pass<V, DIR, 6>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 8: stockham_pass<V, DIR, 8>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 9: stockham_pass<V, DIR, 9>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 10: stockham_pass<V, DIR, 10>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 12: stockham_pass<V, DIR, 12>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      case 15: stockham_pass<V, DIR, 15>(src, dst, tw, n, Ns, fs, tid, nthr); break;
      default: stockham_pass<V, DIR, 16>(src, dst, tw, n, Ns, fs, tid, nthr); break;
    }
    __syncthreads();
    V* t = src;
    src = dst;
    dst = t;
    Ns *= R;
  }
  *result = src;
}

// One Stockham pass in place (one LDS buffer): every butterfly's inputs
// (twiddled) are read into registers, a barrier, then the outputs are
// written.  MB: butterflies per thread, at least n / (R nthr).
template <typename V, int DIR, int R, int MB>
__device__ __forceinline__ void stockham_pass_ip(V* buf, const V* __restrict__ tw, int n, int Ns, int tid,
                                                 int nthr) {
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  const FastDiv fn(Ns);
  V v[MB][R];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = tid + b * nthr;
    if (j < nb) {
      const int jq = fn.div(j), jm = j - jq * Ns;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        V x = buf[j + m * nb];
        if (m > 0 && jm > 0) {
          V t = tw[jm * m * twstep];
          if (DIR < 0) t.y = -t.y;
          x = cmul(x, t);
        }
        v[b][m] = x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = tid + b * nthr;
    if (j < nb) {
      const int jq = fn.div(j), jm = j - jq * Ns;
      dft_r<V, DIR, R>(v[b]);
      const int o = jq * Ns * R + jm;
#pragma unroll
      for (int m = 0; m < R; ++m) buf[o + m * Ns] = v[b][m];
    }
  }
  __syncthreads();
}

// All passes in place for a row of n <= NMAX points with NTH threads.
template <typename V, int DIR, int NTH, int NMAX>
__device__ void stockham_lds_ip(V* buf, const V* __restrict__ tw, int n, const int8_t* radix, int npass, int tid) {
  int Ns = 1;
  for (int p = 0; p < npass; ++p) {
    const int R = radix[p];
#define LS_IP(RR) stockham_pass_ip<V, DIR, RR, (NMAX / RR + NTH - 1) / NTH>(buf, tw, n, Ns, tid, NTH)
    switch (R) {
      case 2: LS_IP(2); break;
      case 3: LS_IP(3); break;
      case 4: LS_IP(4); break;
      case 5: LS_IP(5); break;
      case 6: LS_IP(6); break;
      case 8: LS_IP(8); break;
      case 9: LS_IP(9); break;
      case 10: LS_IP(10); break;
      case 12: LS_IP(12); break;
      case 15: LS_IP(15); break;
      default: LS_IP(16); break;
    }
#undef LS_IP
    Ns *= R;
  }
}

// Row transforms with one LDS buffer (half the LDS of k_fft_rows, two
// barriers per pass); rows of at most NMAX points.
template <typename T, int DIR, int NTH>
__global__ void __launch_bounds__(NTH) k_fft_rows_ip(typename C2<T>::t* data, const typename C2<T>::t* __restrict__ tw,
                                                     FftPlan plan, int64_t line_stride, int nload, int nstore,
                                                     int64_t batch_stride) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* b0 = reinterpret_cast<V*>(smem_raw);
  V* x = data + blockIdx.y * batch_stride + (int64_t)blockIdx.x * line_stride;
  const int nl = min(nload, plan.n);
  stage_lds<8>(b0, nl, [&](int i) { return x[i]; }, [](int i) { return i; });
  zero_lds(b0 + nl, plan.n - nl, [](int i) { return i; });
  __syncthreads();
  stockham_lds_ip<V, DIR, NTH, kRowIpMax>(b0, tw, plan.n, plan.radix, plan.npass, threadIdx.x);
  for (int i = threadIdx.x; i < nstore; i += NTH) x[i] = b0[i];
}

// transforms along the contiguous axis: one line per workgroup
// (entries past nload are zero padding: not read; entries past nstore are
// not needed downstream: not written)
template <typename T, int DIR, int NTH>
__global__ void __launch_bounds__(NTH) k_fft_rows(typename C2<T>::t* data, const typename C2<T>::t* __restrict__ tw,
                                                  FftPlan plan, int64_t line_stride, int nload, int nstore,
                                                  int64_t batch_stride, int64_t zstride = 0) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* b0 = reinterpret_cast<V*>(smem_raw);
  V* b1 = b0 + plan.n;
  const int line = blockIdx.x;
  const int batch = blockIdx.y;
  V* x = data + blockIdx.z * zstride + batch * batch_stride + (int64_t)line * line_stride;
  const int nl = min(nload, plan.n);
  stage_lds<8>(b0, nl, [&](int i) { return x[i]; }, [](int i) { return i; });
  zero_lds(b0 + nl, plan.n - nl, [](int i) { return i; });
  __syncthreads();
  V* res;
  stockham_lds<V, DIR>(b0, b1, tw, plan.n, plan.radix, plan.npass, 1, threadIdx.x, blockDim.x, &res);
  for (int i = threadIdx.x; i < nstore; i += blockDim.x) x[i] = res[i];
}

// transforms of short contiguous lines, L lines per workgroup: the lines are
// read along their length (coalesced) and interleaved in LDS with stride
// S = L + 1 (a padding lane against bank conflicts; S = 1 for one line), so
// the Stockham passes run over all L lines at once.  Separate source and
// destination (they may alias: a workgroup reads its lines whole before it
// writes them); source entries past nload are zero padding (not read),
// destination entries past nstore are not written.  Grid: (lines / L,
// batch, z).
template <typename T, int DIR>
__global__ void __launch_bounds__(256) k_fft_lines(const typename C2<T>::t* src, typename C2<T>::t* dst,
                                                   const typename C2<T>::t* __restrict__ tw, FftPlan plan, int nlines,
                                                   int L, int64_t s_line, int64_t s_batch, int64_t s_z, int64_t d_line,
                                                   int64_t d_batch, int64_t d_z, int nload, int nstore) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  const int n = plan.n, S = L == 1 ? 1 : L + 1;
  V* b0 = reinterpret_cast<V*>(smem_raw);
  V* b1 = b0 + (size_t)n * S;
  V* twl = b1 + (size_t)n * S;   // the twiddles, staged with the data
  const int l0 = blockIdx.x * L;
  const int nl = min(L, nlines - l0);
  const V* x = src + blockIdx.z * s_z + blockIdx.y * s_batch + (int64_t)l0 * s_line;
  // lanes l >= nl transform a copy of the last line and are not stored
  const int ne = min(nload, n), nz = n - ne;
  const FastDiv fe(ne);
  stage_lds<8>(
      b0, L * ne,
      [&](int i) {
        const int l = fe.div(i);
        return x[(int64_t)min(l, nl - 1) * s_line + (i - l * ne)];
      },
      [&](int i) {
        const int l = fe.div(i);
        return (i - l * ne) * S + l;
      });
  if (nz > 0) {
    const FastDiv fz(nz);
    zero_lds(b0, L * nz, [&](int i) {
      const int l = fz.div(i);
      return (ne + i - l * nz) * S + l;
    });
  }
  stage_lds<4>(twl, n, [&](int i) { return tw[i]; }, [](int i) { return i; });
  __syncthreads();
  V* res;
  stockham_lds<V, DIR>(b0, b1, twl, n, plan.radix, plan.npass, S, threadIdx.x, blockDim.x, &res);
  V* y = dst + blockIdx.z * d_z + blockIdx.y * d_batch + (int64_t)l0 * d_line;
  const FastDiv fst(nstore);
  for (int i = threadIdx.x; i < nstore * L; i += blockDim.x) {
    const int l = fst.div(i), e = i - l * nstore;
    if (l < nl) y[(int64_t)l * d_line + e] = res[e * S + l];
  }
}

// XCD-aware column tiles: workgroups are dispatched round-robin over the 8
// XCDs (block b on XCD b % 8), so XCD x is given the contiguous tiles
// [x per, (x + 1) per); a workgroup reads TC columns (a quarter of a 128-byte
// line at TC = 4 in single precision), and its neighbours, now on the same
// XCD, find the rest of the line in that XCD's L2 instead of fetching it
// again.  Launch with grid.x = 8 per; -1 past the last tile.
__device__ __forceinline__ int xcd_tile(int ntiles) {
  const int per = gridDim.x / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  return t < ntiles ? t : -1;
}
inline unsigned xcd_grid(int ntiles) { return 8u * (unsigned)((ntiles + 7) / 8); }

// transforms along the strided axis: a workgroup takes TC adjacent columns
template <typename T, int DIR>
// (rows past nload are zero padding: not read; rows past nstore: not written)
__global__ void __launch_bounds__(256) k_fft_cols(typename C2<T>::t* data, const typename C2<T>::t* __restrict__ tw,
                                                  FftPlan plan, int ncols, int TC, int64_t batch_stride, int nload,
                                                  int nstore, int64_t zstride = 0) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* b0 = reinterpret_cast<V*>(smem_raw);
  V* b1 = b0 + plan.n * TC;
  V* twl = b1 + plan.n * TC;   // the twiddles, staged with the data
  const int tile = xcd_tile((ncols + TC - 1) / TC);
  if (tile < 0) return;
  const int c0 = tile * TC;
  const int batch = blockIdx.y;
  const int tc = min(TC, ncols - c0);
  V* x = data + blockIdx.z * zstride + batch * batch_stride + c0;
  // columns col >= tc (last tile) transform copies of column tc - 1 and are
  // not stored; rows >= nload are zero padding
  const int nr = min(nload, plan.n);
  const FastDiv ft(TC);
  stage_lds<8>(
      b0, nr * TC,
      [&](int i) {
        const int row = ft.div(i), col = i - row * TC;
        return x[(int64_t)row * ncols + min(col, tc - 1)];
      },
      [](int i) { return i; });
  zero_lds(b0 + nr * TC, (plan.n - nr) * TC, [](int i) { return i; });
  stage_lds<4>(twl, plan.n, [&](int i) { return tw[i]; }, [](int i) { return i; });
  __syncthreads();
  V* res;
  stockham_lds<V, DIR>(b0, b1, twl, plan.n, plan.radix, plan.npass, TC, threadIdx.x, blockDim.x, &res);
  for (int i = threadIdx.x; i < nstore * TC; i += blockDim.x) {
    const int row = ft.div(i), col = i - row * TC;
    if (col < tc) x[(int64_t)row * ncols + col] = res[i];
  }
}

// The fused pass along the normal axis of the 3-D face lattices: as
// k_fft_cols_conv (forward transform of both kinds of a TC-column tile,
// spectral product, inverse transform, rows < na of kind 0 written back),
// with the kernel spectra read from one octant.  The monopole kernel
// lattice is even in each axis offset and the dipole one odd in the normal
// offset and even in the other two, so their spectra are even per axis,
// except the dipole's, odd along the normal axis: the entry at frequency
// (ka, kb, kc) is that at (min(ka, Pa - ka), min(kb, Pb - kb), min(kc, Pc -
// kc)) in khs [2][Pa/2 + 1][Pb/2 + 1][Pc/2 + 1], the dipole's negated when
// ka > Pa / 2.  Rows (normal-axis planes) are rstride >= Pb Pc apart, a
// kind's array vol; grid: (tiles, sets), set s at lat + 2 s vol.
template <typename T, int NTH>
__global__ void __launch_bounds__(NTH) k_fft_conv_octant(typename C2<T>::t* lat, const typename C2<T>::t* __restrict__ tw,
                                                         const typename C2<T>::t* __restrict__ khs, FftPlan plan,
                                                         int Pb, int Pc, int TC, int64_t rstride, int64_t vol, int na) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  const int n = plan.n, W = 2 * TC, ncols = Pb * Pc;
  const int hb = Pb / 2 + 1, hc = Pc / 2 + 1;
  const int64_t hsz = (int64_t)(n / 2 + 1) * hb * hc;
  V* b0 = reinterpret_cast<V*>(smem_raw);   // [n][2 TC]: monopole columns, then dipole columns
  V* b1 = b0 + (size_t)n * W;
  V* twl = b1 + (size_t)n * W;               // the twiddles, staged with the data
  const int tile = xcd_tile((ncols + TC - 1) / TC);
  if (tile < 0) return;
  const int c0 = tile * TC;
  const int tc = min(TC, ncols - c0);
  V* mp = lat + (int64_t)blockIdx.y * 2 * vol + c0;
  // columns col >= tc (last tile) transform copies of column tc - 1 and
  // give zero products (not stored); rows >= na are zero padding
  const int nr = min(na, n);
  const FastDiv fw(W), ft(TC);
  stage_lds<8>(
      b0, nr * W,
      [&](int i) {
        const int row = fw.div(i), cc = i - row * W, kind = cc >= TC, col = cc - kind * TC;
        return mp[kind * vol + (int64_t)row * rstride + min(col, tc - 1)];
      },
      [](int i) { return i; });
  zero_lds(b0 + nr * W, (n - nr) * W, [](int i) { return i; });
  stage_lds<4>(twl, n, [&](int i) { return tw[i]; }, [](int i) { return i; });
  // octant entry of product entry i (row = normal frequency, column
  // within the tile; columns past tc read a valid entry, their product is 0)
  const FastDiv fpc(Pc);
  auto kidx = [&](int i) {
    const int row = ft.div(i), cg = c0 + min(i - row * TC, tc - 1), kb = fpc.div(cg), kc = cg - kb * Pc;
    const int ma = row <= n - row ? row : n - row, mb = kb <= Pb - kb ? kb : Pb - kb,
              mc = kc <= Pc - kc ? kc : Pc - kc;
    return ((int64_t)ma * hb + mb) * hc + mc;
  };
  // the spectra of this thread's first KP product entries, loaded now so
  // they arrive during the forward transform
  constexpr int KP = 8;
  const int np = n * TC;
  V pg[KP], pd[KP];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int64_t k = kidx(min((int)threadIdx.x + u * NTH, np - 1));
    pg[u] = khs[k];
    pd[u] = khs[hsz + k];
  }
  __syncthreads();
  V* res;
  stockham_lds<V, 1>(b0, b1, twl, n, plan.radix, plan.npass, W, threadIdx.x, blockDim.x, &res);
  V* fr = res == b0 ? b1 : b0;               // free buffer: two [n][TC] halves
  auto product = [&](int i, V g, V d) {
    const int row = ft.div(i), col = i - row * TC;
    V o = czero<V>();
    if (col < tc) {
      if (row > n - row) {   // the dipole spectrum is odd along the normal axis
        d.x = -d.x;
        d.y = -d.y;
      }
      o = cmul(res[row * W + col], g);
      o = cfma(res[row * W + TC + col], d, o);
    }
    fr[i] = o;
  };
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int i = threadIdx.x + u * NTH;
    if (i < np) product(i, pg[u], pd[u]);
  }
  for (int i = threadIdx.x + KP * NTH; i < np; i += NTH) {
    const int64_t k = kidx(i);
    product(i, khs[k], khs[hsz + k]);
  }
  __syncthreads();
  V* res2;
  stockham_lds<V, -1>(fr, fr + (size_t)n * TC, twl, n, plan.radix, plan.npass, TC, threadIdx.x, blockDim.x, &res2);
  for (int i = threadIdx.x; i < na * TC; i += blockDim.x) {
    const int row = ft.div(i), col = i - row * TC;
    if (col < tc) mp[(int64_t)row * rstride + col] = res2[i];
  }
}

// Lines of n = R1 R2 points (two Stockham passes) without staging: 16
// threads per line (one per butterfly), 16 lines per workgroup.  The first
// pass reads its R1 inputs straight from memory (for each of them the 16
// threads of a line read 16 consecutive points: coalesced; points past
// nload are zero), writes the intermediate to LDS with a span of R1 + 1 per
// R1 values (no bank conflicts), and after one barrier the second pass
// writes points < nstore straight to the destination.  Same arguments and
// results as k_fft_lines.  Requires R1 == R2 == 16.
template <int DIR, int R1, int R2>
__global__ void __launch_bounds__(256) k_fft_lines2(const float2* src, float2* dst, const float2* __restrict__ tw,
                                                    int nlines, int64_t s_line, int64_t s_batch, int64_t s_z,
                                                    int64_t d_line, int64_t d_batch, int64_t d_z, int nload,
                                                    int nstore) {
  static_assert(R1 == 16 && R2 == 16, "one thread per butterfly of each pass");
  using V = float2;
  constexpr int n = R1 * R2, TPL = 16, L = 256 / TPL, SPAN = R2 * (R1 + 1);
  extern __shared__ unsigned char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);   // [L][R2][R1 + 1]
  V* twl = buf + (size_t)L * SPAN;           // [n] twiddles
  for (int i = threadIdx.x; i < n; i += blockDim.x) twl[i] = tw[i];
  const int l = threadIdx.x / TPL, j = threadIdx.x % TPL;
  const int l0 = blockIdx.x * L;
  const int nl = min(L, nlines - l0);
  const int lc = min(l, nl - 1);             // lines past the last: a copy of it, not stored
  const V* x = src + blockIdx.z * s_z + blockIdx.y * s_batch + (int64_t)(l0 + lc) * s_line;
  const int ne = min(nload, n);
  V* b = buf + l * SPAN;
  {
    V v[R1];
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const int e = j + m * R2;
      v[m] = e < ne ? x[e] : czero<V>();     // masked: padding is not loaded
    }
    dft_r<V, DIR, R1>(v);
#pragma unroll
    for (int m = 0; m < R1; ++m) b[j * (R1 + 1) + m] = v[m];
  }
  __syncthreads();
  {
    V v[R2];
#pragma unroll
    for (int m = 0; m < R2; ++m) {
      V t = b[m * (R1 + 1) + j];   // intermediate row j + m R1
      if (m > 0 && j > 0) {
        V wv = twl[j * m];
        if (DIR < 0) wv.y = -wv.y;
        t = cmul(t, wv);
      }
      v[m] = t;
    }
    dft_r<V, DIR, R2>(v);
    if (l < nl) {
      V* y = dst + blockIdx.z * d_z + blockIdx.y * d_batch + (int64_t)(l0 + l) * d_line;
#pragma unroll
      for (int m = 0; m < R2; ++m) {
        const int e = j + m * R1;
        if (e < nstore) y[e] = v[m];
      }
    }
  }
}

// Column transforms of length n = R1 R2 (two Stockham passes) without
// staging: the first pass reads its R1 inputs per column straight from
// memory (rows past nload are zero padding, not loaded), writes
// the intermediate to one LDS buffer; after one barrier the second pass
// (twiddles from LDS) writes rows < nstore straight back.  Same grid,
// arguments and results as k_fft_cols, half its LDS and none of its staging
// copies.
template <int DIR, int R1, int R2>
__global__ void __launch_bounds__(256) k_fft_cols2(float2* data, const float2* __restrict__ tw, int ncols, int TC,
                                                   int64_t batch_stride, int nload, int nstore, int64_t zstride) {
  using V = float2;
  constexpr int n = R1 * R2;
  extern __shared__ unsigned char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);   // [n][TC]
  V* twl = buf + (size_t)n * TC;              // [n] twiddles
  const int tile = xcd_tile((ncols + TC - 1) / TC);
  if (tile < 0) return;
  const int c0 = tile * TC;
  const int tc = min(TC, ncols - c0);
  V* x = data + blockIdx.z * zstride + blockIdx.y * batch_stride + c0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) twl[i] = tw[i];
  const FastDiv ft(TC);
  const int nl = min(nload, n);
  // pass 1 (span 1): column lane, butterfly j reads rows j + m R2
  for (int w = threadIdx.x; w < R2 * TC; w += blockDim.x) {
    const int j = ft.div(w), lane = w - j * TC, col = min(lane, tc - 1);
    V v[R1];
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const int row = j + m * R2;
      v[m] = row < nl ? x[(int64_t)row * ncols + col] : czero<V>();   // masked: padding is not loaded
    }
    dft_r<V, DIR, R1>(v);
#pragma unroll
    for (int m = 0; m < R1; ++m) buf[(j * R1 + m) * TC + lane] = v[m];
  }
  __syncthreads();
  // pass 2 (span R1): butterfly j < R1 reads rows j + m R1, twiddles
  // W_n^(j m), writes rows j + m R1
  for (int w = threadIdx.x; w < R1 * TC; w += blockDim.x) {
    const int j = ft.div(w), lane = w - j * TC;
    V v[R2];
#pragma unroll
    for (int m = 0; m < R2; ++m) {
      V t = buf[(j + m * R1) * TC + lane];
      if (m > 0 && j > 0) {
        V wv = twl[j * m];
        if (DIR < 0) wv.y = -wv.y;
        t = cmul(t, wv);
      }
      v[m] = t;
    }
    dft_r<V, DIR, R2>(v);
    if (lane < tc) {
#pragma unroll
      for (int m = 0; m < R2; ++m) {
        const int row = j + m * R1;
        if (row < nstore) x[(int64_t)row * ncols + lane] = v[m];
      }
    }
  }
}

// The fused normal-axis pass of k_fft_conv_octant for n = R1 R2 with two
// Stockham passes each way, 16-column tiles (both kinds: 32 columns) and
// 256 threads, without staging: the forward radix-R1 pass loads straight
// from memory, the forward radix-R2 pass goes through LDS, the spectral
// product is taken inside the inverse radix-R1 pass (its octant entries
// loaded at entry, so they arrive during the forward transform), and the
// inverse radix-R2 pass stores the na lattice rows straight back.  Same grid,
// arguments and results as k_fft_conv_octant with TC = 16.
template <int R1, int R2>
__global__ void __launch_bounds__(256) k_fft_conv_octant2(float2* lat, const float2* __restrict__ tw,
                                                          const float2* __restrict__ khs, int Pb, int Pc,
                                                          int64_t rstride, int64_t vol, int na) {
  using V = float2;
  constexpr int n = R1 * R2, TC = 16, W = 32;
  extern __shared__ unsigned char smem_raw[];
  // one buffer (19 KB, so eight workgroups fit a compute unit): [n][W]
  // through the forward passes (the radix-R2 pass writes back exactly the
  // entries it read), then [n][TC] from the inverse radix-R1 pass on
  V* A = reinterpret_cast<V*>(smem_raw);
  V* twl = A + n * W;                        // [n]
  const int ncols = Pb * Pc;
  const int hb = Pb / 2 + 1, hc = Pc / 2 + 1;
  const int64_t hsz = (int64_t)(n / 2 + 1) * hb * hc;
  const int tile = xcd_tile((ncols + TC - 1) / TC);
  if (tile < 0) return;
  const int c0 = tile * TC;
  const int tc = min(TC, ncols - c0);
  V* mp = lat + (int64_t)blockIdx.y * 2 * vol + c0;
  const int t = threadIdx.x;
  for (int i = t; i < n; i += 256) twl[i] = tw[i];
  // octant offset of this thread's product column (inverse pass 1: column
  // c = t % TC); the entries are loaded in that pass, from L2 (holding them
  // in registers through the forward transform, or staging the tile's
  // octant rows in LDS, measured slower)
  int64_t koff = 0;
  if (t < R2 * TC) {
    const int c = t % TC;
    const FastDiv fpc(Pc);
    const int cg = c0 + min(c, tc - 1), kb = fpc.div(cg), kc = cg - kb * Pc;
    const int mb = kb <= Pb - kb ? kb : Pb - kb, mc = kc <= Pc - kc ? kc : Pc - kc;
    koff = (int64_t)mb * hc + mc;
  }
  const int nr = min(na, n);
  // forward pass 1 (radix R1, span 1): butterfly j < R2 of column lane;
  // rows >= nr are zero padding and not loaded (masked loads, so a wave
  // whose rows all lie in the padding issues no request)
  if (t < R2 * W) {
    const int j = t / W, lane = t % W, kind = lane / TC, col = min(lane % TC, tc - 1);
    const V* src = mp + kind * vol + col;
    V v[R1];
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const int row = j + m * R2;
      v[m] = row < nr ? src[(int64_t)row * rstride] : czero<V>();
    }
    dft_r<V, 1, R1>(v);
#pragma unroll
    for (int m = 0; m < R1; ++m) A[(j * R1 + m) * W + lane] = v[m];
  }
  __syncthreads();
  // forward pass 2 (radix R2, span R1): butterfly j < R1, in place (it
  // writes back the rows j + m R1 it read, so no barrier between)
  for (int w = t; w < R1 * W; w += 256) {
    const int j = w / W, lane = w % W;
    V v[R2];
#pragma unroll
    for (int m = 0; m < R2; ++m) {
      V x = A[(j + m * R1) * W + lane];
      if (m > 0 && j > 0) x = cmul(x, twl[j * m]);
      v[m] = x;
    }
    dft_r<V, 1, R2>(v);
#pragma unroll
    for (int m = 0; m < R2; ++m) A[(j + m * R1) * W + lane] = v[m];
  }
  __syncthreads();
  // spectral product and inverse pass 1 (radix R1, span 1): butterfly j < R2
  // of column c; the dipole spectrum is odd along the normal axis.  Its
  // output layout [n][TC] overlaps other threads' inputs: all read first.
  V vi[R1];
  if (t < R2 * TC) {
    const int j = t / TC, c = t % TC;
    V pg[R1], pd[R1];
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const int row = j + m * R2, ma = row <= n - row ? row : n - row;
      const int64_t k = (int64_t)ma * hb * hc + koff;
      pg[m] = khs[k];
      pd[m] = khs[hsz + k];
    }
#pragma unroll
    for (int m = 0; m < R1; ++m) {
      const int row = j + m * R2;
      V d = pd[m];
      if (row > n - row) {
        d.x = -d.x;
        d.y = -d.y;
      }
      V o = cmul(A[row * W + c], pg[m]);
      vi[m] = cfma(A[row * W + TC + c], d, o);
    }
    dft_r<V, -1, R1>(vi);
  }
  __syncthreads();
  if (t < R2 * TC) {
    const int j = t / TC, c = t % TC;
#pragma unroll
    for (int m = 0; m < R1; ++m) A[(j * R1 + m) * TC + c] = vi[m];
  }
  __syncthreads();
  // inverse pass 2 (radix R2, span R1): butterfly j < R1; rows < na stored
  if (t < R1 * TC) {
    const int j = t / TC, c = t % TC;
    V v[R2];
#pragma unroll
    for (int m = 0; m < R2; ++m) {
      V x = A[(j + m * R1) * TC + c];
      if (m > 0 && j > 0) {
        V wv = twl[j * m];
        wv.y = -wv.y;
        x = cmul(x, wv);
      }
      v[m] = x;
    }
    dft_r<V, -1, R2>(v);
    if (c < tc) {
#pragma unroll
      for (int m = 0; m < R2; ++m) {
        const int row = j + m * R1;
        if (row < nr) mp[(int64_t)row * rstride + c] = v[m];
      }
    }
  }
}

// Column transforms, spectral product and inverse column transform in one
// workgroup per TC-column tile of one set: the tile's monopole and dipole
// columns are transformed together (2 TC interleaved columns), multiplied by
// the set's two kernel spectra (set s's pair at khat + s kset_stride; a
// stride of 0 gives every set the same pair) and summed, and the sum is
// transformed back;
// only rows < na (the ones the interpolation reads) go back to memory, in the
// set's kind-0 plane.
template <typename T, int NTH>
__global__ void __launch_bounds__(NTH) k_fft_cols_conv(typename C2<T>::t* lat, const typename C2<T>::t* __restrict__ tw,
                                                       const typename C2<T>::t* __restrict__ khat, FftPlan plan,
                                                       int ncols, int TC, int64_t plane, int na, int64_t kset_stride) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  const int n = plan.n, W = 2 * TC;
  V* b0 = reinterpret_cast<V*>(smem_raw);   // [n][2 TC]: monopole columns, then dipole columns
  V* b1 = b0 + (size_t)n * W;
  V* twl = b1 + (size_t)n * W;               // the twiddles, staged with the data
  const int tile = xcd_tile((ncols + TC - 1) / TC);
  if (tile < 0) return;
  const int c0 = tile * TC;
  const int s = blockIdx.y & 1, r = blockIdx.y >> 1;
  const int tc = min(TC, ncols - c0);
  V* mp = lat + ((int64_t)(r * 2 + s) * 2) * plane + c0;
  // columns col >= tc (last tile) transform copies of column tc - 1 and
  // give zero products (not stored); rows >= na are zero padding
  const int nr = min(na, n);
  const FastDiv fw(W), ft(TC);
  stage_lds<8>(
      b0, nr * W,
      [&](int i) {
        const int row = fw.div(i), cc = i - row * W, kind = cc >= TC, col = cc - kind * TC;
        return mp[kind * plane + (int64_t)row * ncols + min(col, tc - 1)];
      },
      [](int i) { return i; });
  zero_lds(b0 + nr * W, (n - nr) * W, [](int i) { return i; });
  stage_lds<4>(twl, n, [&](int i) { return tw[i]; }, [](int i) { return i; });
  // the spectra of this thread's first KP product entries, loaded now so
  // they arrive during the forward transform
  constexpr int KP = sizeof(T) == 4 ? 8 : 4;
  const int np = n * TC;
  const V* km = khat + s * kset_stride + c0;
  auto kidx = [&](int i) {
    const int row = ft.div(i), col = i - row * TC;
    return (int64_t)row * ncols + min(col, tc - 1);
  };
  V pg[KP], pd[KP];
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int64_t k = kidx(min((int)threadIdx.x + u * NTH, np - 1));
    pg[u] = km[k];
    pd[u] = km[plane + k];
  }
  __syncthreads();
  V* res;
  stockham_lds<V, 1>(b0, b1, twl, n, plan.radix, plan.npass, W, threadIdx.x, blockDim.x, &res);
  V* fr = res == b0 ? b1 : b0;               // free buffer: two [n][TC] halves
#pragma unroll
  for (int u = 0; u < KP; ++u) {
    const int i = threadIdx.x + u * NTH;
    if (i < np) {
      const int row = ft.div(i), col = i - row * TC;
      V o = czero<V>();
      if (col < tc) {
        o = cmul(res[row * W + col], pg[u]);
        o = cfma(res[row * W + TC + col], pd[u], o);
      }
      fr[i] = o;
    }
  }
  for (int i = threadIdx.x + KP * NTH; i < np; i += NTH) {
    const int row = ft.div(i), col = i - row * TC;
    V o = czero<V>();
    if (col < tc) {
      const int64_t k = kidx(i);
      o = cmul(res[row * W + col], km[k]);
      o = cfma(res[row * W + TC + col], km[plane + k], o);
    }
    fr[i] = o;
  }
  __syncthreads();
  V* res2;
  stockham_lds<V, -1>(fr, fr + (size_t)n * TC, twl, n, plan.radix, plan.npass, TC, threadIdx.x, blockDim.x, &res2);
  for (int i = threadIdx.x; i < na * TC; i += blockDim.x) {
    const int row = ft.div(i), col = i - row * TC;
    if (col < tc) mp[(int64_t)row * ncols + col] = res2[i];
  }
}

// spectral product: set s field = FFT(mono) Khat_m + FFT(dip) Khat_d (into kind 0)
template <typename T>
__global__ void k_spectral(typename C2<T>::t* __restrict__ lat, const typename C2<T>::t* __restrict__ khat,
                           int64_t plane) {
  using V = typename C2<T>::t;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= plane) return;
  const int s = blockIdx.y, r = blockIdx.z;
  V* m = lat + ((int64_t)(r * 2 + s) * 2) * plane;
  const V* km = khat + (int64_t)(s * 2) * plane;
  V out = cmul(m[idx], km[idx]);
  out = cfma(m[plane + idx], km[plane + idx], out);
  m[idx] = out;
}

// ---------------------------------------------------------------------------
// a3 + a5: per cell, the face values of the lattice field, Dirichlet fit
// to the cell's nodes, v = u + kappa^2 far.  The adjacent cells' part of
// the field (their equivalent sources seen at the faces) is subtracted
// through the near-field weights, where it was folded in at set-up.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_interp(const typename C2<T>::t* __restrict__ u,
                                                typename C2<T>::t* __restrict__ v,
                                                const typename C2<T>::t* __restrict__ lat,
                                                const typename C2<T>::t* __restrict__ IshT,
                                                const typename C2<T>::t* __restrict__ Ibd,
                                                const int32_t* __restrict__ cell_xy,
                                                const int32_t* __restrict__ slot_map,
                                                const int32_t* __restrict__ cell_start,
                                                const int32_t* __restrict__ cell_nint,
                                                const int32_t* __restrict__ cell_nb,
                                                const int32_t* __restrict__ cell_boff, int q, int F, int S,
                                                int Pa, int Pb, int64_t N, int64_t nband, T k2) {
  // IshT [F][S], IbdT [F][nband]
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* f = reinterpret_cast<V*>(smem_raw);      // F face values
  const int c = blockIdx.x, r = blockIdx.y;
  const int cx = cell_xy[2 * c], cy = cell_xy[2 * c + 1];
  const int64_t plane = (int64_t)Pa * Pb;
  for (int t = threadIdx.x; t < F; t += blockDim.x) {
    int s = t / (2 * q), fj = t % (2 * q), fc = fj / q, j = fj % q;
    int cn = (s == 0 ? cx : cy) + fc, ct = (s == 0 ? cy : cx);
    f[t] = lat[((int64_t)(r * 2 + s) * 2) * plane + (int64_t)cn * Pb + ct * q + j];
  }
  __syncthreads();
  const V* ur = u + (int64_t)r * N;
  V* vr = v + (int64_t)r * N;
  const int nint = cell_nint[c], nb = cell_nb[c];
  for (int a = threadIdx.x; a < S; a += blockDim.x) {
    int j = slot_map[(int64_t)c * S + a];
    if (j < 0) continue;
    V acc = czero<V>();
    for (int t = 0; t < F; ++t) acc = cfma(IshT[(int64_t)t * S + a], f[t], acc);
    vr[j] = cadd(ur[j], cscale(acc, k2));
  }
  const int64_t boff = cell_boff[c];
  const int b0 = cell_start[c] + nint;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    V acc = czero<V>();
    const V* icol = Ibd + boff + b;
    for (int t = 0; t < F; ++t) acc = cfma(icol[t * nband], f[t], acc);
    int64_t j = b0 + b;
    vr[j] = cadd(ur[j], cscale(acc, k2));
  }
}

// Dirichlet fit on the matrix cores (q = 12: F = 48 face values, 64 slots):
// D [16 x 16] = FV [16 x F] IshT [F x slots 16 w .. 16 w + 15] for wave w,
// FV from LDS (row = lane % 16, face values 4 kk + lane / 16), IshT from
// global memory (16 consecutive slots per group).  Single precision: complex
// products as three real products (Gauss), else four.  Shared by the
// per-cell and the per-right-hand-side launches, so both give bitwise the
// same values.
template <typename T>
__device__ __forceinline__ void fit_mfma(const typename C2<T>::t* fv, const typename C2<T>::t* __restrict__ IshT,
                                         int wave, int kl, int col, typename Mfma<T>::v4& dre,
                                         typename Mfma<T>::v4& dim) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int F = 48, S = 64;
  constexpr bool G3 = std::is_same<T, float>::value;
  v4 p3 = v4{0, 0, 0, 0};
  dre = v4{0, 0, 0, 0};
  dim = v4{0, 0, 0, 0};
#pragma unroll 4
  for (int kk = 0; kk < F / 4; ++kk) {
    const int t = 4 * kk + kl;
    const V x = fv[col * F + t];
    const V w = IshT[t * S + 16 * wave + col];
    if (G3) {
      dre = M::op(x.x + x.y, w.x, dre);
      dim = M::op(x.y, w.x + w.y, dim);
      p3 = M::op(x.x, w.y - w.x, p3);
    } else {
      dre = M::op(x.x, w.x, dre);
      dre = M::op(-x.y, w.y, dre);
      dim = M::op(x.x, w.y, dim);
      dim = M::op(x.y, w.x, dim);
    }
  }
  if (G3) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T p1 = dre[q];
      dre[q] = p1 - dim[q];
      dim[q] = p1 + p3[q];
    }
  }
}

// Interpolation for 16 consecutive cells per workgroup (q = 12: F = 48 face
// values, S = 64 slots) on the matrix cores: the cells' face values are
// staged in LDS and fitted to the slots as one contraction (fit_mfma; wave
// w takes slots 16w..16w+15), and to the band nodes
// one row per thread (IbdT [F][nband]).  The adjacent cells' part of the lattice field is
// removed by the near-field weights (folded in at set-up), not here.
template <typename T, int CB>
__global__ void __launch_bounds__(256) k_interp_mfma(const typename C2<T>::t* __restrict__ u,
                                                     typename C2<T>::t* __restrict__ v,
                                                     const typename C2<T>::t* __restrict__ lat,
                                                     const typename C2<T>::t* __restrict__ IshT,
                                                     const typename C2<T>::t* __restrict__ Ibd,
                                                     const int32_t* __restrict__ cell_xy,
                                                     const int32_t* __restrict__ slot_map,
                                                     const int32_t* __restrict__ cell_start,
                                                     const int32_t* __restrict__ cell_nint,
                                                     const int32_t* __restrict__ cell_nb,
                                                     const int32_t* __restrict__ cell_boff, int ncell, int Pa, int Pb,
                                                     int64_t N, int64_t nband, T k2) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int q = 12, F = 4 * q, S = 64;
  static_assert(CB == 16, "one MFMA row per cell");
  extern __shared__ unsigned char smem_raw[];
  V* fv = reinterpret_cast<V*>(smem_raw);                    // [CB][F] face values
  int* cinfo = reinterpret_cast<int*>(fv + CB * F);          // [CB][2] cell x, y (-1: past the end)
  const int c0 = blockIdx.x * CB, r = blockIdx.y, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, kl = lane >> 4, col = lane & 15;
  const int64_t plane = (int64_t)Pa * Pb;
  if (tid < CB) {
    const int c = c0 + tid;
    cinfo[2 * tid] = c < ncell ? cell_xy[2 * c] : -1;
    cinfo[2 * tid + 1] = c < ncell ? cell_xy[2 * c + 1] : -1;
  }
  __syncthreads();
  for (int i = tid; i < CB * F; i += blockDim.x) {
    const int cb = i / F, t = i % F;
    const int cx = cinfo[2 * cb], cy = cinfo[2 * cb + 1];
    V val = czero<V>();
    if (cx >= 0) {
      const int s2 = t / (2 * q), fj = t % (2 * q), fc = fj / q, j = fj % q;
      const int cn = (s2 == 0 ? cx : cy) + fc, ct = (s2 == 0 ? cy : cx);
      val = lat[((int64_t)(r * 2 + s2) * 2) * plane + (int64_t)cn * Pb + ct * q + j];
    }
    fv[i] = val;
  }
  __syncthreads();
  const V* ur = u + (int64_t)r * N;
  V* vr = v + (int64_t)r * N;
  {
    // fit = FV [cells x F] IshT [F x slots]: output element (cell, slot),
    // the 16 lanes of a group on 16 consecutive slots of one cell
    v4 dre, dim;
    fit_mfma<T>(fv, IshT, wave, kl, col, dre, dim);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int c = c0 + M::row(lane, rr);
      if (c >= ncell) continue;
      const int j = slot_map[(int64_t)c * S + 16 * wave + col];
      if (j >= 0) {
        V o2;
        o2.x = dre[rr];
        o2.y = dim[rr];
        vr[j] = cadd(ur[j], cscale(o2, k2));
      }
    }
  }
  const int cl = min(c0 + CB, ncell) - 1;
  const int64_t bb = cell_boff[c0], be = (int64_t)cell_boff[cl] + cell_nb[cl];
  for (int64_t ib = bb + tid; ib < be; ib += blockDim.x) {
    int cb = 0;
    while (c0 + cb + 1 <= cl && cell_boff[c0 + cb + 1] <= ib) ++cb;
    const int c = c0 + cb;
    const V* icol = Ibd + ib;     // IbdT [F][nband]: lanes read consecutive words
    V s1 = czero<V>();
#pragma unroll 8
    for (int t = 0; t < F; ++t) s1 = cfma(icol[t * nband], fv[cb * F + t], s1);
    const int64_t j = cell_start[c] + cell_nint[c] + (ib - cell_boff[c]);
    vr[j] = cadd(ur[j], cscale(s1, k2));
  }
}

// The same interpolation for 16 right-hand sides of one cell per workgroup
// (batched applies): the MFMA rows are the 16 right-hand sides instead of
// 16 cells, and each band node's fit row is read once for all of them.  Every
// output goes through the same products in the same order as in
// k_interp_mfma, so results are bitwise those of the per-right-hand-side
// launch.
template <typename T>
__global__ void __launch_bounds__(256) k_interp_rb(const typename C2<T>::t* __restrict__ u,
                                                   typename C2<T>::t* __restrict__ v,
                                                   const typename C2<T>::t* __restrict__ lat,
                                                   const typename C2<T>::t* __restrict__ IshT,
                                                   const typename C2<T>::t* __restrict__ Ibd,
                                                   const int32_t* __restrict__ cell_xy,
                                                   const int32_t* __restrict__ slot_map,
                                                   const int32_t* __restrict__ cell_start,
                                                   const int32_t* __restrict__ cell_nint,
                                                   const int32_t* __restrict__ cell_nb,
                                                   const int32_t* __restrict__ cell_boff, int Pa, int Pb, int64_t N,
                                                   int64_t nband, int nrhs, T k2) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int q = 12, F = 4 * q, S = 64, RB = 16;
  __shared__ V fv[RB * F];   // [rhs][F] face values
  const int c = blockIdx.x, r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, kl = lane >> 4, col = lane & 15;
  const int64_t plane = (int64_t)Pa * Pb;
  const int cx = cell_xy[2 * c], cy = cell_xy[2 * c + 1];
  for (int i = tid; i < RB * F; i += blockDim.x) {
    const int qr = i / F, t = i % F, r = r0 + qr;
    V val = czero<V>();
    if (r < nrhs) {
      const int s2 = t / (2 * q), fj = t % (2 * q), fc = fj / q, j = fj % q;
      const int cn = (s2 == 0 ? cx : cy) + fc, ct = (s2 == 0 ? cy : cx);
      val = lat[((int64_t)(r * 2 + s2) * 2) * plane + (int64_t)cn * Pb + ct * q + j];
    }
    fv[i] = val;
  }
  __syncthreads();
  {
    // fit = FV [rhs x F] IshT [F x slots]: output element (rhs, slot), the
    // 16 lanes of a group on 16 consecutive slots of one right-hand side
    v4 dre, dim;
    fit_mfma<T>(fv, IshT, wave, kl, col, dre, dim);
    const int j = slot_map[(int64_t)c * S + 16 * wave + col];
    if (j >= 0) {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int r = r0 + M::row(lane, rr);
        if (r >= nrhs) continue;
        V o2;
        o2.x = dre[rr];
        o2.y = dim[rr];
        v[(int64_t)r * N + j] = cadd(u[(int64_t)r * N + j], cscale(o2, k2));
      }
    }
  }
  const int nb = cell_nb[c];
  const int64_t boff = cell_boff[c], b0 = cell_start[c] + cell_nint[c];
  const int nr = min(RB, nrhs - r0);
  for (int b = tid; b < nb; b += blockDim.x) {
    const V* icol = Ibd + boff + b;     // IbdT [F][nband]
    V s1[RB];
#pragma unroll
    for (int qr = 0; qr < RB; ++qr) s1[qr] = czero<V>();
    for (int t = 0; t < F; ++t) {
      const V w = icol[t * nband];
#pragma unroll
      for (int qr = 0; qr < RB; ++qr) s1[qr] = cfma(w, fv[qr * F + t], s1[qr]);
    }
    const int64_t j = b0 + b;
#pragma unroll
    for (int qr = 0; qr < RB; ++qr)
      if (qr < nr) v[(int64_t)(r0 + qr) * N + j] = cadd(u[(int64_t)(r0 + qr) * N + j], cscale(s1[qr], k2));
  }
}

// ---------------------------------------------------------------------------
// a4, interior x interior: out[a][cell] += sum_b W[a][b] psi[b][cell] over
// the 5x5-cell window (translation invariant weights).  Tiled: a workgroup
// takes CT cells; W and psi chunks staged in LDS.
// ---------------------------------------------------------------------------
template <typename T, int CT, int KC>
__global__ void __launch_bounds__(256) k_near_shared(const typename C2<T>::t* __restrict__ u,
                                                     typename C2<T>::t* __restrict__ v,
                                                     const typename C2<T>::t* __restrict__ W,
                                                     const T* __restrict__ dw,
                                                     const int32_t* __restrict__ icells,
                                                     const int32_t* __restrict__ cell_xy,
                                                     const int32_t* __restrict__ cell_map,
                                                     const int32_t* __restrict__ slot_map, int L, int ch,
                                                     int S, int nicell, int64_t N, T k2) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* Ws = reinterpret_cast<V*>(smem_raw);            // S x KC
  V* Xs = Ws + S * KC;                               // KC x CT
  int* wc = reinterpret_cast<int*>(Xs + KC * CT);    // 25 x CT window cell ids
  const int Wn = 5 * ch, K = Wn * Wn;
  const int r = blockIdx.y;
  const int cbase = blockIdx.x * CT;
  const V* ur = u + (int64_t)r * N;
  for (int i = threadIdx.x; i < 25 * CT; i += blockDim.x) {
    int cc = i / 25, o = i % 25;
    int cid = cbase + cc < nicell ? icells[cbase + cc] : -1;
    int res = -1;
    if (cid >= 0) {
      int nx = cell_xy[2 * cid] + o % 5 - 2, ny = cell_xy[2 * cid + 1] + o / 5 - 2;
      if (nx >= 0 && ny >= 0 && nx < L && ny < L) res = cell_map[ny * L + nx];
    }
    wc[cc * 25 + o] = res;
  }
  // each thread owns outputs (a, cc) for a = tid % S + k*?  -> S*CT / 256 outputs
  constexpr int MAXO = 8;
  const int nout = (S * CT + blockDim.x - 1) / blockDim.x;
  V acc[MAXO];
  for (int k = 0; k < MAXO; ++k) acc[k] = czero<V>();
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += KC) {
    const int kc = min(KC, K - k0);
    for (int i = threadIdx.x; i < S * KC; i += blockDim.x) {
      int a = i / KC, kk = i % KC;
      Ws[i] = kk < kc ? W[(int64_t)a * K + k0 + kk] : czero<V>();
    }
    for (int i = threadIdx.x; i < KC * CT; i += blockDim.x) {
      int kk = i / CT, cc = i % CT;
      V val = czero<V>();
      if (kk < kc) {
        int b = k0 + kk;
        int wx = b % Wn, wy = b / Wn;
        int cn = wc[cc * 25 + (wy / ch) * 5 + (wx / ch)];
        if (cn >= 0) {
          int j = slot_map[(int64_t)cn * S + (wy % ch) * ch + (wx % ch)];
          if (j >= 0) val = cscale(ur[j], dw[j]);
        }
      }
      Xs[i] = val;
    }
    __syncthreads();
    for (int o = 0; o < nout && o < MAXO; ++o) {
      int id = threadIdx.x + o * blockDim.x;
      if (id >= S * CT) break;
      int a = id % S, cc = id / S;
      V s = acc[o];
      for (int kk = 0; kk < kc; ++kk) s = cfma(Ws[a * KC + kk], Xs[kk * CT + cc], s);
      acc[o] = s;
    }
    __syncthreads();
  }
  V* vr = v + (int64_t)r * N;
  for (int o = 0; o < nout && o < MAXO; ++o) {
    int id = threadIdx.x + o * blockDim.x;
    if (id >= S * CT) break;
    int a = id % S, cc = id / S;
    if (cbase + cc >= nicell) continue;
    int cid = icells[cbase + cc];
    int j = slot_map[(int64_t)cid * S + a];
    if (j < 0) continue;
    V t = vr[j];
    vr[j] = cadd(t, cscale(acc[o], k2));
  }
}

// a4, interior x interior on matrix cores.  The interior density
// psi = m omega u is first laid out on the lattice (two empty cells of
// padding on each side), so that the 5x5-cell window of a cell is a plain
// 40 x 40 block of rows.  out[slot][cell] = sum_b W[slot][b] psi[b][cell]
// is then a dense contraction: a workgroup takes 16*NT cells, wave w the
// slots 16w..16w+15, K runs over the window row by row (W row and psi rows
// staged in LDS), complex products as four real MFMA 16x16x4 updates.
// The psi lattice of RB right-hand sides per thread (the node of a lattice
// point is looked up once for all of them).
template <typename T, int RB>
__global__ void k_psi_grid(const typename C2<T>::t* __restrict__ u, typename C2<T>::t* __restrict__ grid,
                           const T* __restrict__ dw, const int32_t* __restrict__ cell_map,
                           const int32_t* __restrict__ slot_map, int L, int ch, int S, int Gw, int64_t N,
                           int nrhs) {
  using V = typename C2<T>::t;
  const int64_t gsz = (int64_t)Gw * Gw;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= gsz) return;
  const int r0 = blockIdx.y * RB;
  const int gy = (int)(idx / Gw), gx = (int)(idx % Gw);
  const int cx = gx / ch - 2, cy = gy / ch - 2;
  int j = -1;
  if (cx >= 0 && cy >= 0 && cx < L && cy < L) {
    const int c = cell_map[cy * L + cx];
    if (c >= 0) j = slot_map[(int64_t)c * S + (gy % ch) * ch + (gx % ch)];
  }
  const T w = j >= 0 ? dw[j] : (T)0;
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int r = r0 + q;
    if (r >= nrhs) break;
    grid[(int64_t)r * gsz + idx] = j >= 0 ? cscale(u[(int64_t)r * N + j], w) : czero<V>();
  }
}


template <typename T, int NT>
__global__ void __launch_bounds__(256) k_near_shared_mfma(const typename C2<T>::t* __restrict__ grid,
                                                          typename C2<T>::t* __restrict__ v,
                                                          const typename C2<T>::t* __restrict__ W,
                                                          const int32_t* __restrict__ icells,
                                                          const int32_t* __restrict__ cell_xy,
                                                          const int32_t* __restrict__ slot_map, int Gw,
                                                          int nicell, int64_t N, T k2, int64_t gstride) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  using v4 = typename M::v4;
  constexpr int CH = 8, S = 64, WN = 40, KP = WN + 1, NC = 16 * NT;
  __shared__ V Xs[NC * KP];
  __shared__ V Ws[S * KP];
  __shared__ int cx0[NC], cy0[NC];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r = blockIdx.y;
  const int cb = blockIdx.x * NC;
  const V* g = grid + (int64_t)r * gstride;
  for (int c = tid; c < NC; c += blockDim.x) {
    int cid = cb + c < nicell ? icells[cb + c] : -1;
    cx0[c] = cid >= 0 ? cell_xy[2 * cid] * CH : -1;
    cy0[c] = cid >= 0 ? cell_xy[2 * cid + 1] * CH : -1;
  }
  v4 acc_re[NT], acc_im[NT];
  for (int t = 0; t < NT; ++t) {
    acc_re[t] = v4{0, 0, 0, 0};
    acc_im[t] = v4{0, 0, 0, 0};
  }
  for (int wy = 0; wy < WN; ++wy) {
    __syncthreads();
    for (int i = tid; i < NC * WN; i += blockDim.x) {
      int c = i / WN, wx = i % WN;
      V val = czero<V>();
      if (cx0[c] >= 0) val = g[(int64_t)(cy0[c] + wy) * Gw + cx0[c] + wx];
      Xs[c * KP + wx] = val;
    }
    for (int i = tid; i < S * WN; i += blockDim.x) {
      int a = i / WN, wx = i % WN;
      Ws[a * KP + wx] = W[(int64_t)a * WN * WN + wy * WN + wx];
    }
    __syncthreads();
#pragma unroll 2
    for (int kk = 0; kk < WN / 4; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      const V wa = Ws[(16 * wave + (lane & 15)) * KP + k];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const V xb = Xs[(16 * t + (lane & 15)) * KP + k];
        acc_re[t] = M::op(wa.x, xb.x, acc_re[t]);
        acc_re[t] = M::op(-wa.y, xb.y, acc_re[t]);
        acc_im[t] = M::op(wa.x, xb.y, acc_im[t]);
        acc_im[t] = M::op(wa.y, xb.x, acc_im[t]);
      }
    }
  }
  V* vr = v + (int64_t)r * N;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = cb + 16 * t + (lane & 15);
    if (c >= nicell) continue;
    const int cid = icells[c];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = 16 * wave + M::row(lane, q);
      const int j = slot_map[(int64_t)cid * S + a];
      if (j < 0) continue;
      V o = vr[j];
      o.x += k2 * acc_re[t][q];
      o.y += k2 * acc_im[t][q];
      vr[j] = o;
    }
  }
}

// Single-precision form of the window contraction above with the staging
// double-buffered: while the MFMAs contract window row wy from one LDS
// buffer, the loads of row wy+1 are in flight in registers and land in the
// other buffer, so each row costs one barrier and no exposed load latency.
// A workgroup of 4 CT waves takes 16 CT cells: wave w contracts slots
// 16 (w % 4) .. +15 against cells 16 (w / 4) .. +15, so one staged row of W
// serves 16 CT cells (CT = 1: most workgroups, CT = 4: least W traffic).
template <int CT, bool G3 = false>
__global__ void __launch_bounds__(256 * CT) k_near_shared_mfma_db(const float2* __restrict__ grid,
                                                                  float2* __restrict__ v,
                                                                  const float2* __restrict__ W,
                                                                  const int32_t* __restrict__ icells,
                                                                  const int32_t* __restrict__ cell_xy,
                                                                  const int32_t* __restrict__ slot_map, int Gw,
                                                                  int nicell, int64_t N, float k2, int64_t gstride) {
  using M = Mfma<float>;
  using v4 = M::v4;
  constexpr int CH = 8, S = 64, WN = 40, KP = WN + 1, NC = 16 * CT, NTH = 256 * CT;
  constexpr int XPT = (NC * WN + NTH - 1) / NTH, WPT = (S * WN + NTH - 1) / NTH;
  __shared__ float2 Xs[2][NC * KP];
  __shared__ float2 Ws[2][S * KP];
  __shared__ int cx0[NC], cy0[NC];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int st = wave & 3, ct = wave >> 2;     // slot tile, cell tile
  const int r = blockIdx.y;
  const int cb = blockIdx.x * NC;
  const float2* g = grid + (int64_t)r * gstride;   // (grid stride Gw, gstride per right-hand side)
  if (tid < NC) {
    const int cid = cb + tid < nicell ? icells[cb + tid] : -1;
    cx0[tid] = cid >= 0 ? cell_xy[2 * cid] * CH : -1;
    cy0[tid] = cid >= 0 ? cell_xy[2 * cid + 1] * CH : -1;
  }
  __syncthreads();
  float2 xr[XPT], wr[WPT];
  auto gload = [&](int wy) {
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int i = tid + NTH * q;
      float2 val = make_float2(0.f, 0.f);
      if (i < NC * WN) {
        const int c = i / WN, wx = i % WN;
        if (cx0[c] >= 0) val = g[(int64_t)(cy0[c] + wy) * Gw + cx0[c] + wx];
      }
      xr[q] = val;
    }
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int i = tid + NTH * q;
      if (i < S * WN) wr[q] = W[(int64_t)(i / WN) * WN * WN + wy * WN + i % WN];
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int q = 0; q < XPT; ++q) {
      const int i = tid + NTH * q;
      if (i < NC * WN) Xs[b][(i / WN) * KP + i % WN] = xr[q];
    }
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int i = tid + NTH * q;
      if (i < S * WN) Ws[b][(i / WN) * KP + i % WN] = wr[q];
    }
  };
  // G3: complex products as three real products (Gauss): with
  // p1 = Wr (Xr + Xi), p2 = (Wr + Wi) Xi, p3 = (Wi - Wr) Xr the result is
  // p1 - p2 + i (p1 + p3); else the four real products
  v4 are = v4{0, 0, 0, 0}, aim = v4{0, 0, 0, 0}, a3 = v4{0, 0, 0, 0};
  gload(0);
  sstore(0);
  __syncthreads();
  for (int wy = 0; wy < WN; ++wy) {
    const int b = wy & 1;
    if (wy + 1 < WN) gload(wy + 1);
#pragma unroll 2
    for (int kk = 0; kk < WN / 4; ++kk) {
      const int k = 4 * kk + (lane >> 4);
      const float2 wa = Ws[b][(16 * st + (lane & 15)) * KP + k];
      const float2 xb = Xs[b][(16 * ct + (lane & 15)) * KP + k];
      if (G3) {
        are = M::op(wa.x, xb.x + xb.y, are);
        aim = M::op(wa.x + wa.y, xb.y, aim);
        a3 = M::op(wa.y - wa.x, xb.x, a3);
      } else {
        are = M::op(wa.x, xb.x, are);
        are = M::op(-wa.y, xb.y, are);
        aim = M::op(wa.x, xb.y, aim);
        aim = M::op(wa.y, xb.x, aim);
      }
    }
    if (wy + 1 < WN) sstore(b ^ 1);
    __syncthreads();
  }
  if (G3) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float p1 = are[q];
      are[q] = p1 - aim[q];
      aim[q] = p1 + a3[q];
    }
  }
  const int c = cb + 16 * ct + (lane & 15);
  if (c >= nicell) return;
  const int cid = icells[c];
  float2* vr = v + (int64_t)r * N;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = 16 * st + M::row(lane, q);
    const int j = slot_map[(int64_t)cid * S + a];
    if (j < 0) continue;
    float2 o = vr[j];
    o.x += k2 * are[q];
    o.y += k2 * aim[q];
    vr[j] = o;
  }
}

// (Row kernels: input right-hand side r at u + r ldu, ldu = N, or the
// length of x = [u ; refined band values] with Fourier refinement; output
// right-hand side r at v + r N.)
// Single-precision rows touching the boundary patch with 16-bit column
// offsets, rows stored padded to a multiple of four entries (zero weights,
// offset 0): each lane takes four consecutive entries per step (one 32-byte
// weight load and one 8-byte offset load), each weight applied to up to four
// right-hand sides.
__global__ void __launch_bounds__(256) k_near_csr4(const float2* __restrict__ u, float2* __restrict__ v,
                                                   const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ colbase,
                                                   const uint16_t* __restrict__ coloff,
                                                   const float2* __restrict__ vals, int nrows, int64_t N, int nrhs,
                                                   float k2, int64_t ldu) {
  constexpr int RB = 4;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= nrows) return;
  const int64_t b = rowptr[row] >> 2, e = rowptr[row + 1] >> 2;
  const float2* __restrict__ ub = u + colbase[row];
  const float4* __restrict__ v4 = (const float4*)vals;
  const uint2* __restrict__ o4 = (const uint2*)coloff;
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    const int nr = min(RB, nrhs - r0);
    float2 acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = czero<float2>();
    for (int64_t k = b + lane; k < e; k += 64) {
      const float4 wa = v4[2 * k], wb = v4[2 * k + 1];
      const uint2 cc = o4[k];
      const int c0 = cc.x & 0xffff, c1 = cc.x >> 16, c2 = cc.y & 0xffff, c3 = cc.y >> 16;
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        if (q < nr) {
          const float2* uq = ub + (int64_t)(r0 + q) * ldu;
          acc[q] = cfma(make_float2(wa.x, wa.y), uq[c0], acc[q]);
          acc[q] = cfma(make_float2(wa.z, wa.w), uq[c1], acc[q]);
          acc[q] = cfma(make_float2(wb.x, wb.y), uq[c2], acc[q]);
          acc[q] = cfma(make_float2(wb.z, wb.w), uq[c3], acc[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      if (q >= nr) break;
      float2 a = acc[q];
      for (int off = 32; off > 0; off >>= 1) {
        a.x += __shfl_down(a.x, off, 64);
        a.y += __shfl_down(a.y, off, 64);
      }
      if (lane == 0) {
        const int64_t j = rows[row];
        float2* vr = v + (int64_t)(r0 + q) * N;
        float2 t = vr[j];
        vr[j] = cadd(t, cscale(a, k2));
      }
    }
  }
}

// Single-precision rows touching the boundary patch, columns stored as runs
// of consecutive operator indices (the nodes are sorted by cell, so a row is
// a few dozen runs): run r of a row covers its entries [pre[r], pre[r+1]) at
// columns cs[r], cs[r]+1, ...  One wavefront per row stages the row's run
// table in LDS; each lane finds the run of its four consecutive entries by
// bisection.  Weights as in k_near_csr4 (rows padded to four entries; the
// padding sits in a final run at column 0 with zero weights).  The tables
// take dynamic LDS, 4 (2 rmax + 1) words per workgroup for rows of at most
// rmax runs (the operator's largest).
__global__ void __launch_bounds__(256) k_near_csr4r(const float2* __restrict__ u, float2* __restrict__ v,
                                                    const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ rows,
                                                    const int32_t* __restrict__ run_ptr,
                                                    const int32_t* __restrict__ run_cs,
                                                    const int32_t* __restrict__ run_pre,
                                                    const float2* __restrict__ vals, int nrows, int64_t N, int nrhs,
                                                    float k2, int rmax, int64_t ldu) {
  constexpr int RB = 4;
  extern __shared__ int tables[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wv;
  if (row >= nrows) return;
  const int64_t b = rowptr[row], e = rowptr[row + 1];
  const int len = (int)(e - b);
  const int r0 = run_ptr[row], nr = run_ptr[row + 1] - r0;
  int* cs = tables + wv * (2 * rmax + 1);
  int* pre = cs + rmax;
  for (int i = lane; i < nr; i += 64) {
    cs[i] = run_cs[r0 + i];
    pre[i] = run_pre[r0 + i];
  }
  if (lane == 0) pre[nr] = len;
  // each wave reads only its own row's table: a wavefront-scope barrier
  // (release / acquire on LDS) is enough, the other rows do not wait
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float4* __restrict__ v4 = (const float4*)(vals + b);
  for (int r00 = 0; r00 < nrhs; r00 += RB) {
    const int nrr = min(RB, nrhs - r00);
    float2 acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = czero<float2>();
    for (int k = lane; 4 * k < len; k += 64) {
      const float4 wa = v4[2 * k], wb = v4[2 * k + 1];
      const int e0 = 4 * k;
      int lo = 0, hi = nr;          // largest r with pre[r] <= e0
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= e0) lo = mid; else hi = mid;
      }
      int c[4];
      int rr = lo;
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        while (pre[rr + 1] <= e0 + z) ++rr;
        c[z] = cs[rr] + (e0 + z - pre[rr]);
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        if (q < nrr) {
          const float2* uq = u + (int64_t)(r00 + q) * ldu;
          acc[q] = cfma(make_float2(wa.x, wa.y), uq[c[0]], acc[q]);
          acc[q] = cfma(make_float2(wa.z, wa.w), uq[c[1]], acc[q]);
          acc[q] = cfma(make_float2(wb.x, wb.y), uq[c[2]], acc[q]);
          acc[q] = cfma(make_float2(wb.z, wb.w), uq[c[3]], acc[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      if (q >= nrr) break;
      float2 a = acc[q];
      for (int off = 32; off > 0; off >>= 1) {
        a.x += __shfl_down(a.x, off, 64);
        a.y += __shfl_down(a.y, off, 64);
      }
      if (lane == 0) {
        const int64_t j = rows[row];
        float2* vr = v + (int64_t)(r00 + q) * N;
        float2 t = vr[j];
        vr[j] = cadd(t, cscale(a, k2));
      }
    }
  }
}

// Set-up: folds the adjacent far-field subtraction into the rows touching
// the boundary patch.  The far field at target i of cell c leaves out the
// equivalent sources of the 3 x 3 adjacent cells, i.e. it carries
// -I_i T_off P_j c_j u_j for every source j of the adjacent cell c + off
// (P_j: j's projection column, I_i: i's fit row).  The rows of boundary-patch
// targets hold every point of those cells, the rows of interior targets
// every boundary-patch point, so the term is added to the stored weights
// (once per precision, with that precision's projection; the far-field
// stage then skips it).  One workgroup per row: g_off = I_i T_off for the 9
// offsets in LDS, then one dot of length U per entry.
__global__ void __launch_bounds__(256) k_fold_rows(const int64_t* __restrict__ rowptr,
                                                   const int64_t* __restrict__ olen,
                                                   const int32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ colbase,
                                                   const uint16_t* __restrict__ coloff,
                                                   const int32_t* __restrict__ cols32,
                                                   const int32_t* __restrict__ pt_cell,
                                                   const int32_t* __restrict__ pt_idx,
                                                   const int32_t* __restrict__ cell_xy,
                                                   const double2* __restrict__ IshT, const double2* __restrict__ IbdT,
                                                   const double2* __restrict__ ToffT,
                                                   const double2* __restrict__ PshT64,
                                                   const float2* __restrict__ PshT32,
                                                   const double2* __restrict__ Pbd64,
                                                   const float2* __restrict__ Pbd32, const double* __restrict__ cw,
                                                   double2* __restrict__ vals64, float2* __restrict__ vals32,
                                                   int F, int U, int S, int64_t nband) {
  extern __shared__ unsigned char smem_raw[];
  double2* I = reinterpret_cast<double2*>(smem_raw);   // [F]
  double2* g = I + F;                                  // [9][U]
  const int r = blockIdx.x;
  const int i = rows[r], c = pt_cell[i], idx = pt_idx[i];
  const bool tb = idx < 0;
  const int cx = cell_xy[2 * c], cy = cell_xy[2 * c + 1];
  for (int t = threadIdx.x; t < F; t += blockDim.x)
    I[t] = tb ? IbdT[(int64_t)t * nband + (-idx - 1)] : IshT[(int64_t)t * S + idx];
  __syncthreads();
  for (int e = threadIdx.x; e < 9 * U; e += blockDim.x) {
    const double2* Tr = ToffT + (int64_t)e * F;   // [o][u][t]
    double2 acc = make_double2(0.0, 0.0);
    for (int t = 0; t < F; ++t) acc = cfma(I[t], Tr[t], acc);
    g[e] = acc;
  }
  __syncthreads();
  const int64_t b0 = rowptr[r], len = olen[r];
  for (int64_t k = threadIdx.x; k < len; k += blockDim.x) {
    const int32_t j = colbase[r] + (coloff ? (int32_t)coloff[b0 + k] : cols32[b0 + k]);
    const int cj = pt_cell[j];
    const int dx = cell_xy[2 * cj] - cx, dy = cell_xy[2 * cj + 1] - cy;
    if (dx < -1 || dx > 1 || dy < -1 || dy > 1) continue;
    const int jdx = pt_idx[j];
    const bool jb = jdx < 0;
    if (!tb && !jb) continue;      // interior to interior: in the shared window
    const double2* go = g + ((dy + 1) * 3 + dx + 1) * U;
    const double2* p64 = jb ? Pbd64 + (int64_t)(-jdx - 1) * U : PshT64 + (int64_t)jdx * U;
    const float2* p32 = jb ? Pbd32 + (int64_t)(-jdx - 1) * U : PshT32 + (int64_t)jdx * U;
    double2 a64 = make_double2(0.0, 0.0), a32 = make_double2(0.0, 0.0);
    for (int u2 = 0; u2 < U; ++u2) {
      a64 = cfma(go[u2], p64[u2], a64);
      const float2 pf = p32[u2];
      a32 = cfma(go[u2], make_double2(pf.x, pf.y), a32);
    }
    const double w = cw[j];
    const double2 base = vals64[b0 + k];
    vals32[b0 + k] = make_float2((float)(base.x - w * a32.x), (float)(base.y - w * a32.y));
    vals64[b0 + k] = make_double2(base.x - w * a64.x, base.y - w * a64.y);
  }
}

hipError_t launch_fold_rows(const DevView<double>& a, const DevView<float>& b, const int64_t* olen,
                            const int32_t* pt_cell, const int32_t* pt_idx, hipStream_t st) {
  if (a.nrows == 0) return hipSuccess;
  const size_t sh = (size_t)(a.F + 9 * a.U) * sizeof(double2);
  hipLaunchKernelGGL(k_fold_rows, dim3(a.nrows), dim3(256), sh, st, a.rowptr, olen, a.rows, a.colbase, a.coloff,
                     a.cols32, pt_cell, pt_idx, a.cell_xy, (const double2*)a.Ish, (const double2*)a.Ibd,
                     (const double2*)a.Toff, (const double2*)a.PshT, (const float2*)b.PshT, (const double2*)a.Pbd,
                     (const float2*)b.Pbd, a.cw, (double2*)a.vals, (float2*)b.vals, a.F, a.U, a.S, a.nband);
  return hipGetLastError();
}

// Right-hand-side-major copy for the batched row kernel: ut[i * R + r] = u[r * N + i]
// (32 x 32 tiles through LDS, both sides coalesced).
template <typename V>
__global__ void __launch_bounds__(256) k_rhs_major(const V* __restrict__ u, V* __restrict__ ut, int64_t N, int R) {
  __shared__ V tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k;
    const int64_t i = i0 + tx;
    tile[k][tx] = (r < R && i < N) ? u[(int64_t)r * N + i] : czero<V>();
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t i = i0 + k;
    const int r = r0 + tx;
    if (i < N && r < R) ut[i * R + r] = tile[tx][k];
  }
}

// a4 on the matrix cores, dense tiles of 16 rows (single or double
// precision, R a multiple of 16 right-hand sides, input right-hand-side-major).  One
// wavefront per (16-row tile, 16 NT right-hand sides) computes the tile's
// product as V^T = U^T W^T: MFMA A operand = 16 right-hand sides x 4 columns
// of the input (row = lane % 16, column k = lane / 16: 16 consecutive words
// per column), B operand = 4 columns x 16 target rows of the tile's weights
// (stored so that a step reads 64 consecutive values), complex products as
// four real products.  Output element (right-hand side 4 (lane / 16) + r,
// target lane % 16): the 16 lanes of a group add into 16 targets of one
// right-hand side.  Rows of different tiles are distinct, so the adds do not
// race.
template <typename T, int NT, bool G3 = false>
__global__ void __launch_bounds__(256) k_near_blk(const typename C2<T>::t* __restrict__ ut,
                                                  typename C2<T>::t* __restrict__ v,
                                                  const int32_t* __restrict__ bt_rows,
                                                  const int32_t* __restrict__ bt_info,
                                                  const int64_t* __restrict__ bt_woff,
                                                  const int32_t* __restrict__ bt_cols,
                                                  const typename C2<T>::t* __restrict__ bt_w, int ntiles, int64_t N,
                                                  int R, T k2) {
  using V = typename C2<T>::t;
  using M = Mfma<T>;
  typedef typename M::v4 v4;
  const int lane = threadIdx.x & 63;
  const int nch = (R + 16 * NT - 1) / (16 * NT);
  const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t t = gw / nch;
  if (t >= ntiles) return;
  const int n0 = (int)(gw % nch) * 16 * NT;
  const int ntv = min(NT, (R - n0) / 16);
  const int K = bt_info[2 * t];
  const V* __restrict__ W = bt_w + bt_woff[t] + lane;
  const int32_t* __restrict__ cl = bt_cols + bt_info[2 * t + 1];
  const V* __restrict__ ub = ut + n0 + (lane & 15);
  v4 re[NT], im[NT], r3[G3 ? NT : 1];
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    re[g] = v4{0, 0, 0, 0};
    im[g] = v4{0, 0, 0, 0};
    if (G3) r3[g] = v4{0, 0, 0, 0};
  }
  // the tile's columns 64 at a time, one per lane; step s (4 columns) takes
  // its column from lane 4 (s % 16) + lane / 16.  Operands of step s + 1 are
  // loaded before the products of step s.
  const int nsteps = K / 4;
  int colreg = cl[min(lane, K - 1)];
  V wn = W[0], an[NT];
  {
    const V* __restrict__ uc = ub + (int64_t)__shfl(colreg, lane >> 4, 64) * R;
#pragma unroll
    for (int g = 0; g < NT; ++g) an[g] = g < ntv ? uc[16 * g] : czero<V>();
  }
  for (int s = 0; s < nsteps; ++s) {
    const V w = wn;
    V a[NT];
#pragma unroll
    for (int g = 0; g < NT; ++g) a[g] = an[g];
    const int s1 = s + 1;
    if (s1 < nsteps) {
      if ((s1 & 15) == 0) colreg = cl[min(4 * s1 + lane, K - 1)];
      wn = W[(int64_t)s1 * 64];
      const V* __restrict__ uc = ub + (int64_t)__shfl(colreg, 4 * (s1 & 15) + (lane >> 4), 64) * R;
#pragma unroll
      for (int g = 0; g < NT; ++g) an[g] = g < ntv ? uc[16 * g] : czero<V>();
    }
    if (G3) {
      // three real products (Gauss): p1 = (Ur + Ui) Wr, p2 = Ui (Wr + Wi),
      // p3 = Ur (Wi - Wr); real part p1 - p2, imaginary part p1 + p3
      const T ws = w.x + w.y, wd = w.y - w.x;
#pragma unroll
      for (int g = 0; g < NT; ++g) {
        re[g] = M::op(a[g].x + a[g].y, w.x, re[g]);
        im[g] = M::op(a[g].y, ws, im[g]);
        r3[g] = M::op(a[g].x, wd, r3[g]);
      }
    } else {
#pragma unroll
      for (int g = 0; g < NT; ++g) {
        re[g] = M::op(a[g].x, w.x, re[g]);
        re[g] = M::op(-a[g].y, w.y, re[g]);
        im[g] = M::op(a[g].x, w.y, im[g]);
        im[g] = M::op(a[g].y, w.x, im[g]);
      }
    }
  }
  if (G3) {
#pragma unroll
    for (int g = 0; g < NT; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T p1 = re[g][r];
        re[g][r] = p1 - im[g][r];
        im[g][r] = p1 + r3[g][r];
      }
  }
  const int j = bt_rows[t * 16 + (lane & 15)];
  if (j < 0) return;
#pragma unroll
  for (int g = 0; g < NT; ++g) {
    if (g >= ntv) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      V* p = v + (int64_t)(n0 + 16 * g + M::row(lane, r)) * N + j;
      V x;
      x.x = re[g][r];
      x.y = im[g][r];
      *p = cadd(*p, cscale(x, k2));
    }
  }
}

// a4, rows touching the boundary patch: one wavefront per row; each weight
// is loaded once and applied to up to four right-hand sides; four entries
// per lane in flight.
template <typename T, typename VT, typename CT>
__global__ void __launch_bounds__(256) k_near_csr(const typename C2<T>::t* __restrict__ u,
                                                  typename C2<T>::t* __restrict__ v,
                                                  const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ rows,
                                                  const int32_t* __restrict__ colbase,
                                                  const CT* __restrict__ coloff, const VT* __restrict__ vals,
                                                  int nrows, int64_t N, int nrhs, T k2, int64_t ldu) {
  using V = typename C2<T>::t;
  constexpr int RB = 4;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= nrows) return;
  const int64_t b = rowptr[row], e = rowptr[row + 1];
  const int cb = colbase[row];
  const V* __restrict__ ub = u + cb;
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    const int nr = min(RB, nrhs - r0);
    V acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = czero<V>();
    int64_t k = b + lane;
    for (; k + 3 * 64 < e; k += 4 * 64) {
      VT w[4];
      int c[4];
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        w[z] = vals[k + z * 64];
        c[z] = coloff[k + z * 64];
      }
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        V ww;
        ww.x = (T)w[z].x;
        ww.y = (T)w[z].y;
#pragma unroll
        for (int q = 0; q < RB; ++q)
          if (q < nr) acc[q] = cfma(ww, ub[(int64_t)(r0 + q) * ldu + c[z]], acc[q]);
      }
    }
    for (; k < e; k += 64) {
      VT w = vals[k];
      int c = coloff[k];
      V ww;
      ww.x = (T)w.x;
      ww.y = (T)w.y;
#pragma unroll
      for (int q = 0; q < RB; ++q)
        if (q < nr) acc[q] = cfma(ww, ub[(int64_t)(r0 + q) * ldu + c], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      if (q >= nr) break;
      V a = acc[q];
      for (int off = 32; off > 0; off >>= 1) {
        a.x += __shfl_down(a.x, off, 64);
        a.y += __shfl_down(a.y, off, 64);
      }
      if (lane == 0) {
        int64_t j = rows[row];
        V* vr = v + (int64_t)(r0 + q) * N;
        V t = vr[j];
        vr[j] = cadd(t, cscale(a, k2));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// GMRES helpers (FP64): dots d[j][r] = <V_j r, w_r>, w -= sum_j h V_j, norms
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_dots(const double2* __restrict__ Vb, const double2* __restrict__ w,
                                              double2* __restrict__ partial, int nvec, int64_t N, int nrhs,
                                              int64_t vstride) {
  // grid.x: blocks over N; grid.y: rhs.  partial[(r * nvec + j) * gridDim.x + blockIdx.x]
  __shared__ double2 red[256];
  const int r = blockIdx.y;
  const double2* wr = w + (int64_t)r * N;
  for (int j = 0; j < nvec; ++j) {
    const double2* vj = Vb + j * vstride + (int64_t)r * N;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
      double2 a = vj[i], b = wr[i];
      acc.x += a.x * b.x + a.y * b.y;    // conj(a) b
      acc.y += a.x * b.y - a.y * b.x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        red[threadIdx.x].x += red[threadIdx.x + s].x;
        red[threadIdx.x].y += red[threadIdx.x + s].y;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[((int64_t)r * nvec + j) * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// Fused CGS steps.  For a block of basis vectors V_0..V_{n-1} (vstride
// apart) and the work vector w of each right-hand side:
//   mode 0:  d_j = <V_j, w>
//   mode 1:  w -= sum_j h_j V_j, then d_j = <V_j, w> (next CGS pass)
//   mode 2:  w -= sum_j h_j V_j, then d_0 = <w, w>
// Partial sums per workgroup go to partial[(r * nout + j) * gridDim.x + block].
constexpr int GM_JB = 8;
__global__ void __launch_bounds__(256) k_cgs(const double2* __restrict__ Vb, double2* __restrict__ w,
                                             const double2* __restrict__ h, double2* __restrict__ partial,
                                             int nvec, int64_t N, int64_t vstride, int mode) {
  __shared__ double red[2 * GM_JB][256];
  const int r = blockIdx.y;
  double2* wr = w + (int64_t)r * N;
  const double2* V0 = Vb + (int64_t)r * N;
  const int nout = mode == 2 ? 1 : nvec;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (mode != 0) {
    for (int64_t i = i0; i < N; i += stride) {
      double2 acc = wr[i];
      for (int j = 0; j < nvec; ++j) {
        double2 hj = h[r * nvec + j];
        double2 a = V0[j * vstride + i];
        acc.x -= hj.x * a.x - hj.y * a.y;
        acc.y -= hj.x * a.y + hj.y * a.x;
      }
      wr[i] = acc;
    }
  }
  for (int j0 = 0; j0 < nout; j0 += GM_JB) {
    double ax[GM_JB], ay[GM_JB];
#pragma unroll
    for (int q = 0; q < GM_JB; ++q) ax[q] = ay[q] = 0.0;
    for (int64_t i = i0; i < N; i += stride) {
      double2 b = wr[i];
      if (mode == 2) {
        ax[0] += b.x * b.x + b.y * b.y;
      } else {
#pragma unroll
        for (int q = 0; q < GM_JB; ++q) {
          if (j0 + q < nvec) {
            double2 a = V0[(j0 + q) * vstride + i];
            ax[q] += a.x * b.x + a.y * b.y;      // conj(a) b
            ay[q] += a.x * b.y - a.y * b.x;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < GM_JB; ++q) {
      red[2 * q][threadIdx.x] = ax[q];
      red[2 * q + 1][threadIdx.x] = ay[q];
    }
    __syncthreads();
    for (int sft = blockDim.x / 2; sft > 0; sft >>= 1) {
      if (threadIdx.x < sft)
#pragma unroll
        for (int q = 0; q < 2 * GM_JB; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + sft];
      __syncthreads();
    }
    if (threadIdx.x < GM_JB && j0 + threadIdx.x < nout)
      partial[((int64_t)r * nout + j0 + threadIdx.x) * gridDim.x + blockIdx.x] =
          make_double2(red[2 * threadIdx.x][0], red[2 * threadIdx.x + 1][0]);
    __syncthreads();
  }
}

// one workgroup per output: out[i] = sum_p partial[i * nparts + p]
__global__ void __launch_bounds__(256) k_reduce_partials(const double2* __restrict__ partial,
                                                         double2* __restrict__ out, int nparts, int count) {
  __shared__ double rx[256], ry[256];
  const int i = blockIdx.x;
  if (i >= count) return;
  double sx = 0.0, sy = 0.0;
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
    double2 v = partial[(int64_t)i * nparts + p];
    sx += v.x;
    sy += v.y;
  }
  rx[threadIdx.x] = sx;
  ry[threadIdx.x] = sy;
  __syncthreads();
  for (int s2 = blockDim.x / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) {
      rx[threadIdx.x] += rx[threadIdx.x + s2];
      ry[threadIdx.x] += ry[threadIdx.x + s2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = make_double2(rx[0], ry[0]);
}

__global__ void k_update(const double2* __restrict__ Vb, double2* __restrict__ w, const double2* __restrict__ h,
                         int nvec, int64_t N, int nrhs, int64_t vstride) {
  const int r = blockIdx.y;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double2 acc = w[(int64_t)r * N + i];
  for (int j = 0; j < nvec; ++j) {
    double2 hj = h[r * nvec + j];
    double2 a = Vb[j * vstride + (int64_t)r * N + i];
    acc.x -= hj.x * a.x - hj.y * a.y;
    acc.y -= hj.x * a.y + hj.y * a.x;
  }
  w[(int64_t)r * N + i] = acc;
}

__global__ void k_inv_norm(const double2* __restrict__ dd, double* __restrict__ s, int nrhs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double v = dd[r].x;
  s[r] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
}

__global__ void k_scale_copy(const double2* __restrict__ src, double2* __restrict__ dst, const double* __restrict__ s,
                             int64_t N) {
  const int r = blockIdx.y;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double f = s[r];
  double2 a = src[(int64_t)r * N + i];
  dst[(int64_t)r * N + i] = make_double2(a.x * f, a.y * f);
}

__global__ void k_axpy_combo(double2* __restrict__ x, const double2* __restrict__ Vb, const double2* __restrict__ y,
                             int nvec, int64_t N, int64_t vstride) {
  // x_r += sum_j y[r][j] V_j r
  const int r = blockIdx.y;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double2 acc = x[(int64_t)r * N + i];
  for (int j = 0; j < nvec; ++j) {
    double2 c = y[r * nvec + j];
    // a zero coefficient (a right-hand side the solver froze) leaves x as it
    // is even where its basis vector holds non-finite values
    if (c.x == 0.0 && c.y == 0.0) continue;
    double2 a = Vb[j * vstride + (int64_t)r * N + i];
    acc.x += c.x * a.x - c.y * a.y;
    acc.y += c.x * a.y + c.y * a.x;
  }
  x[(int64_t)r * N + i] = acc;
}

__global__ void k_sub(const double2* __restrict__ a, const double2* __restrict__ b, double2* __restrict__ out,
                      int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = make_double2(a[i].x - b[i].x, a[i].y - b[i].y);
}

__global__ void k_add(double2* __restrict__ x, const double2* __restrict__ e, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = make_double2(x[i].x + e[i].x, x[i].y + e[i].y);
}

__global__ void k_to_f32(const double2* __restrict__ a, float2* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

__global__ void k_to_f64(const float2* __restrict__ a, double2* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  b[i] = make_double2((double)a[i].x, (double)a[i].y);
}

// ---------------------------------------------------------------------------
// GMRES helpers with a single-precision Krylov basis (complex float vectors;
// every reduction is finished in double).  Partial sums per workgroup go to
// partial[(r * nv + j) * gridDim.x + block] and are folded by k_fold.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// d_j = <V_j, w> (conj(V_j) . w) for j < nv <= NV <= 32.  Each thread keeps
// its own partial sums; the workgroup reduces them by a transpose through LDS
// (16 basis vectors at a time) rather than by cross-lane shuffles.
// Element pair (2i, 2i+1) of a vector slice: one 16-byte access when the
// slice starts 16-byte aligned, else two 8-byte ones (same values, so the
// arithmetic, and the result, is the same either way).
__device__ __forceinline__ bool al16(const void* p) { return ((uintptr_t)p & 15) == 0; }
__device__ __forceinline__ float4 ld_pair(const float2* p, int64_t i, bool al) {
  if (al) return reinterpret_cast<const float4*>(p)[i];
  const float2 a = p[2 * i], b = p[2 * i + 1];
  return make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void st_pair(float2* p, int64_t i, bool al, float4 v) {
  if (al) {
    reinterpret_cast<float4*>(p)[i] = v;
  } else {
    p[2 * i] = make_float2(v.x, v.y);
    p[2 * i + 1] = make_float2(v.z, v.w);
  }
}

// Two complex values (an element pair) per lane and step, 16-byte accesses
// where the slice is aligned; an odd last element is taken by thread 0 of
// workgroup 0.
template <int NV>
__global__ void __launch_bounds__(256) k_dots32(const float2* __restrict__ Vb, const float2* __restrict__ w,
                                                double2* __restrict__ partial, int nv, int64_t N,
                                                int64_t vstride) {
  static_assert(NV <= 32, "at most 32 basis vectors per pass");
  __shared__ float buf[32][264];
  const int r = blockIdx.y;
  const float2* wr = w + (int64_t)r * N;
  const float2* V0 = Vb + (int64_t)r * N;
  float ax[NV], ay[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) ax[j] = ay[j] = 0.f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned amask = 0;     // bit j: slice of V_j 16-byte aligned
#pragma unroll
  for (int j = 0; j < NV; ++j)
    if (j < nv && al16(V0 + j * vstride)) amask |= 1u << j;
  const bool wal = al16(wr);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N / 2; i += stride) {
    const float4 b = ld_pair(wr, i, wal);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      if (j < nv) {
        const float4 a = ld_pair(V0 + j * vstride, i, (amask >> j) & 1u);
        ax[j] += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
        ay[j] += a.x * b.y - a.y * b.x + a.z * b.w - a.w * b.z;
      }
    }
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const float2 b = wr[N - 1];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      if (j < nv) {
        const float2 a = V0[j * vstride + N - 1];
        ax[j] += a.x * b.x + a.y * b.y;
        ay[j] += a.x * b.y - a.y * b.x;
      }
    }
  }
  const int t = threadIdx.x;
  const int o = t >> 3, sub = t & 7;       // row o of the transpose (vector h0 + o/2, part o%2), 8 lanes per row
#pragma unroll
  for (int h0 = 0; h0 < NV; h0 += 16) {
    if (h0 < nv) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        if (h0 + q < NV) {
          buf[2 * q][t] = ax[h0 + q < NV ? h0 + q : 0];
          buf[2 * q + 1][t] = ay[h0 + q < NV ? h0 + q : 0];
        }
      }
      __syncthreads();
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 32; ++q) acc += (double)buf[o][q * 8 + sub];
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      acc += __shfl_xor(acc, 4, 64);
      const int j = h0 + (o >> 1);
      if (sub == 0 && j < nv) {
        double* pp = (double*)&partial[((int64_t)r * nv + j) * gridDim.x + blockIdx.x];
        pp[o & 1] = acc;
      }
    }
  }
}

// dst = src - sum_{j < nv} h[r * ldh + j] V_j, nv <= NV <= 32 (src may equal dst); when
// partial != nullptr also |dst|^2 per workgroup (partial[r * gridDim.x + block])
template <int NV>
__global__ void __launch_bounds__(256) k_update32(const float2* __restrict__ Vb, const float2* src, float2* dst,
                                                  const double2* __restrict__ h, int nv, int ldh, int64_t N,
                                                  int64_t vstride, double2* __restrict__ partial) {
  __shared__ float2 hs[NV];
  __shared__ double red[4];
  const int r = blockIdx.y;
  if ((int)threadIdx.x < nv) {
    const double2 t = h[(int64_t)r * ldh + threadIdx.x];
    hs[threadIdx.x] = make_float2((float)t.x, (float)t.y);
  }
  __syncthreads();
  const float2* sr = src + (int64_t)r * N;
  float2* dr = dst + (int64_t)r * N;
  const float2* V0 = Vb + (int64_t)r * N;
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned amask = 0;     // bit j: slice of V_j 16-byte aligned
#pragma unroll
  for (int j = 0; j < NV; ++j)
    if (j < nv && al16(V0 + j * vstride)) amask |= 1u << j;
  const bool sal = al16(sr), dal = al16(dr);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N / 2; i += stride) {
    float4 acc = ld_pair(sr, i, sal);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      if (j < nv) {
        const float4 a = ld_pair(V0 + j * vstride, i, (amask >> j) & 1u);
        const float2 c = hs[j];
        acc.x -= c.x * a.x - c.y * a.y;
        acc.y -= c.x * a.y + c.y * a.x;
        acc.z -= c.x * a.z - c.y * a.w;
        acc.w -= c.x * a.w + c.y * a.z;
      }
    }
    st_pair(dr, i, dal, acc);
    nrm += (double)acc.x * acc.x + (double)acc.y * acc.y + ((double)acc.z * acc.z + (double)acc.w * acc.w);
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    float2 acc = sr[N - 1];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      if (j < nv) {
        const float2 a = V0[j * vstride + N - 1];
        const float2 c = hs[j];
        acc.x -= c.x * a.x - c.y * a.y;
        acc.y -= c.x * a.y + c.y * a.x;
      }
    }
    dr[N - 1] = acc;
    nrm += (double)acc.x * acc.x + (double)acc.y * acc.y;
  }
  if (partial == nullptr) return;
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
}

// out[r * ldo + off + j] = sum_p partial[(r * nv + j) * nparts + p], one workgroup per output
__global__ void __launch_bounds__(256) k_fold(const double2* __restrict__ partial, double2* __restrict__ out,
                                              int nparts, int nv, int ldo, int off) {
  __shared__ double rx[4], ry[4];
  const int o = blockIdx.x;
  double sx = 0.0, sy = 0.0;
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
    const double2 v = partial[(int64_t)o * nparts + p];
    sx += v.x;
    sy += v.y;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  if ((threadIdx.x & 63) == 0) {
    rx[threadIdx.x >> 6] = sx;
    ry[threadIdx.x >> 6] = sy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int r = o / nv, j = o % nv;
    out[(int64_t)r * ldo + off + j] = make_double2(rx[0] + rx[1] + rx[2] + rx[3], ry[0] + ry[1] + ry[2] + ry[3]);
  }
}

// dst = f - a (a may be null: dst = f), rounded to single; |f - a|^2 in double per workgroup
__global__ void __launch_bounds__(256) k_resid32(const double2* __restrict__ f, const float2* __restrict__ a,
                                                 float2* __restrict__ dst, int64_t N, double2* __restrict__ partial) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    double2 t = f[(int64_t)r * N + i];
    if (a) {
      const float2 b = a[(int64_t)r * N + i];
      t.x -= b.x;
      t.y -= b.y;
    }
    dst[(int64_t)r * N + i] = make_float2((float)t.x, (float)t.y);
    nrm += t.x * t.x + t.y * t.y;
  }
  nrm = wave_sum(nrm);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = make_double2(red[0] + red[1] + red[2] + red[3], 0.0);
}

__global__ void k_scale32(float2* __restrict__ v, const double* __restrict__ s, int64_t N) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const float f = (float)s[r];
  float2 a = v[(int64_t)r * N + i];
  a.x *= f;
  a.y *= f;
  v[(int64_t)r * N + i] = a;
}

// x_r += sum_j y[r * nvec + j] V_j (basis in single precision, sum in double)
__global__ void k_axpy_combo32(double2* __restrict__ x, const float2* __restrict__ Vb, const double2* __restrict__ y,
                               int nvec, int64_t N, int64_t vstride) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double2 acc = x[(int64_t)r * N + i];
  for (int j = 0; j < nvec; ++j) {
    const double2 c = y[r * nvec + j];
    if (c.x == 0.0 && c.y == 0.0) continue;   // frozen right-hand side (see k_axpy_combo)
    const float2 a = Vb[j * vstride + (int64_t)r * N + i];
    acc.x += c.x * a.x - c.y * a.y;
    acc.y += c.x * a.y + c.y * a.x;
  }
  x[(int64_t)r * N + i] = acc;
}

// ---------------------------------------------------------------------------
// Scattered field at points off the scatterer (outside: no singular part):
// u^s(x) = -kappa^2 [ far(x) + sum_{j in adjacent cells} G(|x - y_j|) c_j u_j ].
// One workgroup per target cell (a cell of the lattice box, occupied or
// not): the cell's face values of the lattice field minus its 3 x 3
// neighbours' equivalent-source fields give, through the cell's Dirichlet fit
// (one row per target, like a boundary-patch node), the field of the
// non-adjacent cells; the adjacent cells' sources are a stored row per target.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_targets(const typename C2<T>::t* __restrict__ u,
                                                 typename C2<T>::t* __restrict__ out,
                                                 const typename C2<T>::t* __restrict__ lat,
                                                 const typename C2<T>::t* __restrict__ sigma,
                                                 const typename C2<T>::t* __restrict__ ToffT,
                                                 const int32_t* __restrict__ tcell_xy,
                                                 const int32_t* __restrict__ tstart,
                                                 const int32_t* __restrict__ torig,
                                                 const typename C2<T>::t* __restrict__ Itg,
                                                 const int64_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ cols,
                                                 const typename C2<T>::t* __restrict__ vals,
                                                 const int32_t* __restrict__ cell_map, int L, int q, int U, int F,
                                                 int ncell, int Pa, int Pb, int64_t N, int64_t ntarg, T scale) {
  using V = typename C2<T>::t;
  extern __shared__ unsigned char smem_raw[];
  V* f = reinterpret_cast<V*>(smem_raw);      // F face values
  V* sg = f + F;                              // 9 * U neighbour strengths
  V* part = sg + 9 * U;                       // 9 * F adjacent fields
  int* nbr = reinterpret_cast<int*>(part + 9 * F);
  const int c = blockIdx.x, r = blockIdx.y;
  const int cx = tcell_xy[2 * c], cy = tcell_xy[2 * c + 1];
  const int64_t plane = (int64_t)Pa * Pb;
  if (threadIdx.x < 9) {
    const int nx = cx + (int)threadIdx.x % 3 - 1, ny = cy + (int)threadIdx.x / 3 - 1;
    nbr[threadIdx.x] = (nx >= 0 && ny >= 0 && nx < L && ny < L) ? cell_map[ny * L + nx] : -1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 9 * U; i += blockDim.x) {
    const int cn = nbr[i / U];
    sg[i] = cn >= 0 ? sigma[((int64_t)r * ncell + cn) * U + i % U] : czero<V>();
  }
  for (int t = threadIdx.x; t < F; t += blockDim.x) {
    const int s2 = t / (2 * q), fj = t % (2 * q), fc = fj / q, j = fj % q;
    const int cn = (s2 == 0 ? cx : cy) + fc, ct = (s2 == 0 ? cy : cx);
    f[t] = lat[((int64_t)(r * 2 + s2) * 2) * plane + (int64_t)cn * Pb + ct * q + j];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 9 * F; i += blockDim.x) {
    const int o = i / F, t = i % F, s2 = t / (2 * q);
    V acc = czero<V>();
    if (nbr[o] >= 0) {
      const V* Tcol = ToffT + ((int64_t)o * U + s2 * 4 * q) * F + t;
      const V* sv = sg + o * U + s2 * 4 * q;
      for (int k = 0; k < 4 * q; ++k) acc = cfma(Tcol[(int64_t)k * F], sv[k], acc);
    }
    part[i] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < F; t += blockDim.x) {
    V acc = f[t];
    for (int o = 0; o < 9; ++o) acc = csub(acc, part[o * F + t]);
    f[t] = acc;
  }
  __syncthreads();
  const V* ur = u + (int64_t)r * N;
  for (int ti = tstart[c] + threadIdx.x; ti < tstart[c + 1]; ti += blockDim.x) {
    V acc = czero<V>();
    const V* irow = Itg + (int64_t)ti * F;
    for (int t = 0; t < F; ++t) acc = cfma(irow[t], f[t], acc);
    for (int64_t k = rowptr[ti]; k < rowptr[ti + 1]; ++k) acc = cfma(vals[k], ur[cols[k]], acc);
    out[(int64_t)r * ntarg + torig[ti]] = cscale(acc, scale);
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
// x[i] = 0 and v[i] += x[i] over n complex values (the concurrent near
// field's buffer: cleared by a kernel, not a memset, so that graph capture
// records a kernel node)
template <typename V>
__global__ void k_zero_c(V* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = czero<V>();
}
template <typename V>
__global__ void k_add_c(V* __restrict__ v, const V* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = cadd(v[i], x[i]);
}

// Strided copies and clears, one block of n per right-hand side (grid: (n /
// 256, nrhs)).
template <typename V>
__global__ void __launch_bounds__(256) k_copy_strided(const V* __restrict__ src, int64_t ss, V* __restrict__ dst,
                                                      int64_t ds, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[(int64_t)blockIdx.y * ds + i] = src[(int64_t)blockIdx.y * ss + i];
}
template <typename V>
__global__ void __launch_bounds__(256) k_zero_strided(V* __restrict__ x, int64_t ds, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[(int64_t)blockIdx.y * ds + i] = czero<V>();
}

// Fourier refinement of the boundary patch's t1 lines (Sec. 3.1), first
// step: copies each right-hand side's u into the head of its block of x (ldx
// entries) and forms the density on the band grid, phi[line][v] = dens u[idx]
// (zero where the grid node is not an unknown).  Grid: (max(N, nl) / 256,
// nrhs).
template <typename T>
__global__ void __launch_bounds__(256) k_refine_gather(const typename C2<T>::t* __restrict__ u,
                                                       typename C2<T>::t* __restrict__ x,
                                                       typename C2<T>::t* __restrict__ phi,
                                                       const int32_t* __restrict__ idx, const T* __restrict__ dens,
                                                       int64_t N, int64_t ldx, int nl) {
  using V = typename C2<T>::t;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  const V* ur = u + (int64_t)r * N;
  if (i < N) x[(int64_t)r * ldx + i] = ur[i];
  if (i < nl) {
    const int j = idx[i];
    V p = czero<V>();
    if (j >= 0) {
      const V a = ur[j];
      const T c = dens[i];
      p.x = c * a.x;
      p.y = c * a.y;
    }
    phi[(int64_t)r * nl + i] = p;
  }
}

// Second step, after the forward line transforms: each line's spectrum
// times the phase ramp of the shift s / rf (ph[(s - 1) n1 + k], carrying the
// inverse transform's 1 / n1 and the Nyquist term split between +-n1/2) into
// the block of x for s; the inverse line transforms then leave the values at
// t1 = v + s / rf there.  Grid: (nl / 256, nrhs, rf - 1).
template <typename T>
__global__ void __launch_bounds__(256) k_refine_phase(const typename C2<T>::t* __restrict__ spec,
                                                      typename C2<T>::t* __restrict__ xt,
                                                      const typename C2<T>::t* __restrict__ ph, int n1, int nl,
                                                      int64_t ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nl) return;
  const int r = blockIdx.y, s1 = blockIdx.z;
  const int k = i % n1;
  xt[(int64_t)r * ldx + (int64_t)s1 * nl + i] = cmul(spec[(int64_t)r * nl + i], ph[(int64_t)s1 * n1 + k]);
}

// Interior refinement, after the forward 2-D transforms of the psi grids
// (M x M, row gy, column gx): the spectrum times the phase ramps of the shift
// (s1, s2) / rf, s = s2 rf + s1 = blockIdx.z + 1 (ph[s][k]: ramp along one
// axis, 1 / M included), into the refined grid of shift s in x (blocks of M^2
// from xt, ldx per right-hand side).  Grid: (M^2 / 256, nrhs, rf^2 - 1).
template <typename T>
__global__ void __launch_bounds__(256) k_refine_phase2(const typename C2<T>::t* __restrict__ spec,
                                                       typename C2<T>::t* __restrict__ xt,
                                                       const typename C2<T>::t* __restrict__ ph, int M, int rf,
                                                       int64_t ldx) {
  const int64_t M2 = (int64_t)M * M;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M2) return;
  const int r = blockIdx.y, s = blockIdx.z + 1;
  const int ky = (int)(i / M), kx = (int)(i - (int64_t)ky * M);
  const int s1 = s % rf, s2 = s / rf;
  xt[(int64_t)r * ldx + (int64_t)blockIdx.z * M2 + i] =
      cmul(cmul(spec[(int64_t)r * M2 + i], ph[(int64_t)s1 * M + kx]), ph[(int64_t)s2 * M + ky]);
}

template <typename T>
hipError_t launch_apply(const DevView<T>& d, const void* u_, void* v_, int nrhs, void* ws_, hipStream_t st,
                        hipEvent_t* ev, bool lattice_only) {
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], st);
  };
  using V = typename C2<T>::t;
  const V* u = static_cast<const V*>(u_);
  V* v = static_cast<V*>(v_);
  V* sigma = static_cast<V*>(ws_);
  V* lat = sigma + (size_t)nrhs * d.ncell * d.U;
  const int64_t plane = (int64_t)d.Pa * d.Pb;
  const T k2 = (T)(d.kappa * d.kappa);
  // near-field buffer of the concurrent apply (then the refinement's x and
  // line buffers)
  V* vn = lat + (size_t)nrhs * 4 * plane + (size_t)nrhs * (size_t)d.gw * d.gw;
  mark(0);
  // far field: a0 - a3 + a5 on the caller's stream (writes v)
  auto far_field = [&]() {
    // a0 + a1
    {
      size_t sh = (size_t)(d.S + d.max_nb) * sizeof(V);
      constexpr int RB = sizeof(T) == 4 ? 16 : 8;
      const size_t shb = ((size_t)(64 + d.max_nb) * RB + (size_t)RB * 96) * sizeof(V);
      if (d.q == 12 && d.S == 64 && d.PshT && d.bcells && d.proj_mfma) {
        // interior slots of every cell on the matrix cores, then the
        // boundary-patch nodes cell by cell
        constexpr bool G3 = std::is_same<T, float>::value;
        if (d.nicell > 0) {
          const int64_t ncols = (int64_t)d.nicell * nrhs;
          // tiles of 16 pairs; single-precision batches: the persistent
          // kernel, one workgroup per compute unit; otherwise one tile per
          // wave (the same products per pair either way)
          const int64_t ntl = (ncols + 15) / 16;
          bool done = false;
          if constexpr (G3) {
            if (ntl >= 256 * 8) {
              hipLaunchKernelGGL((k_project_int_walk<T, G3>), dim3(256), dim3(512), (size_t)64 * 96 * sizeof(V),
                                 st, u, sigma, (const V*)d.PshT, d.cw, d.slot_map, d.icells, d.nicell, d.ncell, d.N,
                                 nrhs);
              done = true;
            }
          }
          if (!done)
            hipLaunchKernelGGL((k_project_int<T, G3>), dim3((unsigned)((ntl + 3) / 4)), dim3(256),
                               (size_t)64 * 96 * sizeof(V), st, u, sigma, (const V*)d.PshT, d.cw, d.slot_map,
                               d.icells, d.nicell, d.ncell, d.N, nrhs);
        }
        // boundary-patch nodes: batches of 64 or more right-hand sides on the
        // matrix cores; fewer on the vector units (beside the interior
        // contraction of the concurrent apply, the matrix-core kernel slowed
        // it more than it saved)
        if (d.nbcell > 0 && nrhs >= 64) {
          hipLaunchKernelGGL((k_project_band_mfma<T, G3>), dim3(d.nbcell, (nrhs + 15) / 16), dim3(384), 0, st, u,
                             sigma, (const V*)d.Pbd, d.cw, d.bcells, d.cell_start, d.cell_nint, d.cell_nb,
                             d.cell_boff, d.N, d.ncell, nrhs);
        } else if (d.nbcell > 0) {
          const int RBB = nrhs >= 16 ? 16 : nrhs >= 4 ? 4 : 1;
          const size_t shp = ((size_t)d.max_nb * RBB + (size_t)RBB * 96) * sizeof(V);
          const dim3 gb(d.nbcell, (nrhs + RBB - 1) / RBB);
          if (RBB == 16)
            hipLaunchKernelGGL((k_project_band<T, 16>), gb, dim3(192), shp, st, u, sigma, (const V*)d.Pbd, d.cw,
                               d.bcells, d.cell_start, d.cell_nint, d.cell_nb, d.cell_boff, d.N, d.ncell, nrhs);
          else if (RBB == 4)
            hipLaunchKernelGGL((k_project_band<T, 4>), gb, dim3(192), shp, st, u, sigma, (const V*)d.Pbd, d.cw,
                               d.bcells, d.cell_start, d.cell_nint, d.cell_nb, d.cell_boff, d.N, d.ncell, nrhs);
          else
            hipLaunchKernelGGL((k_project_band<T, 1>), gb, dim3(192), shp, st, u, sigma, (const V*)d.Pbd, d.cw,
                               d.bcells, d.cell_start, d.cell_nint, d.cell_nb, d.cell_boff, d.N, d.ncell, nrhs);
        }
      } else if (d.q == 12 && d.S == 64 && d.PshT && nrhs >= RB && shb <= 64 * 1024) {
        hipLaunchKernelGGL((k_project_rb<T, RB>), dim3(d.ncell, (nrhs + RB - 1) / RB), dim3(192), shb, st, u, sigma,
                           (const V*)d.PshT, (const V*)d.Pbd, d.cw, d.slot_map, d.cell_start, d.cell_nint, d.cell_nb,
                           d.cell_boff, d.N, d.ncell, nrhs);
      } else if (d.q == 12 && d.S == 64 && d.PshT) {
        const size_t shm = (size_t)(96 + 64 + d.max_nb) * sizeof(V);
        hipLaunchKernelGGL(k_project2<T>, dim3(d.ncell, nrhs), dim3(192), shm, st, u, sigma, (const V*)d.PshT,
                           (const V*)d.Pbd, d.cw, d.slot_map, d.cell_start, d.cell_nint, d.cell_nb, d.cell_boff, d.N,
                           d.ncell);
      } else {
        hipLaunchKernelGGL(k_project<T>, dim3(d.ncell, nrhs), dim3(128), sh, st, u, sigma, (const V*)d.Psh,
                           (const V*)d.Pbd, d.cw, d.slot_map, d.cell_start, d.cell_nint, d.cell_nb, d.cell_boff,
                           d.S, d.U, d.N, d.ncell);
      }
    }
    mark(1);
    // lattice fill
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)(((int64_t)d.na * d.nb + 255) / 256), 2, nrhs), dim3(256), 0, st, sigma, lat,
                       d.cell_map, d.L, d.q, d.U, d.ncell, d.na, d.nb, d.Pa, d.Pb);
    mark(2);
    // a2: forward transforms of all 4 arrays per rhs
    const int nbatch = nrhs * 4;
    const int TCP = d.tc;   // columns per workgroup in the column transforms
    {
      size_t sh = 2 * (size_t)d.pb.n * sizeof(V);
      // rows a >= na are zero padding: their transforms stay zero
      if (d.rows_ip) {
        auto rows_f = d.rows_nth == 1024 ? k_fft_rows_ip<T, 1, 1024> : d.rows_nth == 512 ? k_fft_rows_ip<T, 1, 512>
                                                                                           : k_fft_rows_ip<T, 1, 256>;
        hipLaunchKernelGGL(rows_f, dim3(d.na, nbatch), dim3(d.rows_nth), sh / 2, st, lat, (const V*)d.twb, d.pb,
                           (int64_t)d.Pb, d.nb, d.Pb, plane);
      } else {
        auto rows_f = d.rows_nth == 1024 ? k_fft_rows<T, 1, 1024> : d.rows_nth == 512 ? k_fft_rows<T, 1, 512>
                                                                                       : k_fft_rows<T, 1, 256>;
        hipLaunchKernelGGL(rows_f, dim3(d.na, nbatch), dim3(d.rows_nth), sh, st, lat, (const V*)d.twb, d.pb,
                           (int64_t)d.Pb, d.nb, d.Pb, plane, (int64_t)0);
      }
      int TC = TCP;
      if (d.fft_variant == 1) {
        // fused column transforms + spectral product + inverse column transforms
        size_t shc = (4 * (size_t)TC + 1) * d.pa.n * sizeof(V);
        auto conv = d.cols_nth == 512 ? k_fft_cols_conv<T, 512> : k_fft_cols_conv<T, 256>;
        hipLaunchKernelGGL(conv, dim3(xcd_grid((d.Pb + TC - 1) / TC), nrhs * 2), dim3(d.cols_nth), shc, st, lat,
                           (const V*)d.twa, (const V*)d.khat, d.pa, d.Pb, TC, plane, d.na, 2 * plane);
      } else {
        size_t shc = (2 * (size_t)TC + 1) * d.pa.n * sizeof(V);
        hipLaunchKernelGGL((k_fft_cols<T, 1>), dim3(xcd_grid((d.Pb + TC - 1) / TC), nbatch), dim3(256), shc, st, lat,
                           (const V*)d.twa, d.pa, d.Pb, TC, plane, d.na, d.Pa, (int64_t)0);
      }
    }
    mark(3);
    if (d.fft_variant != 1)
      hipLaunchKernelGGL(k_spectral<T>, dim3((unsigned)((plane + 255) / 256), 2, nrhs), dim3(256), 0, st, lat,
                         (const V*)d.khat, plane);
    mark(4);
    {
      // inverse transforms of kind 0 of each set: batch stride 2 planes
      int TC = TCP;
      size_t shc = (2 * (size_t)TC + 1) * d.pa.n * sizeof(V);
      if (d.fft_variant != 1)
        hipLaunchKernelGGL((k_fft_cols<T, -1>), dim3(xcd_grid((d.Pb + TC - 1) / TC), nrhs * 2), dim3(256), shc, st,
                           lat,
                           (const V*)d.twa, d.pa, d.Pb, TC, 2 * plane, d.Pa, d.na, (int64_t)0);
      size_t sh = 2 * (size_t)d.pb.n * sizeof(V);
      if (d.rows_ip) {
        auto rows_i = d.rows_nth == 1024 ? k_fft_rows_ip<T, -1, 1024> : d.rows_nth == 512 ? k_fft_rows_ip<T, -1, 512>
                                                                                            : k_fft_rows_ip<T, -1, 256>;
        hipLaunchKernelGGL(rows_i, dim3(d.na, nrhs * 2), dim3(d.rows_nth), sh / 2, st, lat, (const V*)d.twb, d.pb,
                           (int64_t)d.Pb, d.Pb, d.nb, 2 * plane);
      } else {
        auto rows_i = d.rows_nth == 1024 ? k_fft_rows<T, -1, 1024> : d.rows_nth == 512 ? k_fft_rows<T, -1, 512>
                                                                                        : k_fft_rows<T, -1, 256>;
        hipLaunchKernelGGL(rows_i, dim3(d.na, nrhs * 2), dim3(d.rows_nth), sh, st, lat, (const V*)d.twb, d.pb,
                           (int64_t)d.Pb, d.Pb, d.nb, 2 * plane, (int64_t)0);
      }
    }
    mark(5);
    if (lattice_only) return;   // the caller evaluates the field itself
    // a3 + a5
    {
      if (d.q == 12 && d.S == 64 && nrhs >= 16) {
        hipLaunchKernelGGL(k_interp_rb<T>, dim3(d.ncell, (nrhs + 15) / 16), dim3(256), 0, st, u, v, (const V*)lat,
                           (const V*)d.Ish, (const V*)d.Ibd, d.cell_xy, d.slot_map, d.cell_start, d.cell_nint,
                           d.cell_nb, d.cell_boff, d.Pa, d.Pb, d.N, d.nband, nrhs, k2);
      } else if (d.q == 12 && d.S == 64) {
        constexpr int CB = 16;
        const size_t shm = (size_t)CB * 48 * sizeof(V) + 2 * CB * sizeof(int);
        hipLaunchKernelGGL((k_interp_mfma<T, CB>), dim3((d.ncell + CB - 1) / CB, nrhs), dim3(256), shm, st, u, v,
                           (const V*)lat, (const V*)d.Ish, (const V*)d.Ibd, d.cell_xy, d.slot_map, d.cell_start,
                           d.cell_nint, d.cell_nb, d.cell_boff, d.ncell, d.Pa, d.Pb, d.N, d.nband, k2);
      } else {
        hipLaunchKernelGGL(k_interp<T>, dim3(d.ncell, nrhs), dim3(256), (size_t)d.F * sizeof(V), st, u, v,
                           (const V*)lat, (const V*)d.Ish, (const V*)d.Ibd, d.cell_xy, d.slot_map, d.cell_start,
                           d.cell_nint, d.cell_nb, d.cell_boff, d.q, d.F, d.S, d.Pa, d.Pb, d.N, d.nband, k2);
      }
    }
  };
  if (lattice_only) {
    far_field();
    return hipGetLastError();
  }
  // Fourier refinement of the band's t1 lines for the rows (Sec. 3.1):
  // x = [u ; values at t1 = v + s / rf, s = 1 .. rf - 1] per right-hand side
  auto refine_band = [&](hipStream_t ns, V* x, V* phi) {
    const int n1 = d.rf_n1, nl = d.rf_lines * n1;
    const int64_t nmax = std::max<int64_t>(d.N, nl);
    hipLaunchKernelGGL(k_refine_gather<T>, dim3((unsigned)((nmax + 255) / 256), nrhs), dim3(256), 0, ns, u, x, phi,
                       d.rf_idx, d.rf_dens, d.N, d.ldx, nl);
    // (only N2 + 1 lines, a few dozen workgroups: each 4096-point line takes
    // about 24 us in single precision, 1024 threads per line no faster)
    const size_t sh = (size_t)n1 * sizeof(V);
    hipLaunchKernelGGL((k_fft_rows_ip<T, 1, 256>), dim3(d.rf_lines, nrhs), dim3(256), sh, ns, phi, (const V*)d.rf_tw,
                       d.rf_plan, (int64_t)n1, n1, n1, (int64_t)nl);
    hipLaunchKernelGGL(k_refine_phase<T>, dim3((unsigned)((nl + 255) / 256), nrhs, d.rf - 1), dim3(256), 0, ns,
                       (const V*)phi, x + d.N, (const V*)d.rf_ph, n1, nl, d.ldx);
    hipLaunchKernelGGL((k_fft_rows_ip<T, -1, 256>), dim3(d.rf_lines * (d.rf - 1), nrhs), dim3(256), sh, ns, x + d.N,
                       (const V*)d.rf_tw, d.rf_plan, (int64_t)n1, n1, n1, d.ldx);
  };
  // workspace of the refinements: x = [u ; refined band values ; refined psi
  // grids] (ldx per right-hand side), the band lines, the psi grids' spectra
  V* const rf_x = vn + (size_t)nrhs * d.N;
  V* const rf_phi = rf_x + (size_t)nrhs * d.ldx;
  V* const rf_spec = rf_phi + (size_t)nrhs * d.rf_lines * d.rf_n1;
  // the interior psi grids (after the face lattices)
  V* const grid = lat + (size_t)nrhs * 4 * plane;
  // Fourier refinement of the interior lattice (Sec. 3.1): the psi grids'
  // 2-D transforms (M x M, M = gw), times the phase ramps of each shift
  // (s1, s2) / rf, inverse transforms into the refined grids in x
  auto refine_interior = [&](hipStream_t ns) {
    const int M = d.gw;
    const int64_t M2 = (int64_t)M * M;
    const bool dbl = sizeof(T) == 8;
    const int TC = dbl ? 2 : 4;
    const int nsh = d.rfi * d.rfi - 1;
    V* xt = rf_x + d.N + d.rf_ioff;
    (void)launch_fft_lines(dbl, 1, grid, rf_spec, d.rf_itw, d.rf_iplan, M, M, M2, 0, M, M2, 0, nrhs, 1, M, M, ns);
    (void)launch_fft_strided(dbl, 1, rf_spec, d.rf_itw, d.rf_iplan, M, TC, M2, nrhs, M, M, 0, 1, ns);
    hipLaunchKernelGGL(k_refine_phase2<T>, dim3((unsigned)((M2 + 255) / 256), nrhs, nsh), dim3(256), 0, ns,
                       (const V*)rf_spec, xt, (const V*)d.rf_iph, M, d.rfi, d.ldx);
    (void)launch_fft_strided(dbl, -1, xt, d.rf_itw, d.rf_iplan, M, TC, d.ldx, nrhs, M, M, M2, nsh, ns);
    (void)launch_fft_lines(dbl, -1, xt, xt, d.rf_itw, d.rf_iplan, M, M, d.ldx, M2, M, d.ldx, M2, nrhs, nsh, M, M,
                           ns);
  };
  // a4 between interior nodes, into vt on stream ns
  auto psi_grid = [&](hipStream_t ns) {
    const int Gw = d.gw;
    const int64_t gsz = (int64_t)Gw * Gw;
    if (nrhs >= 8)
      hipLaunchKernelGGL((k_psi_grid<T, 8>), dim3((unsigned)((gsz + 255) / 256), (nrhs + 7) / 8), dim3(256), 0, ns, u,
                         grid, d.dw, d.cell_map, d.slot_map, d.L, 8, d.S, Gw, d.N, nrhs);
    else
      hipLaunchKernelGGL((k_psi_grid<T, 1>), dim3((unsigned)((gsz + 255) / 256), nrhs), dim3(256), 0, ns, u, grid,
                         d.dw, d.cell_map, d.slot_map, d.L, 8, d.S, Gw, d.N, nrhs);
  };
  // the refinements the near field reads (band lines, interior psi grids),
  // issued once per apply ahead of the first near-field kernel that needs them
  bool prepped = false;
  auto prep = [&](hipStream_t ns) {
    if (prepped) return;
    prepped = true;
    if (d.rf > 1) {
      refine_band(ns, rf_x, rf_phi);
    } else if (d.ldx > d.N) {
      // x without band refinement (off-grid shortcut only): u into its head
      hipLaunchKernelGGL(k_copy_strided<V>, dim3((unsigned)((d.N + 255) / 256), nrhs), dim3(256), 0, ns, u, d.N,
                         rf_x, d.ldx, d.N);
    }
    if (d.rfi > 1) {
      psi_grid(ns);
      refine_interior(ns);
    }
  };
  auto near_shared = [&](hipStream_t ns, V* vt) {
    if (d.ch == 8) {
      const int Gw = d.gw;
      if (d.rfi > 1) prep(ns);
      else psi_grid(ns);
      // one contraction per shift of the refined lattice (shift 0: the psi
      // grid itself)
      for (int s = 0; s < d.rfi * d.rfi; ++s) {
        const V* gs = s == 0 ? grid : rf_x + d.N + d.rf_ioff + (size_t)(s - 1) * Gw * Gw;
        const int64_t gstride = s == 0 ? (int64_t)Gw * Gw : d.ldx;
        const V* Ws = (const V*)d.Wsh + (size_t)s * d.S * (5 * 8) * (5 * 8);
        if (std::is_same<T, float>::value && d.near_variant != 1) {
          const int CT = d.near_variant == 2 ? 2 : d.near_variant >= 3 ? 4 : 1;
          const dim3 gr((d.nicell + 16 * CT - 1) / (16 * CT), nrhs), bl(256 * CT);
          if (d.near_variant == 4)
            hipLaunchKernelGGL((k_near_shared_mfma_db<4, true>), gr, bl, 0, ns, (const float2*)gs, (float2*)vt,
                               (const float2*)Ws, d.icells, d.cell_xy, d.slot_map, Gw, d.nicell, d.N, (float)k2,
                               gstride);
          else if (CT == 1)
            hipLaunchKernelGGL(k_near_shared_mfma_db<1>, gr, bl, 0, ns, (const float2*)gs, (float2*)vt,
                               (const float2*)Ws, d.icells, d.cell_xy, d.slot_map, Gw, d.nicell, d.N, (float)k2,
                               gstride);
          else if (CT == 2)
            hipLaunchKernelGGL(k_near_shared_mfma_db<2>, gr, bl, 0, ns, (const float2*)gs, (float2*)vt,
                               (const float2*)Ws, d.icells, d.cell_xy, d.slot_map, Gw, d.nicell, d.N, (float)k2,
                               gstride);
          else
            hipLaunchKernelGGL(k_near_shared_mfma_db<4>, gr, bl, 0, ns, (const float2*)gs, (float2*)vt,
                               (const float2*)Ws, d.icells, d.cell_xy, d.slot_map, Gw, d.nicell, d.N, (float)k2,
                               gstride);
        } else {
          constexpr int NT = 2;
          hipLaunchKernelGGL((k_near_shared_mfma<T, NT>), dim3((d.nicell + 16 * NT - 1) / (16 * NT), nrhs),
                             dim3(256), 0, ns, (const V*)gs, vt, Ws, d.icells, d.cell_xy, d.slot_map, Gw, d.nicell,
                             d.N, k2, gstride);
        }
      }
    } else {
      constexpr int CT = 16, KC = 32;
      size_t sh = (size_t)(d.S * KC + KC * CT) * sizeof(V) + 25 * CT * sizeof(int);
      hipLaunchKernelGGL((k_near_shared<T, CT, KC>), dim3((d.nicell + CT - 1) / CT, nrhs), dim3(256), sh, ns, u, vt,
                         (const V*)d.Wsh, d.dw, d.icells, d.cell_xy, d.cell_map, d.slot_map, d.L, d.ch, d.S,
                         d.nicell, d.N, k2);
    }
  };
  // a4 rows of the boundary patch, into vt on stream ns
  auto near_rows = [&](hipStream_t ns, V* vt) {
    if (d.nrows > 0) {
      const dim3 g((d.nrows + 3) / 4), b(256);
      // dense tiles (either precision): right-hand-side-major input copied
      // into the lattice region (free after the interpolation; large
      // enough, checked here)
      const bool blk = d.bt_ntiles > 0 && d.csr_variant >= 3 && nrhs % 16 == 0 && (int64_t)4 * plane >= d.N;
      // with Fourier refinement the rows read x = [u ; refined band lines]
      const V* ux = u;
      int64_t ldu = d.N;
      if (d.ldx > d.N) {
        prep(ns);
        ux = rf_x;
        ldu = d.ldx;
      }
      if (d.nsr > 0) {
        // off-grid shortcut: the boundary rule at the patch's grid nodes
        // into s (in x), then s refined along t1 like the densities
        const int nl = d.rf_lines * d.rf_n1;
        V* sreg = rf_x + d.N + d.sc_off;
        hipLaunchKernelGGL(k_zero_strided<V>, dim3((unsigned)((nl + 255) / 256), nrhs), dim3(256), 0, ns, sreg, d.ldx,
                           (int64_t)nl);
        if (std::is_same<T, double>::value)
          hipLaunchKernelGGL((k_near_csr<T, double2, int32_t>), dim3((d.nsr + 3) / 4), b, 0, ns, (const V*)rf_x, rf_x,
                             d.sr_rowptr, d.sr_rows, d.sr_colbase, d.sr_cols32, (const double2*)d.sr_vals, d.nsr,
                             d.ldx, nrhs, (T)1, d.ldx);
        else
          hipLaunchKernelGGL((k_near_csr<T, float2, int32_t>), dim3((d.nsr + 3) / 4), b, 0, ns, (const V*)rf_x, rf_x,
                             d.sr_rowptr, d.sr_rows, d.sr_colbase, d.sr_cols32, (const float2*)d.sr_vals, d.nsr,
                             d.ldx, nrhs, (T)1, d.ldx);
        if (d.rf > 1) {
          const int n1 = d.rf_n1;
          const size_t sh = (size_t)n1 * sizeof(V);
          hipLaunchKernelGGL(k_copy_strided<V>, dim3((unsigned)((nl + 255) / 256), nrhs), dim3(256), 0, ns,
                             (const V*)sreg, d.ldx, rf_phi, (int64_t)nl, (int64_t)nl);
          hipLaunchKernelGGL((k_fft_rows_ip<T, 1, 256>), dim3(d.rf_lines, nrhs), dim3(256), sh, ns, rf_phi,
                             (const V*)d.rf_tw, d.rf_plan, (int64_t)n1, n1, n1, (int64_t)nl);
          hipLaunchKernelGGL(k_refine_phase<T>, dim3((unsigned)((nl + 255) / 256), nrhs, d.rf - 1), dim3(256), 0, ns,
                             (const V*)rf_phi, sreg + nl, (const V*)d.rf_ph, n1, nl, d.ldx);
          hipLaunchKernelGGL((k_fft_rows_ip<T, -1, 256>), dim3(d.rf_lines * (d.rf - 1), nrhs), dim3(256), sh, ns,
                             sreg + nl, (const V*)d.rf_tw, d.rf_plan, (int64_t)n1, n1, n1, d.ldx);
        }
      }
      if (d.csr_f64 && !blk) {
        if (d.coloff)
          hipLaunchKernelGGL((k_near_csr<T, double2, uint16_t>), g, b, 0, ns, ux, vt, d.rowptr, d.rows, d.colbase,
                             d.coloff, (const double2*)d.vals, d.nrows, d.N, nrhs, k2, ldu);
        else
          hipLaunchKernelGGL((k_near_csr<T, double2, int32_t>), g, b, 0, ns, ux, vt, d.rowptr, d.rows, d.colbase,
                             d.cols32, (const double2*)d.vals, d.nrows, d.N, nrhs, k2, ldu);
      } else {
        if (blk) {
          V* ut = lat;
          hipLaunchKernelGGL(k_rhs_major<V>, dim3((unsigned)((d.N + 31) / 32), (nrhs + 31) / 32), dim3(256), 0, ns,
                             u, ut, d.N, nrhs);
          constexpr int NT = 4;
          const int64_t waves = (int64_t)d.bt_ntiles * ((nrhs + 16 * NT - 1) / (16 * NT));
          if (std::is_same<T, float>::value && d.csr_variant == 4)
            hipLaunchKernelGGL((k_near_blk<T, NT, true>), dim3((unsigned)((waves + 3) / 4)), b, 0, ns,
                               (const V*)ut, vt, d.bt_rows, d.bt_info, d.bt_woff, d.bt_cols, (const V*)d.bt_w,
                               d.bt_ntiles, d.N, nrhs, k2);
          else
            hipLaunchKernelGGL((k_near_blk<T, NT>), dim3((unsigned)((waves + 3) / 4)), b, 0, ns, (const V*)ut, vt,
                               d.bt_rows, d.bt_info, d.bt_woff, d.bt_cols, (const V*)d.bt_w, d.bt_ntiles, d.N,
                               nrhs, k2);
        } else if (d.run_ptr && std::is_same<T, float>::value && d.csr_variant >= 2)
          hipLaunchKernelGGL(k_near_csr4r, g, b, (size_t)4 * (2 * d.run_max + 1) * sizeof(int), ns, (const float2*)ux,
                             (float2*)vt, d.rowptr, d.rows, d.run_ptr, d.run_cs, d.run_pre, (const float2*)d.vals,
                             d.nrows, d.N, nrhs, (float)k2, d.run_max, ldu);
        else if (d.coloff && std::is_same<T, float>::value && d.csr_variant == 0)
          hipLaunchKernelGGL(k_near_csr4, g, b, 0, ns, (const float2*)ux, (float2*)vt, d.rowptr, d.rows, d.colbase,
                             d.coloff, (const float2*)d.vals, d.nrows, d.N, nrhs, (float)k2, ldu);
        else if (d.coloff)
          hipLaunchKernelGGL((k_near_csr<T, float2, uint16_t>), g, b, 0, ns, ux, vt, d.rowptr, d.rows, d.colbase,
                             d.coloff, (const float2*)d.vals, d.nrows, d.N, nrhs, k2, ldu);
        else
          hipLaunchKernelGGL((k_near_csr<T, float2, int32_t>), g, b, 0, ns, ux, vt, d.rowptr, d.rows, d.colbase,
                             d.cols32, (const float2*)d.vals, d.nrows, d.N, nrhs, k2, ldu);
      }
    }
  };
  // The far field (projection through interpolation, which writes v) and the
  // near field touch disjoint workspace regions and read only u, so unless
  // the stages are being timed one by one, the near field runs concurrently
  // on the side stream into a cleared buffer after the interior grid, added
  // into v once both are done.  (Measured: the interior near field on the
  // caller's stream after the interpolation instead slows the concurrent
  // rows more than it shortens the side stream.)  The dense-tile form
  // borrows the lattice region and stays on the caller's stream after the
  // far field.
  const bool blk_rows = d.bt_ntiles > 0 && d.csr_variant >= 3 && nrhs % 16 == 0;
  const bool fork = d.side && !ev && !blk_rows;
  const int64_t nv = d.N * nrhs;
  const unsigned nvb = (unsigned)((nv + 255) / 256);
  if (fork) {
    // cleared before the fork: on the side stream the clear would queue
    // behind the projection's workgroups and delay the whole near field
    hipLaunchKernelGGL(k_zero_c<V>, dim3(nvb), dim3(256), 0, st, vn, nv);
    hipError_t e = hipEventRecord(d.ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(d.side, d.ev_fork, 0);
    if (e != hipSuccess) return e;
    if (d.rows_first) {
      near_rows(d.side, vn);
      near_shared(d.side, vn);
    } else {
      near_shared(d.side, vn);
      near_rows(d.side, vn);
    }
    if ((e = hipEventRecord(d.ev_join, d.side)) != hipSuccess) return e;
  }
  far_field();
  if (fork) {
    hipError_t e = hipStreamWaitEvent(st, d.ev_join, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_add_c<V>, dim3(nvb), dim3(256), 0, st, v, (const V*)vn, nv);
  } else {
    mark(6);
    near_shared(st, v);
    mark(7);
    near_rows(st, v);
  }
  mark(8);
  return hipGetLastError();
}

template hipError_t launch_apply<double>(const DevView<double>&, const void*, void*, int, void*, hipStream_t,
                                         hipEvent_t*, bool);
template hipError_t launch_apply<float>(const DevView<float>&, const void*, void*, int, void*, hipStream_t,
                                        hipEvent_t*, bool);

// Transforms along one axis of a multi-dimensional array (3-D face
// lattices): `lines` transforms contiguous lines, several per workgroup
// (grid lines / L x nbatch x nz), from src to dst; `strided` transforms
// columns of an nrows x ncols slab in tiles of TC columns (grid tiles x
// nbatch x nz); precision from `dbl`, direction from `dir`.
int fft_lines_per_group(bool dbl, int n) { return std::max(1, std::min(16, (dbl ? 1024 : 2048) / n)); }

hipError_t launch_fft_lines(bool dbl, int dir, const void* src, void* dst, const void* tw, const FftPlan& plan,
                            int nlines, int64_t s_line, int64_t s_batch, int64_t s_z, int64_t d_line, int64_t d_batch,
                            int64_t d_z, int nbatch, int nz, int nload, int nstore, hipStream_t st) {
  const int L = fft_lines_per_group(dbl, plan.n), S = L == 1 ? 1 : L + 1;
  const dim3 g((nlines + L - 1) / L, nbatch, nz), b(256);
  if (dbl) {
    const size_t sh = (2 * (size_t)S + 1) * plan.n * sizeof(double2);
    auto k = dir > 0 ? k_fft_lines<double, 1> : k_fft_lines<double, -1>;
    hipLaunchKernelGGL(k, g, b, sh, st, (const double2*)src, (double2*)dst, (const double2*)tw, plan, nlines, L,
                       s_line, s_batch, s_z, d_line, d_batch, d_z, nload, nstore);
  } else if (plan.npass == 2 && plan.radix[0] == 16 && plan.radix[1] == 16) {
    const size_t sh = ((size_t)16 * 16 * 17 + 256) * sizeof(float2);
    auto k = dir > 0 ? k_fft_lines2<1, 16, 16> : k_fft_lines2<-1, 16, 16>;
    hipLaunchKernelGGL(k, dim3((nlines + 15) / 16, nbatch, nz), b, sh, st, (const float2*)src, (float2*)dst,
                       (const float2*)tw, nlines, s_line, s_batch, s_z, d_line, d_batch, d_z, nload, nstore);
  } else {
    const size_t sh = (2 * (size_t)S + 1) * plan.n * sizeof(float2);
    auto k = dir > 0 ? k_fft_lines<float, 1> : k_fft_lines<float, -1>;
    hipLaunchKernelGGL(k, g, b, sh, st, (const float2*)src, (float2*)dst, (const float2*)tw, plan, nlines, L,
                       s_line, s_batch, s_z, d_line, d_batch, d_z, nload, nstore);
  }
  return hipGetLastError();
}

hipError_t launch_fft_strided(bool dbl, int dir, void* data, const void* tw, const FftPlan& plan, int ncols, int TC,
                              int64_t batch_stride, int nbatch, int nload, int nstore, int64_t zstride, int nz,
                              hipStream_t st) {
  const dim3 g(xcd_grid((ncols + TC - 1) / TC), nbatch, nz), b(256);
  if (dbl) {
    const size_t sh = (2 * (size_t)TC + 1) * plan.n * sizeof(double2);
    auto k = dir > 0 ? k_fft_cols<double, 1> : k_fft_cols<double, -1>;
    hipLaunchKernelGGL(k, g, b, sh, st, (double2*)data, (const double2*)tw, plan, ncols, TC, batch_stride, nload,
                       nstore, zstride);
  } else if (plan.npass == 2 && plan.radix[0] == 16 && plan.radix[1] == 16) {
    const size_t sh = ((size_t)TC + 1) * plan.n * sizeof(float2);
    auto k = dir > 0 ? k_fft_cols2<1, 16, 16> : k_fft_cols2<-1, 16, 16>;
    hipLaunchKernelGGL(k, g, b, sh, st, (float2*)data, (const float2*)tw, ncols, TC, batch_stride, nload, nstore,
                       zstride);
  } else {
    const size_t sh = (2 * (size_t)TC + 1) * plan.n * sizeof(float2);
    auto k = dir > 0 ? k_fft_cols<float, 1> : k_fft_cols<float, -1>;
    hipLaunchKernelGGL(k, g, b, sh, st, (float2*)data, (const float2*)tw, plan, ncols, TC, batch_stride, nload,
                       nstore, zstride);
  }
  return hipGetLastError();
}

hipError_t launch_fft_conv_octant(void* data, const void* tw, const void* khs, const FftPlan& plan, int Pb, int Pc,
                                  int TC, int nth, int64_t rstride, int64_t vol, int na, int nsets, hipStream_t st) {
  if (TC == 16 && nth == 256 && plan.npass == 2 && plan.radix[0] == 12 && plan.radix[1] == 6) {
    const size_t sh2 = (32 + 1) * (size_t)plan.n * sizeof(float2);
    hipLaunchKernelGGL((k_fft_conv_octant2<12, 6>), dim3(xcd_grid((Pb * Pc + 15) / 16), nsets), dim3(256), sh2, st,
                       (float2*)data, (const float2*)tw, (const float2*)khs, Pb, Pc, rstride, vol, na);
    return hipGetLastError();
  }
  const size_t sh = (4 * (size_t)TC + 1) * plan.n * sizeof(float2);
  auto k = nth == 512 ? k_fft_conv_octant<float, 512> : k_fft_conv_octant<float, 256>;
  hipLaunchKernelGGL(k, dim3(xcd_grid((Pb * Pc + TC - 1) / TC), nsets), dim3(nth == 512 ? 512 : 256), sh, st,
                     (float2*)data, (const float2*)tw, (const float2*)khs, plan, Pb, Pc, TC, rstride, vol, na);
  return hipGetLastError();
}

hipError_t set_fft_lds_limits(size_t bytes) {
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  };
  set((const void*)k_fft_rows<double, 1, 256>);
  set((const void*)k_fft_rows<double, -1, 256>);
  set((const void*)k_fft_rows<double, 1, 512>);
  set((const void*)k_fft_rows<double, -1, 512>);
  set((const void*)k_fft_rows<double, 1, 1024>);
  set((const void*)k_fft_rows<double, -1, 1024>);
  set((const void*)k_fft_rows<float, 1, 512>);
  set((const void*)k_fft_rows<float, -1, 512>);
  set((const void*)k_fft_rows<float, 1, 1024>);
  set((const void*)k_fft_rows<float, -1, 1024>);
  set((const void*)k_fft_cols<double, 1>);
  set((const void*)k_fft_cols<double, -1>);
  set((const void*)k_fft_rows<float, 1, 256>);
  set((const void*)k_fft_rows<float, -1, 256>);
  set((const void*)k_fft_rows_ip<float, 1, 256>);
  set((const void*)k_fft_rows_ip<float, -1, 256>);
  set((const void*)k_fft_rows_ip<float, 1, 512>);
  set((const void*)k_fft_rows_ip<float, -1, 512>);
  set((const void*)k_fft_rows_ip<float, 1, 1024>);
  set((const void*)k_fft_rows_ip<float, -1, 1024>);
  set((const void*)k_fft_rows_ip<double, 1, 256>);
  set((const void*)k_fft_rows_ip<double, -1, 256>);
  set((const void*)k_fft_rows_ip<double, 1, 512>);
  set((const void*)k_fft_rows_ip<double, -1, 512>);
  set((const void*)k_fft_rows_ip<double, 1, 1024>);
  set((const void*)k_fft_rows_ip<double, -1, 1024>);
  set((const void*)k_fft_cols<float, 1>);
  set((const void*)k_fft_cols<float, -1>);
  set((const void*)k_project_int_walk<float, true>);
  set((const void*)k_project_int<double, false>);
  set((const void*)k_project_int<float, true>);
  set((const void*)k_project_band<double, 16>);
  set((const void*)k_project_band<double, 4>);
  set((const void*)k_project_band<double, 1>);
  set((const void*)k_project_band<float, 16>);
  set((const void*)k_project_band<float, 4>);
  set((const void*)k_project_band<float, 1>);
  set((const void*)k_fft_cols_conv<double, 256>);
  set((const void*)k_fft_cols_conv<float, 256>);
  set((const void*)k_fft_cols_conv<double, 512>);
  set((const void*)k_fft_cols_conv<float, 512>);
  set((const void*)k_fft_lines<double, 1>);
  set((const void*)k_fft_lines<double, -1>);
  set((const void*)k_fft_lines<float, 1>);
  set((const void*)k_fft_lines<float, -1>);
  set((const void*)k_fft_conv_octant<float, 256>);
  set((const void*)k_fft_conv_octant<float, 512>);
  set((const void*)k_fft_cols2<1, 16, 16>);
  set((const void*)k_fft_lines2<1, 16, 16>);
  set((const void*)k_fft_lines2<-1, 16, 16>);
  set((const void*)k_fft_cols2<-1, 16, 16>);
  return e;
}

hipError_t launch_fft_kernels_forward(const DevView<double>& d, void* data, int nbatch, hipStream_t st) {
  using V = double2;
  const int64_t plane = (int64_t)d.Pa * d.Pb;
  size_t sh = 2 * (size_t)d.pb.n * sizeof(V);
  hipLaunchKernelGGL((k_fft_rows<double, 1, 256>), dim3(d.Pa, nbatch), dim3(256), sh, st, (V*)data, (const V*)d.twb,
                     d.pb, (int64_t)d.Pb, d.Pb, d.Pb, plane, (int64_t)0);
  int TC = d.tc;
  size_t shc = (2 * (size_t)TC + 1) * d.pa.n * sizeof(V);
  hipLaunchKernelGGL((k_fft_cols<double, 1>), dim3(xcd_grid((d.Pb + TC - 1) / TC), nbatch), dim3(256), shc, st,
                     (V*)data,
                     (const V*)d.twa, d.pa, d.Pb, TC, plane, d.Pa, d.Pa, (int64_t)0);
  return hipGetLastError();
}

// GMRES launchers
hipError_t gm_dots(const void* Vb, const void* w, void* partial, void* out, int nvec, int64_t N, int nrhs,
                   int64_t vstride, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(nparts, nrhs), dim3(256), 0, st, (const double2*)Vb, (const double2*)w,
                     (double2*)partial, nvec, N, nrhs, vstride);
  int count = nvec * nrhs;
  hipLaunchKernelGGL(k_reduce_partials, dim3(count), dim3(256), 0, st, (const double2*)partial, (double2*)out,
                     nparts, count);
  return hipGetLastError();
}
hipError_t gm_cgs(const void* Vb, void* w, const void* h, void* partial, void* out, int nvec, int64_t N,
                  int nrhs, int64_t vstride, int nparts, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_cgs, dim3(nparts, nrhs), dim3(256), 0, st, (const double2*)Vb, (double2*)w,
                     (const double2*)h, (double2*)partial, nvec, N, vstride, mode);
  int count = (mode == 2 ? 1 : nvec) * nrhs;
  hipLaunchKernelGGL(k_reduce_partials, dim3(count), dim3(256), 0, st, (const double2*)partial, (double2*)out,
                     nparts, count);
  return hipGetLastError();
}
hipError_t gm_inv_norm(const void* dd, double* s, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_inv_norm, dim3((nrhs + 63) / 64), dim3(64), 0, st, (const double2*)dd, s, nrhs);
  return hipGetLastError();
}
hipError_t gm_update(const void* Vb, void* w, const void* h, int nvec, int64_t N, int nrhs, int64_t vstride,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_update, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, (const double2*)Vb,
                     (double2*)w, (const double2*)h, nvec, N, nrhs, vstride);
  return hipGetLastError();
}
hipError_t gm_scale_copy(const void* src, void* dst, const double* s, int64_t N, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, (const double2*)src,
                     (double2*)dst, s, N);
  return hipGetLastError();
}
hipError_t gm_axpy_combo(void* x, const void* Vb, const void* y, int nvec, int64_t N, int nrhs, int64_t vstride,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_combo, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, (double2*)x,
                     (const double2*)Vb, (const double2*)y, nvec, N, vstride);
  return hipGetLastError();
}
hipError_t gm_sub(const void* a, const void* b, void* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double2*)a,
                     (const double2*)b, (double2*)out, n);
  return hipGetLastError();
}
hipError_t gm_add(void* x, const void* e, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (double2*)x, (const double2*)e, n);
  return hipGetLastError();
}
hipError_t gm_to_f32(const void* a, void* b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const double2*)a, (float2*)b, n);
  return hipGetLastError();
}
hipError_t gm_to_f64(const void* a, void* b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const float2*)a, (double2*)b, n);
  return hipGetLastError();
}

// single-precision-basis launchers
namespace {
int nv_bucket(int nv) { return nv <= 8 ? 8 : nv <= 16 ? 16 : 32; }
}  // namespace

hipError_t gm32_dots(const void* Vb, const void* w, void* partial, void* out, int nvec, int ldo, int64_t N,
                     int nrhs, int64_t vstride, int nparts, hipStream_t st) {
  // at most 32 basis vectors per pass: 64 accumulators per thread keep six waves per SIMD resident
  for (int c0 = 0; c0 < nvec; c0 += 32) {
    const int nv = nvec - c0 < 32 ? nvec - c0 : 32;
    const float2* V = (const float2*)Vb + (int64_t)c0 * vstride;
    dim3 g(nparts, nrhs);
    auto kern = nv_bucket(nv) == 8 ? k_dots32<8> : nv_bucket(nv) == 16 ? k_dots32<16> : k_dots32<32>;
    hipLaunchKernelGGL(kern, g, dim3(256), 0, st, V, (const float2*)w, (double2*)partial, nv, N, vstride);
    hipLaunchKernelGGL(k_fold, dim3(nv * nrhs), dim3(256), 0, st, (const double2*)partial, (double2*)out, nparts, nv,
                       ldo, c0);
  }
  return hipGetLastError();
}

hipError_t gm32_update(const void* Vb, const void* src, void* dst, const void* h, int nvec, int64_t N, int nrhs,
                       int64_t vstride, int nparts, void* partial, void* norm_out, hipStream_t st) {
  // at most 32 basis vectors per pass (64 values per thread in flight at full occupancy)
  const float2* in = (const float2*)src;
  for (int c0 = 0; c0 < nvec; c0 += 32) {
    const int nv = nvec - c0 < 32 ? nvec - c0 : 32;
    const bool last = c0 + 32 >= nvec;
    const float2* V = (const float2*)Vb + (int64_t)c0 * vstride;
    const double2* hh = (const double2*)h + c0;
    double2* part = (last && norm_out) ? (double2*)partial : nullptr;
    dim3 g(nparts, nrhs);
    auto kern = nv_bucket(nv) == 8 ? k_update32<8> : nv_bucket(nv) == 16 ? k_update32<16> : k_update32<32>;
    hipLaunchKernelGGL(kern, g, dim3(256), 0, st, V, in, (float2*)dst, hh, nv, nvec, N, vstride, part);
    in = (const float2*)dst;
  }
  if (norm_out)
    hipLaunchKernelGGL(k_fold, dim3(nrhs), dim3(256), 0, st, (const double2*)partial, (double2*)norm_out, nparts, 1, 1, 0);
  return hipGetLastError();
}

hipError_t gm32_resid(const void* f, const void* a, void* dst, int64_t N, int nrhs, int nparts, void* partial,
                      void* norm_out, hipStream_t st) {
  hipLaunchKernelGGL(k_resid32, dim3(nparts, nrhs), dim3(256), 0, st, (const double2*)f, (const float2*)a,
                     (float2*)dst, N, (double2*)partial);
  hipLaunchKernelGGL(k_fold, dim3(nrhs), dim3(256), 0, st, (const double2*)partial, (double2*)norm_out, nparts, 1, 1, 0);
  return hipGetLastError();
}

hipError_t gm32_scale(void* v, const double* s, int64_t N, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_scale32, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, (float2*)v, s, N);
  return hipGetLastError();
}

hipError_t gm32_axpy_combo(void* x, const void* Vb, const void* y, int nvec, int64_t N, int nrhs, int64_t vstride,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_combo32, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, (double2*)x,
                     (const float2*)Vb, (const double2*)y, nvec, N, vstride);
  return hipGetLastError();
}

hipError_t launch_targets(const DevView<double>& d, const TargetView& tg, const void* u, void* out, int nrhs,
                          void* ws, hipStream_t st) {
  hipError_t e = launch_apply<double>(d, u, nullptr, nrhs, ws, st, nullptr, true);
  if (e != hipSuccess) return e;
  using V = double2;
  const V* sigma = static_cast<const V*>(ws);
  const V* lat = sigma + (size_t)nrhs * d.ncell * d.U;
  const size_t sh = (size_t)(d.F + 9 * d.U + 9 * d.F) * sizeof(V) + 16 * sizeof(int);
  hipLaunchKernelGGL(k_targets<double>, dim3(tg.ncell, nrhs), dim3(256), sh, st, (const V*)u, (V*)out, lat, sigma,
                     (const V*)d.Toff, tg.cell_xy, tg.start, tg.orig, (const V*)tg.fit, tg.rowptr, tg.cols,
                     (const V*)tg.vals, d.cell_map, d.L, d.q, d.U, d.F, d.ncell, d.Pa, d.Pb, d.N, tg.n,
                     -d.kappa * d.kappa);
  return hipGetLastError();
}

}  // namespace lsx
