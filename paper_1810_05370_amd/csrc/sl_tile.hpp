// LDS halo tiles for the semi-Lagrangian gathers (forward and adjoint).
//
// A block of 256 threads owns a brick of arrival voxels.  For a gather stage it
// reduces the floors of its departure points to their bounding box
// (block_box), widens it by the tricubic stencil's reach -1 .. +2
// (box_fits), copies that box of the needed fields from HBM into LDS once
// (tile_stage: coalesced rows, periodic wrap), and its voxels then read their
// 64 taps from the tile.  Nodes hold G values of one type (a 16-byte node:
// 4 FP32 or 2 FP64 values; 8 bytes for a single FP64 value).
#pragma once
#include <hip/hip_runtime.h>

namespace tumor {

template <typename RC, int G>
struct TileVec {
  typedef RC type __attribute__((ext_vector_type(G)));
};
template <typename RC>
struct TileVec<RC, 1> {
  typedef RC type;
};

template <int G, typename RC>
__device__ __forceinline__ void tile_put(RC* tile, int e, const RC (&v)[G]) {
  typedef typename TileVec<RC, G>::type vt;
  vt t;
  if constexpr (G == 1) {
    t = v[0];
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g) t[g] = v[g];
  }
  reinterpret_cast<vt*>(tile)[e] = t;
}

template <int G, typename RC>
__device__ __forceinline__ void tile_get(const RC* tile, int e, RC (&v)[G]) {
  typedef typename TileVec<RC, G>::type vt;
  const vt t = reinterpret_cast<const vt*>(tile)[e];
  if constexpr (G == 1) {
    v[0] = t;
  } else {
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] = t[g];
  }
}

// Block-wide min and max of three ints (256 threads); every thread gets them.
__device__ __forceinline__ void block_box(int (&lo)[3], int (&hi)[3], int* sh /* 24 ints */) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], off, 64));
      hi[d] = max(hi[d], __shfl_xor(hi[d], off, 64));
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sh[d * 4 + w] = lo[d];
      sh[12 + d * 4 + w] = hi[d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = min(min(sh[d * 4], sh[d * 4 + 1]), min(sh[d * 4 + 2], sh[d * 4 + 3]));
    hi[d] = max(max(sh[12 + d * 4], sh[12 + d * 4 + 1]), max(sh[12 + d * 4 + 2], sh[12 + d * 4 + 3]));
  }
  __syncthreads();  // sh is reused by the next reduction
}

// Copy the box [x0, x0+L[0]) x [y0, ...) x [z0, ...) (unwrapped) of G fields
// into the tile, node (xr, yr, zr) at ((zr L[1] + yr) L[0] + xr).  A null
// source fills its slot with zeros (padding of a 16-byte node).
template <typename RC, int G>
__device__ __forceinline__ void tile_stage(RC* tile, const double* const (&src)[G], const double (&sc)[G], int x0,
                                           int y0, int z0, const int (&L)[3], int n) {
  const int m = n - 1;
  const int rows = L[1] * L[2];
  for (int e = threadIdx.x; e < rows * L[0]; e += 256) {
    const int row = e / L[0];
    const int xr = e - row * L[0];
    const int zr = row / L[1];
    const int yr = row - zr * L[1];
    const long long gi = ((long long)((z0 + zr) & m) * n + ((y0 + yr) & m)) * n + ((x0 + xr) & m);
    RC v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] = src[g] ? RC(sc[g] * src[g][gi]) : RC(0);
    tile_put<G, RC>(tile, e, v);
  }
}

// Box of the stencils whose floors span [lo, hi] per axis: origin lo - 1,
// extent hi - lo + 4.  It fits when it is no wider than the grid plus the
// stencil and holds at most cap nodes (computed in 64 bits, so that garbage
// floors of non-finite points fail the test).
__device__ __forceinline__ bool box_fits(const int (&lo)[3], const int (&hi)[3], int n, long long cap, int (&box)[3],
                                         int (&L)[3]) {
  long long ext[3];
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ext[d] = (long long)hi[d] - (long long)lo[d] + 4;
    ok = ok && ext[d] > 0 && ext[d] <= n + 3;
    box[d] = lo[d] - 1;
    L[d] = ok ? (int)ext[d] : 1;
  }
  return ok && ext[0] * ext[1] * ext[2] <= cap;
}

}  // namespace tumor
