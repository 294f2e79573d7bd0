// Pieces shared by the 2D and 3D FFT products.
#pragma once

#include <hip/hip_runtime.h>

// Optional per-rhs flag (a converged solve): blocks of a finished rhs return
// at once.  With a map, the launch covers only the rhs listed there: block
// row blockIdx.y works on rhs map[blockIdx.y].
struct Skip {
  const int* flag;
  int stride;
  const int* map = nullptr;
  __device__ __forceinline__ bool operator()(int rhs) const { return flag && flag[(long long)rhs * stride]; }
  __device__ __forceinline__ int item(int y) const { return map ? map[y] : y; }
};

// Grid field source of the first pass: nrhs fields of n_nodes values.
template <typename T>
struct SrcGrid {
  const T* v;
  long long n_nodes;
  __device__ __forceinline__ T operator()(int rhs, long long k) const { return v[rhs * n_nodes + k]; }
};
