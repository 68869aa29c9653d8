// hpm_device.h -- device helpers shared by the kernels of libhpm (predicates,
// list searches, block scans, XCD-aware block order).  Not part of the ABI.
#pragma once

#include "hpm_internal.h"

namespace hpm {
namespace {

__device__ __forceinline__ bool vertex_ok(const DevGraph& g, const DevPlan* __restrict__ P, int p,
                                          int32_t v) {
  const uint32_t mask = P->vmask[p];
  if (mask == 0) return true;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c) {
    if (mask & (1u << c)) {
      const int32_t x = g.vcol[c][v];
      ok = ok && x >= P->vlo[p][c] && x <= P->vhi[p][c];
    }
  }
  return ok;
}

__device__ __forceinline__ bool arc_ok(const DevGraph& g, const DevPlan* __restrict__ P, int p,
                                       int q, int32_t e) {
  const uint32_t mask = P->amask[p][q];
  if (mask == 0) return true;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c) {
    if (mask & (1u << c)) {
      const int32_t x = g.ecol[c][e];
      ok = ok && x >= P->alo[p][q][c] && x <= P->ahi[p][q][c];
    }
  }
  return ok;
}

// Same predicate for the arc at in-CSR position j (columns stored in in-CSR order).
__device__ __forceinline__ bool arc_ok_in(const DevGraph& g, const DevPlan* __restrict__ P, int p,
                                          int q, int32_t j) {
  const uint32_t mask = P->amask[p][q];
  if (mask == 0) return true;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c) {
    if (mask & (1u << c)) {
      const int32_t x = g.ecol_in[c][j];
      ok = ok && x >= P->alo[p][q][c] && x <= P->ahi[p][q][c];
    }
  }
  return ok;
}

// Index of key in the ascending run a[lo, hi), or -1.
__device__ __forceinline__ int32_t find_in(const int32_t* __restrict__ a, int32_t lo, int32_t hi,
                                           int32_t key) {
  int32_t l = lo, h = hi;
  while (l < h) {
    const int32_t mid = l + ((h - l) >> 1);
    if (a[mid] < key)
      l = mid + 1;
    else
      h = mid;
  }
  return (l < hi && a[l] == key) ? l : -1;
}

// Orders LDS traffic of one wavefront (a compiler barrier plus wave-scope fences).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First x in [lo, hi) with a[x] >= key (upper == false) or a[x] > key
// (upper == true), hi if none.  Called by all 64 lanes of a wavefront with the
// same arguments: a 64-ary search, so a list of length L costs about
// log64(L) + 1 dependent loads instead of log2(L).
template <typename T>
__device__ __forceinline__ int32_t wave_bound(const T* __restrict__ a, int32_t lo, int32_t hi,
                                              T key, bool upper) {
  const int lane = threadIdx.x & 63;
  while (hi - lo > 64) {
    const int32_t step = (hi - lo + 63) >> 6;
    const int32_t idx = lo + lane * step;
    bool before = false;
    if (idx < hi) {
      const T v = a[idx];
      before = upper ? (v <= key) : (v < key);
    }
    const int cnt = __popcll(__ballot(before));  // the samples before the bound
    if (cnt == 0) return lo;
    const int32_t nhi = lo + cnt * step;
    lo = lo + (cnt - 1) * step + 1;
    hi = nhi < hi ? nhi : hi;
  }
  const int32_t idx = lo + lane;
  bool before = false;
  if (idx < hi) {
    const T v = a[idx];
    before = upper ? (v <= key) : (v < key);
  }
  return lo + __popcll(__ballot(before));
}

// Index of key in the ascending LDS run a[0, len), or -1.
__device__ __forceinline__ int32_t lds_find(const int32_t* a, int32_t len, int32_t key) {
  int32_t l = 0, h = len;
  while (l < h) {
    const int32_t mid = (l + h) >> 1;
    if (a[mid] < key)
      l = mid + 1;
    else
      h = mid;
  }
  return (l < len && a[l] == key) ? l : -1;
}

// Position of key in the ascending run a[lo, hi), or -1.  Must be called by the
// whole wavefront with the same lo, hi and key window [kmin, kmax] (every
// active lane's key lies in it).  The run is first cut to the window; if what
// is left has at most kWaveList entries it is copied into the wavefront's LDS
// buffer wl with coalesced loads and each lane binary-searches it there,
// otherwise each lane searches the cut run in global memory.  Lanes with
// active == false take part in the copy and return -1.
__device__ __forceinline__ int32_t wave_member(const int32_t* __restrict__ a, int32_t lo,
                                               int32_t hi, int32_t key, int32_t kmin,
                                               int32_t kmax, bool active, int32_t* wl, int lane) {
  if (hi - lo > kWaveList) {
    lo = wave_bound<int32_t>(a, lo, hi, kmin, false);
    hi = wave_bound<int32_t>(a, lo, hi, kmax, true);
  }
  const int32_t len = hi - lo;
  if (len <= kWaveList) {
    wave_sync();  // earlier readers of wl are done
    for (int32_t t = lane; t < len; t += 64) wl[t] = a[lo + t];
    wave_sync();
    if (!active) return -1;
    const int32_t x = lds_find(wl, len, key);
    return x >= 0 ? lo + x : -1;
  }
  return active ? find_in(a, lo, hi, key) : -1;
}

// Block-wide exclusive scan of one value per thread; *total gets the sum.
// Uses lds[kWaves + 1]; ends with a barrier so lds may be reused.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* lds, T* total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  T v = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) lds[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      const T t = lds[i];
      lds[i] = s;
      s += t;
    }
    lds[kWaves] = s;
  }
  __syncthreads();
  const T res = lds[wid] + v - x;
  *total = lds[kWaves];
  __syncthreads();
  return res;
}

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* lds) {
  T tot;
  (void)block_exclusive_scan<T>(x, lds, &tot);
  return tot;
}

// Logical block id such that consecutive ids run on the same XCD (blocks are
// dispatched round-robin over the 8 XCDs), so neighbouring tiles -- which
// share rows and adjacency lists -- share an L2.  Requires gridDim.x % 8 == 0.
__device__ __forceinline__ int64_t xcd_block_id() {
  const int64_t b = blockIdx.x;
  const int64_t per = gridDim.x >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ bool test_bit(const uint32_t* __restrict__ bits, int32_t v) {
  return ((bits[v >> 5] >> (v & 31)) & 1u) != 0;
}

}  // namespace
}  // namespace hpm
