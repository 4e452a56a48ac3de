// Device-side helpers shared by the forward and reverse kernels: complex
// arithmetic on interleaved (re, im) pairs, the level rank / unrank of the
// detected lattice, and the per-launch pointer tables.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fd_internal.h"

namespace fd {

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cmake(R x, R y) {
  cx<R> r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename R>
__device__ __forceinline__ cx<R> czero() {
  return cmake<R>(R(0), R(0));
}
// acc += a * b
template <typename R>
__device__ __forceinline__ void cfma(cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename R>
__device__ __forceinline__ void cfma_conj(cx<R>& acc, const cx<R>& a, const cx<R>& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
template <typename R>
__device__ __forceinline__ cx<R> cscale(const cx<R>& a, R s) {
  return cmake<R>(a.x * s, a.y * s);
}
template <typename R>
__device__ __forceinline__ cx<R> cadd(const cx<R>& a, const cx<R>& b) {
  return cmake<R>(a.x + b.x, a.y + b.y);
}

// Value and tangent of one amplitude (forward mode, Sec. 2.5): the tangent
// of an element stored at p lives dT bytes after it.
template <typename R>
struct dual {
  cx<R> v, t;
};
template <typename T>
__device__ __forceinline__ T* tangent_of(T* p, int64_t dT) {
  using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<Byte*>(p) + dT);
}
// acc += a * x for coefficient a and operand x, both with tangents:
// (a x)' = a' x + a x'
template <typename R>
__device__ __forceinline__ void cfma(dual<R>& acc, const dual<R>& a, const dual<R>& x) {
  cfma(acc.v, a.v, x.v);
  cfma(acc.t, a.t, x.v);
  cfma(acc.t, a.v, x.t);
}
template <typename R>
__device__ __forceinline__ dual<R> cscale(const dual<R>& a, R s) {
  dual<R> r;
  r.v = cscale(a.v, s);
  r.t = cscale(a.t, s);
  return r;
}

// Element idx of one level's slab of a family through a 32-bit byte offset
// from the level's base: the memory instruction then takes the base from
// scalar registers and one 32-bit offset register instead of a 64-bit
// address per lane (fewer registers and address instructions).  The planner
// keeps every level of a plan below 2^28 amplitudes, so the offset
// cannot wrap.
template <typename T>
__device__ __forceinline__ T* at32(T* base, uint32_t idx) {
  using Byte = typename std::conditional<std::is_const<T>::value, const unsigned char, unsigned char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<Byte*>(base) + (uint64_t)(idx * (uint32_t)sizeof(T)));
}

// 16-byte / 8-byte vector load and store of one complex element.
__device__ __forceinline__ cx<double> ld(const cx<double>* p) {
  double2 v = *reinterpret_cast<const double2*>(p);
  return cmake<double>(v.x, v.y);
}
__device__ __forceinline__ cx<float> ld(const cx<float>* p) {
  float2 v = *reinterpret_cast<const float2*>(p);
  return cmake<float>(v.x, v.y);
}
__device__ __forceinline__ void st(cx<double>* p, const cx<double>& a) {
  *reinterpret_cast<double2*>(p) = make_double2(a.x, a.y);
}
__device__ __forceinline__ void st(cx<float>* p, const cx<float>& a) {
  *reinterpret_cast<float2*>(p) = make_float2(a.x, a.y);
}

// Zero, load and store of a sweep element: one complex amplitude, or an
// amplitude with its tangent (dT bytes further on).
template <typename E>
struct ET;
template <typename R>
struct ET<cx<R>> {
  static __device__ __forceinline__ cx<R> zero() { return czero<R>(); }
  static __device__ __forceinline__ cx<R> load(const cx<R>* p, int64_t) { return ld(p); }
  static __device__ __forceinline__ void store(cx<R>* p, const cx<R>& v, int64_t) { st(p, v); }
};
template <typename R>
struct ET<dual<R>> {
  static __device__ __forceinline__ dual<R> zero() {
    dual<R> r;
    r.v = r.t = czero<R>();
    return r;
  }
  static __device__ __forceinline__ dual<R> load(const cx<R>* p, int64_t dT) {
    dual<R> r;
    r.v = ld(p);
    r.t = ld(tangent_of(p, dT));
    return r;
  }
  static __device__ __forceinline__ void store(cx<R>* p, const dual<R>& v, int64_t dT) {
    st(p, v.v);
    st(tangent_of(p, dT), v.t);
  }
};

// Per-launch node-0 pointers of every family at the levels a sweep step
// touches: rd = level S-1 (reads), wr = level S (writes), plus F0 at S and
// S+1, and the node records of level S (Algorithm 2 plans).  Entries of
// families not used by the schedule are null.
template <typename R>
struct LevelPtrs {
  const cx<R>* rd[kMaxFam];
  cx<R>* wr[kMaxFam];
  const cx<R>* f0cur;
  cx<R>* f0nxt;
  const int* node;
};

// Node record of lattice point r of the level: m, the ranks of m - 1_j at
// level S-1 and of m + 1_j at level S+1 (one scalar load per unit).
template <int MD>
__device__ __forceinline__ void node_record(const int* node, int r, int* m, int* rdn, int* rup) {
  const int* nr = node + (size_t)r * kNodeStride;
#pragma unroll
  for (int j = 0; j < MD; ++j) {
    m[j] = nr[j];
    rdn[j] = nr[MD + j];
    rup[j] = nr[2 * MD + j];
  }
}

// Orders LDS traffic between the lanes of one wavefront: LDS operations of a
// wavefront execute in order, so only compiler reordering has to be stopped.
__device__ __forceinline__ void wave_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Orders a unit's phases: LDS traffic within the wavefront, or (WG: rows in
// global memory, or a unit shared by several wavefronts) a workgroup-scope
// fence and barrier, which makes one lane's writes visible to every lane of
// the workgroup.
template <bool WG>
__device__ __forceinline__ void unit_sync() {
  if constexpr (WG)
    __syncthreads();
  else
    wave_sync();
}

// Compiler-only barrier: memory accesses are not moved across it, so the
// compiler cannot overlap consecutive loop iterations whose live values would
// otherwise push the register count past an occupancy step.
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Coordinate q of an undetected-block entry: floor(rem / ustride[q]) for
// 0 <= rem < 16384 without an integer division.  (rem + 1/2) / ustride lies
// at least 1 / (2 ustride) >= 2^-15 away from an integer, while one double
// multiply by the rounded reciprocal is off by under 2^-37 for rem < 16384,
// so truncating the product is exact.
__device__ __forceinline__ int ucoord(const DevPlan& P, int rem, int q) { return (int)((rem + 0.5) * P.uinv[q]); }

// PN[d][x] for x in [-1, smax+1]; table row width pnw.
__device__ __forceinline__ int pnv(const int* spn, int pnw, int d, int x) { return spn[d * pnw + x + 1]; }

// Node-order position (level offset + rank) of the detected lattice point
// whose C-order index is x (last detected mode fastest), 0 <= x < prod CD <
// 2^31.  Digits come last mode first, each from one double multiply: (x +
// 1/2) / C lies at least 1 / (2 C) >= 2^-7 from an integer and the rounded
// product is off by under 2^-21, so truncation gives floor(x / C) exactly;
// the suffix sums the rank needs accumulate in the same pass.
__device__ __forceinline__ int64_t node_of_cindex(const DevPlan& P, const int* spn, const int64_t* slv, int x) {
  const int pnw = P.pnw;
  int rem = x, suf = 0, rank = 0;
  for (int d = P.MD - 1; d >= 0; --d) {
    const int q = (int)((rem + 0.5) * P.cinv[d]);
    const int nd = rem - q * P.CD[d];
    rem = q;
    suf += nd;
    rank += pnv(spn, pnw, d + 1, suf) - pnv(spn, pnw, d + 1, suf - nd);
  }
  return slv[suf] + rank;
}

// Lattice point of rank r at level S (lexicographic, first mode slowest).
// s[d] = S - sum_{i<d} m_i.  The count of points of sub-box d+1 whose sum
// lies in (s - v, s] is PN[d+1][s] - PN[d+1][s-v]; m_d is the largest v with
// that count <= r (binary search; counts are monotone in v).
template <int MD>
__device__ __forceinline__ void unrank(const int* spn, int pnw, const int* C, int S, int r, int* m, int* s) {
  s[0] = S;
#pragma unroll
  for (int d = 0; d < MD - 1; ++d) {
    const int sd = s[d];
    const int base = pnv(spn, pnw, d + 1, sd);
    const int target = base - r;
    int lo = 0, hi = min(C[d] - 1, sd);
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pnv(spn, pnw, d + 1, sd - mid) >= target)
        lo = mid;
      else
        hi = mid - 1;
    }
    m[d] = lo;
    r -= base - pnv(spn, pnw, d + 1, sd - lo);
    s[d + 1] = sd - lo;
  }
  m[MD - 1] = s[MD - 1];
  s[MD] = 0;
}

// Ranks of the neighbours of m: rdn[j] = rank of m - 1_j at level S-1 (valid
// when m_j > 0) and rup[K] = rank of m + 1_K at level S+1 (valid when
// m_<K = 0).  With U_d = PN[d+1][s_d] - PN[d+1][s_{d+1}] (the terms of the
// rank of m), the rank of m - 1_j shifts the partial sums of every mode
// before j and of j itself by one; modes after j keep their terms.
template <int MD>
__device__ __forceinline__ void neighbour_ranks(const int* spn, int pnw, const int* s, int* rdn, int* rup) {
  int U[MD];
#pragma unroll
  for (int d = 0; d < MD; ++d) U[d] = pnv(spn, pnw, d + 1, s[d]) - pnv(spn, pnw, d + 1, s[d + 1]);
  int suff = 0;
  int suffU[MD];
#pragma unroll
  for (int d = MD - 1; d >= 0; --d) {
    suffU[d] = suff;
    suff += U[d];
  }
  int pref = 0;
#pragma unroll
  for (int j = 0; j < MD; ++j) {
    rdn[j] = pref + (pnv(spn, pnw, j + 1, s[j] - 1) - pnv(spn, pnw, j + 1, s[j + 1])) + suffU[j];
    rup[j] = (pnv(spn, pnw, j + 1, s[j] + 1) - pnv(spn, pnw, j + 1, s[j + 1])) + suffU[j];
    pref += pnv(spn, pnw, j + 1, s[j] - 1) - pnv(spn, pnw, j + 1, s[j + 1] - 1);
  }
}

}  // namespace fd
