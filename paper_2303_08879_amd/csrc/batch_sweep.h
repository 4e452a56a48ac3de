// Batched forward sweep: many independent circuits of uneven shape (mode
// count, cutoffs, detected/undetected split) in one persistent launch.
//
// The only parallelism statement of the method is that all pivots of one
// weight are independent (Sec. 2.2); across circuits there is no dependence
// at all.  The persistent kernel therefore sweeps step S of every circuit
// together: the sweep of each circuit is cut into work items (circuit, step,
// range of units), a unit being one lattice point (Algorithm 1) or one
// (lattice point, chunk of undetected rows) (Algorithm 2); the wavefronts of
// a grid that fills the device take the items of step S from that step's
// queue, in any order (they are independent), then the grid meets at a
// barrier before step S + 1.  The eight XCDs of the device have separate L2
// caches, so publishing writes to another XCD costs an L2 write-back on the
// writer's side and an invalidation on the reader's: the barrier pays that
// once per wavefront and step, where per-item dependency tracking would pay
// it per item.  The launch is cooperative (every workgroup resident), and
// the barrier's wait is bounded: a wait that runs out sets bit 4 of the
// first circuit's status word and the grid goes on, so it always drains.
//
// The sweep kernel is compiled for a largest detected-mode count of
// Algorithm 1 circuits (MDMAX), of Algorithm 2 circuits (MDBLK) and a largest
// number of undetected block coordinates (NQMAX): (6, 5, 2) -- up to six
// modes with at most one undetected -- and (8, 8, 4), every plan.  It inlines
// the units of every smaller shape and its register budget is that of the
// largest one, so batches within (6, 5, 2) take the smaller build.
#pragma once

#include "fwd_units.h"

namespace fd {

constexpr unsigned kSpinLimit = 1u << 22;   // barrier polls (about 1 us each) before giving up
constexpr int kOutIter = 8;                 // output elements per thread of the batched permutation
constexpr int kTabBytes = 2 * (kMaxCut + 4) * 8;   // sqrt tables at the start of the sweep kernel's LDS

template <typename R>
struct BatchCirc {
  DevPlan P;
  ChunkGeo G, Gh;              // row chunks of a unit: whole-wavefront, and halved for small levels
  PrepArgs pa;
  int kind;                    // 0: Algorithm 1 (point units), 1: Algorithm 2 (block units)
  int steps;                   // sweep steps (0 when no mode is detected)
  int wmax;                    // highest weight of the undetected block fill
  cx<R>* fam[kMaxFam];         // ring base of every family (index 0 unused)
  int64_t fstride[kMaxFam];    // ring slot stride in elements
  cx<R>* f0;                   // F0 at every level (the outputs in node order)
  cx<R>* Ai;                   // interleaved symmetrised A (npos x npos), then b, then c
  const cx<R>* A;
  const cx<R>* b;
  const cx<R>* c;
  cx<R>* rho;
  const int* elist;
  const int* woff;
  int* status;
  int64_t out_elems, N;        // output elements; nodes (prod of detected cutoffs)
};

// A work item: units [u0, u1) of step `step` of circuit `circ`; `half`
// selects the halved row chunks (Algorithm 2 levels with few units, as in
// the per-circuit level launches).
struct BatchItem {
  int circ, step, u0, u1;
  int half, pad[3];
};

// Per-wavefront LDS of the sweep kernel: PN table, then (block circuits) A
// and b, then the F0 rows and bridge pivot rows of a block unit.
struct BatchLds {
  int pn_bytes, sa_bytes, wave_bytes, waves;
};

// Pointers the sweep loads from memory are generic to the compiler, which
// then emits flat loads and stores (counted by both the vector-memory and the
// LDS wait counters, so LDS waits also wait for HBM traffic).  They all point
// into device global memory: say so, and the accesses become global ones.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
// Loads a pointer stored at `slot` as a global-address-space pointer.
template <typename T>
__device__ __forceinline__ T* load_global(T* const* slot) {
  return (T*)(*reinterpret_cast<const gptr<T>*>(slot));
}

// Family pointers of one circuit at one level, computed from the ring bases.
template <typename R>
struct BatchRing {
  const BatchCirc<R>* __restrict__ C;
  int par;
  __device__ __forceinline__ cx<R>* operator[](int f) const {
    return load_global(&C->fam[f]) + (par ? C->fstride[f] : 0);
  }
};
template <typename R>
struct BatchLevel {
  BatchRing<R> rd, wr;
  const cx<R>* f0cur;
  cx<R>* f0nxt;
  const int* node;
};

template <typename R>
__device__ __forceinline__ BatchLevel<R> batch_level(const BatchCirc<R>* __restrict__ C, int S) {
  BatchLevel<R> L;
  L.rd.C = C;
  L.rd.par = (S - 1) & 1;
  L.wr.C = C;
  L.wr.par = S & 1;
  const int64_t* lvl = load_global(&C->P.lvl);
  const size_t B = (size_t)C->P.B;
  cx<R>* f0 = load_global(&C->f0);
  L.f0cur = f0 + (size_t)lvl[S] * B;
  L.f0nxt = S < C->P.smax ? f0 + (size_t)lvl[S + 1] * B : nullptr;
  const int* node = load_global(&C->P.node);
  L.node = node ? node + (size_t)lvl[S] * kNodeStride : nullptr;
  return L;
}

template <int MD, bool ODD, typename R>
__device__ __forceinline__ void run_point_item(const BatchCirc<R>* __restrict__ C, const BatchItem& I,
                                               const int* spn, const R* sq, const R* isq) {
  const BatchLevel<R> L = batch_level(C, I.step);
  const cx<R>* Ai = load_global(&C->Ai);
  const cx<R>* bi = Ai + 4 * MD * MD;
  for (int r = I.u0 + (int)(threadIdx.x & 63); r < I.u1; r += 64)
    fwd_point_unit<MD, ODD, R>(C->P, L, Ai, bi, spn, sq, isq, I.step, r);
}

template <int MD, int NQ, typename R>
__device__ __forceinline__ void run_block_item(const BatchCirc<R>* __restrict__ C, const BatchItem& I,
                                               const int* spn, const R* sq, const R* isq, const cx<R>* sA,
                                               cx<R>* lf0) {
  constexpr int NPOS = NQ + 2 * MD;
  const BatchLevel<R> L = batch_level(C, I.step);
  const ChunkGeo G = I.half ? C->Gh : C->G;
  cx<R>* lpk = lf0 + (size_t)(G.RC + 2) * G.R0;
  for (int u = I.u0; u < I.u1; ++u) {
    const int r = u / G.nchunks, ch = u - r * G.nchunks;
    fwd_block_unit<MD, NQ, R>(C->P, L, sA, sA + NPOS * NPOS, sq, isq, I.step, r, ch, G, lf0, lpk);
  }
}

template <typename R, int MDMAX, int MDBLK, int NQMAX>
__device__ __forceinline__ void run_item(const BatchCirc<R>* __restrict__ C, const BatchItem& I, const int* spn,
                                         const R* sq, const R* isq, const cx<R>* sA, cx<R>* lf0) {
  const int MD = C->P.MD;
  if (C->kind == 0) {
    const bool odd = C->P.odd != 0;
#define FD_POINT_CASE(MDV)                                         \
  case MDV:                                                        \
    if constexpr (MDV <= MDMAX) {                                  \
      if (odd)                                                     \
        run_point_item<MDV, true, R>(C, I, spn, sq, isq);          \
      else                                                         \
        run_point_item<MDV, false, R>(C, I, spn, sq, isq);         \
    }                                                              \
    break;
    switch (MD) {
      FD_POINT_CASE(1)
      FD_POINT_CASE(2)
      FD_POINT_CASE(3)
      FD_POINT_CASE(4)
      FD_POINT_CASE(5)
      FD_POINT_CASE(6)
      FD_POINT_CASE(7)
      FD_POINT_CASE(8)
      default:
        break;
    }
#undef FD_POINT_CASE
  } else {
    const bool nq4 = C->P.nq == 4;
#define FD_BLOCK_CASE(MDV)                                         \
  case MDV:                                                        \
    if constexpr (MDV <= MDBLK) {                                  \
      if constexpr (NQMAX >= 4) {                                  \
        if (nq4)                                                   \
          run_block_item<MDV, 4, R>(C, I, spn, sq, isq, sA, lf0);  \
        else                                                       \
          run_block_item<MDV, 2, R>(C, I, spn, sq, isq, sA, lf0);  \
      } else {                                                     \
        run_block_item<MDV, 2, R>(C, I, spn, sq, isq, sA, lf0);    \
      }                                                            \
    }                                                              \
    break;
    switch (MD) {
      FD_BLOCK_CASE(1)
      FD_BLOCK_CASE(2)
      FD_BLOCK_CASE(3)
      FD_BLOCK_CASE(4)
      FD_BLOCK_CASE(5)
      FD_BLOCK_CASE(6)
      FD_BLOCK_CASE(7)
      FD_BLOCK_CASE(8)
      default:
        break;
    }
#undef FD_BLOCK_CASE
  }
}

// The persistent sweep.  ctl[S] is the queue head of step S (items
// step_off[S] .. step_off[S+1]-1), ctl[nsteps] counts barrier arrivals.
template <typename R, int MDMAX, int MDBLK, int NQMAX>
__global__ __launch_bounds__(kThreads) void k_batch_fwd(const BatchCirc<R>* __restrict__ circs,
                                                        const BatchItem* __restrict__ items,
                                                        const int* __restrict__ step_off, int nsteps, unsigned* ctl,
                                                        int* status, BatchLds lds) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* sq = reinterpret_cast<R*>(smem_raw);
  R* isq = sq + (kMaxCut + 4);
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  unsigned char* wl = smem_raw + kTabBytes + (size_t)(threadIdx.x >> 6) * lds.wave_bytes;
  int* spn = reinterpret_cast<int*>(wl);
  cx<R>* sA = reinterpret_cast<cx<R>*>(wl + lds.pn_bytes);
  cx<R>* lf0 = reinterpret_cast<cx<R>*>(wl + lds.pn_bytes + lds.sa_bytes);
  int cur = -1;
  for (int S = 0; S < nsteps; ++S) {
    const int i0 = step_off[S], cnt = step_off[S + 1] - i0;
    for (;;) {
      int it = 0;
      if (lane == 0) it = (int)atomicAdd(&ctl[S], 1u);
      it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
      if (it >= cnt) break;
      const BatchItem I = items[i0 + it];
      const BatchCirc<R>* __restrict__ C = circs + I.circ;
      if (I.circ != cur) {
        wave_sync();
        const int npn = (C->P.MD + 1) * C->P.pnw;
        const int* pn = load_global(&C->P.pn);
        for (int i = lane; i < npn; i += 64) spn[i] = pn[i];
        if (C->kind) {
          const int na = C->P.npos * C->P.npos + C->P.npos;
          const cx<R>* Ai = load_global(&C->Ai);
          for (int i = lane; i < na; i += 64) sA[i] = ld(Ai + i);
        }
        wave_sync();
        cur = I.circ;
      }
      run_item<R, MDMAX, MDBLK, NQMAX>(C, I, spn, sq, isq, sA, lf0);
    }
    if (S + 1 == nsteps) break;
    // grid barrier: every wavefront's writes of step S reach memory before
    // its workgroup arrives; every wavefront drops stale lines after leaving
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned target = (unsigned)(S + 1) * gridDim.x;
      atomicAdd(&ctl[nsteps], 1u);
      unsigned spins = 0;
      while (__hip_atomic_load(&ctl[nsteps], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          atomicOr(status, 4);
          break;
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
}

// Launchers of the sweep kernel, one translation unit per MDMAX.
struct BatchSweepArgs {
  const void* circs;
  const void* items;
  const int* step_off;
  int nsteps;
  unsigned* ctl;
  int* status;
  BatchLds lds;
  int grid;
  size_t shm;
};
hipError_t batch_sweep_md6(bool c64, const BatchSweepArgs* a, int* per_cu, hipStream_t st);
hipError_t batch_sweep_md8(bool c64, const BatchSweepArgs* a, int* per_cu, hipStream_t st);

// Shared body of the launchers: with per_cu != NULL only sets the LDS limit
// and reports the resident workgroups per CU (-1 when the kernel was built
// with scratch memory: register spills to memory in a cooperative persistent
// launch are refused); otherwise launches cooperatively (the runtime refuses a
// grid that cannot be resident at once).
template <int MDMAX, int MDBLK, int NQMAX>
hipError_t batch_sweep_impl(bool c64, const BatchSweepArgs* a, int* per_cu, hipStream_t st) {
  const void* fn = c64 ? reinterpret_cast<const void*>(&k_batch_fwd<float, MDMAX, MDBLK, NQMAX>)
                       : reinterpret_cast<const void*>(&k_batch_fwd<double, MDMAX, MDBLK, NQMAX>);
  const int threads = 64 * a->lds.waves;
  if (per_cu) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    if (fa.localSizeBytes > 0) {
      *per_cu = -1;
      return hipSuccess;
    }
    if (a->shm > 65536) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)a->shm);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, threads, a->shm);
  }
  const void* circs = a->circs;
  const BatchItem* items = static_cast<const BatchItem*>(a->items);
  const int* step_off = a->step_off;
  int nsteps = a->nsteps;
  unsigned* ctl = a->ctl;
  int* status = a->status;
  BatchLds lds = a->lds;
  void* args[] = {&circs, &items, &step_off, &nsteps, &ctl, &status, &lds};
  return hipLaunchCooperativeKernel(fn, dim3(a->grid), dim3(threads), args, (unsigned)a->shm, st);
}

}  // namespace fd
