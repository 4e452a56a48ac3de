// Reverse sweep of Algorithm 2 plans: the block kernel and its per-level
// launch (the point kernels, the fills and the sweep driver are in
// kernels_vjp.hip).
#include <algorithm>

#include "vjp_common.h"

namespace fd {

// ---------------------------------------------------------------------------
// Algorithm 2 reverse step.  One workgroup of WV wavefronts per (lattice
// point, chunk of rows of the first undetected coordinate).  The undetected
// neighbour terms make the cotangent of a pivot entry pull from the entry one
// row below, so a chunk recomputes the target cotangents of two rows past its
// own (bridge pivots: the rows its diagonal pivot needs; diagonal pivot: one
// row), without storing them.  Four wavefronts with chunks of about 128
// entries each (48 on levels with few units) make that recomputation a small
// part of a chunk; plans whose four-wavefront staging does not fit the LDS,
// and streamed rows, run two wavefronts with 64-entry chunks (the chunk
// heights are set by the planner).
// Abar records are folded per wavefront: each wave stages NB records at a
// time in its own LDS region and reduces them on the matrix cores into its
// own accumulators; the waves' tables are added in wave order at the end.
// ---------------------------------------------------------------------------
template <int MD, int NQ, typename R, int NB, bool ST, int WV>
__global__ __launch_bounds__(64 * WV) void k_vjp_block(DevPlan P, VjpPtrs<R> V, const cx<R>* __restrict__ Ai,
                                                        const cx<R>* __restrict__ bi, int S, int nwork,
                                                        ChunkGeo G, double2* __restrict__ partial) {
  constexpr int NPD = 2 * MD;
  constexpr int NPOS = NQ + NPD;
  constexpr int NR = NPOS + 1;
  constexpr int NPAIR = NPD * NR;
  // Abar / bbar records (the target cotangents h and the read values x of
  // one entry) are staged NB lanes at a time and reduced on the matrix cores,
  // as in the point kernel; the read values of a lane are formed when its
  // batch is staged.
  constexpr int RS = NB + 1;
  static_assert(NB % 4 == 0 && 64 % NB == 0, "batches of whole MFMA steps that tile the wavefront");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int B = P.B, R0 = G.R0, RC = G.RC;
  const int nrow1 = (RC + 1) * R0, nrow2 = (RC + 2) * R0;
  // entries each lane reads back only itself (same entry-to-lane map in every
  // loop of a unit): the workgroup's private slot in global memory, which
  // leaves the LDS to the shared rows and raises the wavefronts per CU
  cx<R>* gpk = V.priv + (size_t)blockIdx.x * V.priv_stride;   // MD x rows [k0, k1+1)
  cx<R>* gbv = gpk + (size_t)MD * nrow1;                       // rows [k0, k1+1)
  cx<R>* g0a = gbv + nrow1;                                    // own rows
  // the forward pivot rows [k0-1, k1) and the undetected-neighbour terms of
  // NQ x rows [k0, k1+2): in LDS, or (ST, blocks whose rows do not fit) the
  // pivot rows read from HBM where they lie and the terms in the private
  // slot after the own rows (the __syncthreads between phases are
  // workgroup-scope fences)
  cx<R>* lfw = reinterpret_cast<cx<R>*>(smem_raw);
  cx<R>* qv = ST ? g0a + (size_t)RC * R0 : lfw + nrow1;
  cx<R>* rec = ST ? lfw : qv + (size_t)NQ * nrow2;   // waves x RS x (NPD + NR)
  cx<R>* sA = rec + (size_t)WV * RS * (NPD + NR);   // A (NPOS x NPOS) then b (NPOS)
  const cx<R>* sb = sA + NPOS * NPOS;
  R* sq = reinterpret_cast<R*>(sA + NPOS * NPOS + NPOS);
  R* isq = sq + (kMaxCut + 4);
  for (int v = threadIdx.x; v < kMaxCut + 4; v += blockDim.x) {
    sq[v] = sqrt(R(v));
    isq[v] = v ? R(1) / sqrt(R(v)) : R(0);
  }
  for (int i = threadIdx.x; i < NPOS * NPOS + NPOS; i += blockDim.x) sA[i] = ld(Ai + i);
  // (one wavefront per workgroup: every phase of a unit starts with a staging
  // loop and a barrier before it reads these tables)
  cx<R>* recw = rec + (size_t)(threadIdx.x >> 6) * RS * (NPD + NR);
  const int lane = threadIdx.x & 63;
  MfmaAcc<(NR + 15) / 16> acc;
  mfma_acc_zero(acc);

  for (int w = blockIdx.x; w < nwork * G.nchunks; w += gridDim.x) {
    const int r = w / G.nchunks, c = w - r * G.nchunks;
    const int k0 = c * RC, k1 = min(G.C0, k0 + RC);
    const int e_own0 = k0 * R0, e_own1 = k1 * R0;
    int m[MD], rdn[MD], rup[MD];
    node_record<MD>(V.node, r, m, rdn, rup);
    int K0 = MD;
#pragma unroll
    for (int d = MD - 1; d >= 0; --d)
      if (m[d] > 0) K0 = d;
    const size_t rB = (size_t)r * B;
    // forward pivot row entry e of the current phase's pivot block
    const cx<R>* fsrc = nullptr;
    auto LF = [&](int e) -> cx<R> {
      if constexpr (ST)
        return ld(at32(fsrc, (uint32_t)e));
      else
        return lfw[e - (k0 - 1) * R0];
    };
    for (int e = e_own0 + threadIdx.x; e < e_own1; e += blockDim.x) g0a[e - e_own0] = ld(at32(V.d0cur, (uint32_t)(r * B + e)));

#pragma unroll
    for (int K = 0; K < MD; ++K) {
      if (K > K0 || m[K] > P.CD[K] - 2) continue;   // uniform
      fsrc = V.fcur[fam_f1k(K)] + rB;
      if constexpr (!ST) {
        const int e0 = max(0, k0 - 1) * R0;
        for (int e = e0 + threadIdx.x; e < e_own1; e += blockDim.x) lfw[e - (k0 - 1) * R0] = ld(fsrc + e);
      }
      __syncthreads();
      const int eq1 = min(G.C0, k1 + 2) * R0, eb1 = min(G.C0, k1 + 1) * R0;
      const bool has_diag_reader = (K > 0) || (m[0] + 1 <= P.CD[0] - 2);
      for (int base = e_own0; base < eq1; base += blockDim.x) {
        const int e = base + threadIdx.x;
        const bool live = e < eq1, own = e < e_own1;
        // the record's read values, loaded by every lane with the cotangents
        // (one memory round trip for both, and for both record batches)
        const bool rec_ok = live && own;
        cx<R> xr[NR];
#pragma unroll
        for (int l = 0; l < NR; ++l) xr[l] = czero<R>();
        if (rec_ok) {
          int rem = e;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int kq = ucoord(P, rem, q);
            rem -= kq * P.ustride[q];
            if (kq > 0) xr[q] = cscale(LF(e - P.ustride[q]), sq[kq]);
          }
          xr[NPOS] = LF(e);
          xr[NQ + 2 * K] = cscale(ld(at32(V.fcur[0], (uint32_t)(r * B + e))), sq[m[K] + 1]);
          if (m[K] > 0)
            xr[NQ + 2 * K + 1] = cscale(ld(at32(V.fprev[fam_f2(MD, K)], (uint32_t)(rdn[K] * B + e))), sq[m[K]]);
#pragma unroll
          for (int j = K + 1; j < MD; ++j) {
            if (m[j] > 0) {
              xr[NQ + 2 * j] = cscale(ld(at32(V.fprev[fam_1001(MD, K, j)], (uint32_t)(rdn[j] * B + e))), sq[m[j]]);
              xr[NQ + 2 * j + 1] = cscale(ld(at32(V.fprev[fam_1010(MD, K, j)], (uint32_t)(rdn[j] * B + e))), sq[m[j]]);
            }
          }
        }
        cx<R> h[NPD];
#pragma unroll
        for (int i = 0; i < NPD; ++i) h[i] = czero<R>();
        if (live) {
          h[2 * K + 1] = cscale(ld(at32(V.gf0nxt, (uint32_t)(rup[K] * B + e))), isq[m[K] + 1]);
          if (m[K] <= P.CD[K] - 3) h[2 * K] = cscale(ld(at32(V.gcur[fam_f2(MD, K)], (uint32_t)(r * B + e))), isq[m[K] + 2]);
#pragma unroll
          for (int j = K + 1; j < MD; ++j) {
            if (m[j] <= P.CD[j] - 2) {
              h[2 * j] = cscale(ld(at32(V.gcur[fam_1010(MD, K, j)], (uint32_t)(r * B + e))), isq[m[j] + 1]);
              h[2 * j + 1] = cscale(ld(at32(V.gcur[fam_1001(MD, K, j)], (uint32_t)(r * B + e))), isq[m[j] + 1]);
            }
          }
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            cx<R> u = czero<R>();
#pragma unroll
            for (int i = 2 * K; i < NPD; ++i) cfma_conj(u, sA[(NQ + i) * NPOS + q], h[i]);
            qv[(size_t)q * nrow2 + (e - e_own0)] = u;
          }
          if (e < eb1) {
            cx<R> gb = czero<R>();
#pragma unroll
            for (int i = 2 * K; i < NPD; ++i) cfma_conj(gb, sb[NQ + i], h[i]);
            gbv[e - e_own0] = gb;
          }
          if (own) {
#pragma unroll
            for (int l = 2 * K; l < NPD; ++l) {
              const int j = l >> 1;
              if (l != 2 * K && m[j] == 0) continue;
              cx<R> u = czero<R>();
#pragma unroll
              for (int i = 2 * K; i < NPD; ++i) cfma_conj(u, sA[(NQ + i) * NPOS + NQ + l], h[i]);
              if (l == 2 * K) {
                g0a[e - e_own0] = cadd(g0a[e - e_own0], cscale(u, sq[m[K] + 1]));
              } else if (l == 2 * K + 1) {
                st(at32(V.gprev[fam_f2(MD, K)], (uint32_t)(rdn[K] * B + e)), cscale(u, sq[m[K]]));
              } else {
                st(at32(V.gprev[(l & 1) ? fam_1010(MD, K, j) : fam_1001(MD, K, j)], (uint32_t)(rdn[j] * B + e)),
                   cscale(u, sq[m[j]]));
              }
            }
          }
        }
        // Abar records of the own entries, NB lanes at a time
#pragma unroll 1
        for (int qb = 0; qb < 64 / NB; ++qb) {
          const bool grp = (lane / NB) == qb;
          if (__ballot(rec_ok && grp) == 0ull) continue;   // uniform over the wave
          if (grp) {
            const int col = lane - qb * NB;
#pragma unroll
            for (int l = 0; l < NR; ++l) recw[(NPD + l) * RS + col] = xr[l];
#pragma unroll
            for (int i = 0; i < NPD; ++i) recw[i * RS + col] = rec_ok ? h[i] : czero<R>();
          }
          wave_sync();
          wave_accum_mfma<R, NPD, NR, NB>(recw, acc);
          wave_sync();
        }
      }
      __syncthreads();
      // total cotangent of the bridge pivot block F1k(K)(m), rows [k0, k1+1)
      for (int e = e_own0 + threadIdx.x; e < eb1; e += blockDim.x) {
        int rem = e;
        const int le = e - e_own0;
        cx<R> v = gbv[le];
        if (has_diag_reader) v = cadd(v, ld(at32(V.gcur[fam_f1k(K)], (uint32_t)(r * B + e))));
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int kq = ucoord(P, rem, q);
          rem -= kq * P.ustride[q];
          if (kq + 1 < P.udims[q]) v = cadd(v, cscale(qv[(size_t)q * nrow2 + le + P.ustride[q]], sq[kq + 1]));
        }
        gpk[(size_t)K * nrow1 + le] = v;
      }
      __syncthreads();
    }

    if (m[0] <= P.CD[0] - 2) {
      fsrc = V.fcur[0] + rB;
      if constexpr (!ST) {
        const int e0 = max(0, k0 - 1) * R0;
        for (int e = e0 + threadIdx.x; e < e_own1; e += blockDim.x) lfw[e - (k0 - 1) * R0] = ld(fsrc + e);
      }
      __syncthreads();
      const int eq1 = min(G.C0, k1 + 1) * R0;
      for (int base = e_own0; base < eq1; base += blockDim.x) {
        const int e = base + threadIdx.x;
        const bool live = e < eq1, own = e < e_own1;
        // the record's read values, loaded with the cotangents
        const bool rec_ok = live && own;
        cx<R> xr[NR];
#pragma unroll
        for (int l = 0; l < NR; ++l) xr[l] = czero<R>();
        if (rec_ok) {
          int rem = e;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int kq = ucoord(P, rem, q);
            rem -= kq * P.ustride[q];
            if (kq > 0) xr[q] = cscale(LF(e - P.ustride[q]), sq[kq]);
          }
          xr[NPOS] = LF(e);
#pragma unroll
          for (int j = 0; j < MD; ++j) {
            if (m[j] > 0) {
              xr[NQ + 2 * j] = cscale(ld(at32(V.fprev[fam_f1b(MD, j)], (uint32_t)(rdn[j] * B + e))), sq[m[j]]);
              xr[NQ + 2 * j + 1] = cscale(ld(at32(V.fprev[fam_f1k(j)], (uint32_t)(rdn[j] * B + e))), sq[m[j]]);
            }
          }
        }
        cx<R> h[NPD];
#pragma unroll
        for (int i = 0; i < NPD; ++i) h[i] = czero<R>();
        if (live) {
          const int le = e - e_own0;
#pragma unroll
          for (int j = 0; j < MD; ++j) {
            if (j == 0 || m[j] <= P.CD[j] - 2) {
              const bool bridge = j <= K0 && m[j] <= P.CD[j] - 2;
              const cx<R> gt = bridge ? gpk[(size_t)j * nrow1 + le] : ld(at32(V.gcur[fam_f1k(j)], (uint32_t)(r * B + e)));
              h[2 * j] = cscale(gt, isq[m[j] + 1]);
            }
            const bool okb = (j == 0) ? (m[0] <= P.CD[0] - 3) : (m[j] <= P.CD[j] - 2);
            if (okb) h[2 * j + 1] = cscale(ld(at32(V.gcur[fam_f1b(MD, j)], (uint32_t)(r * B + e))), isq[m[j] + 1]);
          }
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            cx<R> u = czero<R>();
#pragma unroll
            for (int i = 0; i < NPD; ++i) cfma_conj(u, sA[(NQ + i) * NPOS + q], h[i]);
            qv[(size_t)q * nrow2 + le] = u;
          }
          if (own) {
#pragma unroll
            for (int l = 0; l < NPD; ++l) {
              const int j = l >> 1;
              if (m[j] == 0) continue;
              cx<R> u = czero<R>();
#pragma unroll
              for (int i = 0; i < NPD; ++i) cfma_conj(u, sA[(NQ + i) * NPOS + NQ + l], h[i]);
              st(at32(V.gprev[(l & 1) ? fam_f1k(j) : fam_f1b(MD, j)], (uint32_t)(rdn[j] * B + e)), cscale(u, sq[m[j]]));
            }
            cx<R> gb = czero<R>();
#pragma unroll
            for (int i = 0; i < NPD; ++i) cfma_conj(gb, sb[NQ + i], h[i]);
            g0a[le] = cadd(g0a[le], gb);
          }
        }
        // Abar records of the own entries, NB lanes at a time
#pragma unroll 1
        for (int qb = 0; qb < 64 / NB; ++qb) {
          const bool grp = (lane / NB) == qb;
          if (__ballot(rec_ok && grp) == 0ull) continue;   // uniform over the wave
          if (grp) {
            const int col = lane - qb * NB;
#pragma unroll
            for (int l = 0; l < NR; ++l) recw[(NPD + l) * RS + col] = xr[l];
#pragma unroll
            for (int i = 0; i < NPD; ++i) recw[i * RS + col] = rec_ok ? h[i] : czero<R>();
          }
          wave_sync();
          wave_accum_mfma<R, NPD, NR, NB>(recw, acc);
          wave_sync();
        }
      }
      __syncthreads();
      for (int e = e_own0 + threadIdx.x; e < e_own1; e += blockDim.x) {
        int rem = e;
        const int le = e - e_own0;
        cx<R> v = g0a[le];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int kq = ucoord(P, rem, q);
          rem -= kq * P.ustride[q];
          if (kq + 1 < P.udims[q]) v = cadd(v, cscale(qv[(size_t)q * nrow2 + le + P.ustride[q]], sq[kq + 1]));
        }
        g0a[le] = v;
      }
    }
    for (int e = e_own0 + threadIdx.x; e < e_own1; e += blockDim.x) st(at32(V.gcur[0], (uint32_t)(r * B + e)), g0a[e - e_own0]);
    __syncthreads();
  }
  // fold the waves' pair tables (in wave order) into this block's slot
  cx<double>* red = reinterpret_cast<cx<double>*>(smem_raw);
  __syncthreads();
  mfma_acc_store<NPD, NR, NR>(acc, red + (size_t)(threadIdx.x >> 6) * NPAIR);
  __syncthreads();
  double2* slot = partial + (size_t)blockIdx.x * (NPOS * NR);
  for (int p = threadIdx.x; p < NPAIR; p += blockDim.x) {
    const int i = p / NR, l = p - (p / NR) * NR;
    const int q = (NQ + i) * NR + l;
    double sx = 0.0, sy = 0.0;
    for (int wv = 0; wv < WV; ++wv) {
      sx += red[(size_t)wv * NPAIR + p].x;
      sy += red[(size_t)wv * NPAIR + p].y;
    }
    const double2 v = slot[q];
    slot[q] = make_double2(v.x + sx, v.y + sy);
  }
}

template <int MD, int NQ, typename R, bool ST, int WV>
static void launch_vjp_block_w(size_t shm, int grid, hipStream_t st, const DevPlan& P, const VjpPtrs<R>& Vp,
                               const cx<R>* Ai, const cx<R>* bi, int S, int nwork, const ChunkGeo& G,
                               double2* partial) {
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vjp_block<MD, NQ, R, kBlockBatch, ST, WV>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  hipLaunchKernelGGL((k_vjp_block<MD, NQ, R, kBlockBatch, ST, WV>), dim3(grid), dim3(64 * WV), shm, st, P, Vp, Ai,
                     bi, S, nwork, G, partial);
}
template <int MD, int NQ, typename R, bool ST>
static void launch_vjp_block_k(int waves, size_t shm, int grid, hipStream_t st, const DevPlan& P,
                               const VjpPtrs<R>& Vp, const cx<R>* Ai, const cx<R>* bi, int S, int nwork,
                               const ChunkGeo& G, double2* partial) {
  if constexpr (!ST)
    if (waves == kVjpWaves)
      return launch_vjp_block_w<MD, NQ, R, ST, kVjpWaves>(shm, grid, st, P, Vp, Ai, bi, S, nwork, G, partial);
  launch_vjp_block_w<MD, NQ, R, ST, kVjpWavesLds>(shm, grid, st, P, Vp, Ai, bi, S, nwork, G, partial);
}

template <typename R>
hipError_t launch_vjp_block_level(const Plan& Pl, const DevPlan& P, const VjpPtrs<R>& Vp, const cx<R>* Ai,
                                  const cx<R>* bi, int S, int nwork, double2* partial, hipStream_t st) {
  const int MD = Pl.MD;
  // as in the forward sweep: shorter row chunks on levels with few units
  const ChunkGeo G = vjp_geo(Pl, nwork);
  const size_t shm = vjp_lds_bytes_for(Pl, G);
  if (shm > kMaxLds) return hipErrorInvalidConfiguration;   // rejected before the sweep
  // streamed rows: private slots for at most kStreamSlots workgroups
  const int grid = (int)std::min<int64_t>((int64_t)nwork * G.nchunks,
                                          Pl.st_vjp ? kStreamSlots : kPartialSlots - 1);
#define FD_VJP_BLOCK_NQ(MDV, NQV)                                                                  \
  if (Pl.st_vjp)                                                                                   \
    launch_vjp_block_k<MDV, NQV, R, true>(Pl.vjp_waves, shm, grid, st, P, Vp, Ai, bi, S, nwork, G, partial); \
  else                                                                                             \
    launch_vjp_block_k<MDV, NQV, R, false>(Pl.vjp_waves, shm, grid, st, P, Vp, Ai, bi, S, nwork, G, partial);
#define FD_VJP_BLOCK(MDV)        \
  case MDV:                      \
    if (Pl.nq == 2) {            \
      FD_VJP_BLOCK_NQ(MDV, 2)    \
    } else if (Pl.nq == 4) {     \
      FD_VJP_BLOCK_NQ(MDV, 4)    \
    } else {                     \
      FD_VJP_BLOCK_NQ(MDV, 6)    \
    }                            \
    break;
  switch (MD) {
    FD_VJP_BLOCK(1)
    FD_VJP_BLOCK(2)
    FD_VJP_BLOCK(3)
    FD_VJP_BLOCK(4)
    FD_VJP_BLOCK(5)
    FD_VJP_BLOCK(6)
    FD_VJP_BLOCK(7)
    FD_VJP_BLOCK(8)
    default:
      return hipErrorInvalidValue;
  }
#undef FD_VJP_BLOCK
#undef FD_VJP_BLOCK_NQ
  return hipSuccess;
}

template hipError_t launch_vjp_block_level<float>(const Plan&, const DevPlan&, const VjpPtrs<float>&,
                                                  const cx<float>*, const cx<float>*, int, int, double2*,
                                                  hipStream_t);
template hipError_t launch_vjp_block_level<double>(const Plan&, const DevPlan&, const VjpPtrs<double>&,
                                                   const cx<double>*, const cx<double>*, int, int, double2*,
                                                   hipStream_t);

}  // namespace fd
