// Shared by the reverse point kernels (kernels_vjp.hip) and the reverse
// block kernels (kernels_vjp_block.hip): the per-level pointer table of the
// reverse sweep and the matrix-core reduction of the Abar / bbar records.
#pragma once

#include "fd_device.h"

namespace fd {

template <typename R>
struct VjpPtrs {
  const cx<R>* fprev[kMaxFam];  // forward values, level S-1 (store-all)
  const cx<R>* fcur[kMaxFam];   // forward values, level S (fcur[0] = F0)
  cx<R>* gprev[kMaxFam];        // cotangent ring slot of level S-1
  cx<R>* gcur[kMaxFam];         // cotangent ring slot of level S (gcur[0] = F0)
  const cx<R>* gf0nxt;          // F0 cotangents, level S+1
  const cx<R>* d0cur;           // drho in node order, level S
  const int* node;              // node records of level S (Algorithm 2 plans)
  cx<R>* priv;                  // per-workgroup private slots (Algorithm 2 plans)
  int64_t priv_stride;          // entries per slot
};

// Abar / bbar: every reverse step reduces outer products of per-target
// records (the target cotangents h and the read values x of one pivot
// application) over all targets: D[i][l] = sum_rec h_i conj(x_l), i.e.
// (H^T X-bar)[i][l], a dense contraction over the records.  A wavefront
// stages NB records in LDS (row r of H or X holds value r of every record,
// rows NB + 1 apart so the rows read together fall in different banks) and
// runs NB / 4 FP64 MFMA 16x16x4 steps of four records: lane t feeds value
// t % 16 of record k0 + t / 16 to both operands (one 16-byte LDS read each)
// and keeps D[4 j + t / 16][16 c + t % 16], j = 0..3, of column tile c in its
// accumulators (the gfx950 output layout, checked on the device).  The
// complex products take three real products (Karatsuba's method):
// P1 = Hr Xr, P2 = Hi Xi, P3 = (Hr + Hi)(Xr - Xi), each summed in its own
// accumulator; the real part is P1 + P2 and the imaginary part (Hi Xr -
// Hr Xi) is P3 - P1 + P2.  Three MFMAs per step instead of four, and three
// independent accumulation chains of one MFMA per step instead of two of
// two.  The hardware fixes the order of accumulation, so the sums are
// reproducible.  At most 16 rows of H (NPD) and 32 columns of X (NCOL).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int NT>
struct MfmaAcc {
  mfma_d4 p1[NT], p2[NT], p3[NT];
};

template <int NT>
__device__ __forceinline__ void mfma_acc_zero(MfmaAcc<NT>& a) {
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    a.p1[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    a.p2[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    a.p3[t] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  }
}

template <typename R, int NPD, int NCOL, int NB>
__device__ __forceinline__ void wave_accum_mfma(const cx<R>* recw, MfmaAcc<(NCOL + 15) / 16>& acc) {
  static_assert(NPD <= 16 && NCOL <= 32, "one row tile of H, at most two column tiles of X");
  constexpr int NT = (NCOL + 15) / 16;
  constexpr int RS = NB + 1;   // records per staging batch, padded row stride
  const int lane = threadIdx.x & 63;
  const int row = lane & 15, kq = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const int rc = k0 + kq;
    const cx<R> h = row < NPD ? recw[row * RS + rc] : czero<R>();
    const double hx = (double)h.x, hy = (double)h.y, hs = hx + hy;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = 16 * t + row;
      const cx<R> x = col < NCOL ? recw[(NPD + col) * RS + rc] : czero<R>();
      const double xx = (double)x.x, xy = (double)x.y;
      acc.p1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hx, xx, acc.p1[t], 0, 0, 0);
      acc.p2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hy, xy, acc.p2[t], 0, 0, 0);
      acc.p3[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(hs, xx - xy, acc.p3[t], 0, 0, 0);
    }
  }
}

// Writes this lane's accumulated pairs into red[i * NR + l] (a wave's NPD x NR
// pair table); pairs beyond NCOL columns are the caller's (they stay unset).
template <int NPD, int NR, int NCOL>
__device__ __forceinline__ void mfma_acc_store(const MfmaAcc<(NCOL + 15) / 16>& acc, cx<double>* red) {
  constexpr int NT = (NCOL + 15) / 16;
  const int lane = threadIdx.x & 63;
  const int col0 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int l = 16 * t + col0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 4 * j + kq;
      if (i < NPD && l < NCOL) {
        const double p1 = acc.p1[t][j], p2 = acc.p2[t][j];
        red[i * NR + l] = cmake<double>(p1 + p2, (acc.p3[t][j] - p1) + p2);
      }
    }
  }
}


// One level of the reverse sweep of an Algorithm 2 plan (the block kernel
// for the plan's detected-mode count and block coordinates).
template <typename R>
hipError_t launch_vjp_block_level(const Plan& Pl, const DevPlan& P, const VjpPtrs<R>& Vp, const cx<R>* Ai,
                                  const cx<R>* bi, int S, int nwork, double2* partial, hipStream_t st);

}  // namespace fd
