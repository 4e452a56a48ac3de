// Internal declarations shared by the planner, the kernels and the C ABI.
//
// Storage model (Sec. 3.1.4 / App. B.2): every amplitude the schedule writes
// is diag(n) + offset for one of a few offset types.  With the detected modes
// numbered j = 0..MD-1 (ket position 2j, bra 2j+1 of the detected index):
//   F0          offset 0                          (the outputs)
//   F1k(j)      offset 1_ket(j)                   n_0 <= C_0-2 [, n_j <= C_j-2]
//   F1b(j)      offset 1_bra(j)                   n_0 <= C_0-3 (j=0), else as F1k
//   F2(K)       offset 2*1_ket(K)                 n_<K = 0, n_K <= C_K-3
//   F1010(K,j)  offset 1_ket(K) + 1_ket(j), j>K   n_<K = 0, n_K <= C_K-2, n_j <= C_j-2
//   F1001(K,j)  offset 1_ket(K) + 1_bra(j), j>K   same as F1010
// Each family is indexed by its diagonal coordinate n.  Families of "group"
// K (F2(K), F1010(K,.), F1001(K,.)) only hold n with n_<K = 0; F0 and the
// type-1 families are group 0.
//
// Nodes are stored level-major: level S = |n| holds the lattice points of
// the detected box with sum S in lexicographic order (first mode slowest).
// With that order the points of sub-box K (n_<K = 0) are exactly the first
// Ncnt[K][S] points of level S, so one rank serves every family, and the
// ranks of n - 1_j (level S-1) and n + 1_K (level S+1) are increasing in the
// rank of n: neighbouring threads touch neighbouring addresses.
//
// Every node carries a block of B = prod_U C_u^2 entries (the undetected
// modes' ket/bra indices, C order [k_u..., l_u...]; Algorithm 2); B = 1 when
// every mode is detected (Algorithm 1).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "fockdiag.h"

namespace fd {

constexpr int kMaxModes = 16;
constexpr int kMaxD = 8;                 // detected modes with cutoff >= 2
constexpr int kMaxUq = 6;                // undetected block coordinates (2 per U mode, at most 3 modes)
constexpr int kMaxBlock = 65536;         // entries per node (prod_U C_u^2)
constexpr int kMaxCut = 64;
constexpr int kMaxPos = kMaxUq + 2 * kMaxD;   // positions of the active index
constexpr int kMaxFam = 1 + 3 * kMaxD + kMaxD * (kMaxD - 1);
constexpr int kMaxSmax = kMaxD * (kMaxCut - 1);
constexpr int kPnMax = (kMaxD + 1) * (kMaxSmax + 3);
constexpr int kPartialSlots = 4096;      // deterministic VJP partial accumulators
constexpr int kStreamSlots = 1024;       // workgroups of a block kernel whose rows stream from HBM
constexpr int kThreads = 256;
constexpr int kBT = 64;                  // threads of the block (Algorithm 2) kernels: one wavefront
constexpr int kVjpWaves = 4;             // wavefronts per workgroup of the block reverse kernel,
constexpr int kVjpWavesLds = 2;          // or this many where four wavefronts' staging does not fit the LDS
constexpr int kFwdWaves = 4;             // wavefronts per workgroup of the block forward kernel
constexpr int kFwdChunk = 448;           // own entries of one of its (lattice point, row chunk) units,
constexpr int kFwdChunkSmall = 192;      // on levels with fewer than kSmallLevelUnits units
constexpr int kNodeStride = 3 * kMaxD;   // ints per node record: m, rank(m - 1_j), rank(m + 1_j)
constexpr int kPointBatch = 32;          // Abar records per LDS staging batch, point reverse kernel
constexpr int kBlockBatch = 32;          // the same, block reverse kernel
constexpr int kVjpSlots = 16384;         // reduction slots of the state-vector cotangents

enum FamType { F_F0 = 0, F_F1K, F_F1B, F_F2, F_1010, F_1001 };

__host__ __device__ constexpr inline int fam_f1k(int j) { return 1 + j; }
__host__ __device__ constexpr inline int fam_f1b(int MD, int j) { return 1 + MD + j; }
__host__ __device__ constexpr inline int fam_f2(int MD, int K) { return 1 + 2 * MD + K; }
__host__ __device__ constexpr inline int pair_index(int MD, int K, int j) {
  return K * MD - K * (K + 1) / 2 + (j - K - 1);
}
__host__ __device__ constexpr inline int fam_1010(int MD, int K, int j) { return 1 + 3 * MD + 2 * pair_index(MD, K, j); }
__host__ __device__ constexpr inline int fam_1001(int MD, int K, int j) {
  return 1 + 3 * MD + 2 * pair_index(MD, K, j) + 1;
}

// Plain-old-data view of a plan passed by value to kernels.
struct DevPlan {
  int MD, MU, nq, npos;      // detected modes, undetected modes, U coords, positions
  int B;                     // entries per node
  int smax, pnw;             // max level, row width of the PN table (smax + 3)
  int odd;                   // 1 if type-1 (odd) families are computed
  int CD[kMaxD];             // detected cutoffs (all >= 2)
  int udims[kMaxUq];         // U block dims [C_u.., C_u..]
  int ustride[kMaxUq];
  double uinv[kMaxUq];       // 1 / ustride (exact coordinate split, see ucoord)
  double cinv[kMaxD];        // 1 / CD (exact digit split of C-order indices, see node_of_cindex)
  const int* pn;             // [(MD+1) x pnw]: PN[d][s+1] = #points of sub-box d with sum <= s
  const int64_t* lvl;        // [(MD) x (smax+2)]: node offset of level S for group g (store-all)
  const int* node;           // Algorithm 2 plans: node records in level-major order (else null)
  int64_t ringN[kMaxD];      // ring slot stride in nodes per group (ring mode)
  // debug write counters (fd_plan_set_write_counters): one count per element
  // of the store-all buffer written by the forward kernels; null when off
  unsigned int* wcnt;
  const char* wbase;         // start of the store-all buffer
  int64_t wcnt_n;            // counters
};

// Split of a node's undetected block into chunks of whole rows of the first
// undetected coordinate (rows of R0 = B / C0 entries).
struct ChunkGeo {
  int C0, R0, RC, nchunks;   // rows, entries per row, rows per chunk, chunks per node
};

// Device pointers of one set of family arrays (forward values or cotangents).
template <typename R>
struct FamPtrs {
  R* f[kMaxFam];             // interleaved complex, element pointer of node 0
  int ring;                  // 1: two-slot ring (slot S&1), 0: store-all by level
};

// Optional per-launch HIP-event timing, by kernel kind.
enum KernelKind {
  KK_PREP = 0, KK_UFILL, KK_FWD_LEVEL, KK_OUT_PERM, KK_PERM_IN, KK_VJP_LEVEL, KK_UFILL_VJP, KK_VJP_FINAL,
  KK_ZERO, KK_BATCH_PREP, KK_BATCH_SWEEP, KK_BATCH_OUT, KK_COUNT
};
struct Timing {
  uint32_t mask = 0;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[KK_COUNT];
};

// Cached instantiated graph of one whole sweep, keyed by every pointer it uses.
struct GraphEntry {
  int kind = 0;                      // 0 forward, 1 reverse
  bool odd = false;
  const void* ptr[12] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

struct Plan {
  uint64_t uid = 0;                  // unique per plan (keys of cached batch schedules)
  // caller's view
  int M = 0;
  std::vector<int> cut;
  uint32_t mask = 0;
  fd_dtype dt = FD_C128;
  uint32_t flags = 0;
  // active problem
  int MU = 0, MD = 0, nq = 0, npos = 0, B = 1, smax = 0, nfam = 0;
  std::vector<int> umodes, dmodes, CU, CD, udims, ustride;
  std::vector<int> pos2blk;          // internal position -> block index in [0, 2M)
  std::vector<int> pn;               // (MD+1) x pnw
  std::vector<int64_t> ncnt;         // (MD+1) x (smax+1)
  std::vector<int64_t> lvl;          // MD x (smax+2)
  std::vector<int64_t> group_nodes;  // per group: prod_{i>=g} CD_i
  std::vector<int64_t> maxN;         // per group: max level size
  std::vector<int> fam_group;        // per family
  int64_t nodes_total = 1;           // prod CD (capped plans: lattice points with |n| <= smax)
  int level_cap = -1;                // total photon cutoff of the detected lattice (-1: the box)
  int64_t out_elems = 1;
  // structure counts (App. B)
  int64_t pivots = 0, stored[6] = {0, 0, 0, 0, 0, 0}, targets = 0, terms = 0;
  // device state
  int device = -1;
  int* d_pn = nullptr;
  int64_t* d_lvl = nullptr;
  int* d_node = nullptr;             // node records (Algorithm 2 plans)
  double* d_mass = nullptr;          // per-level probability masses (stopping rule)
  int* d_status = nullptr;
  // undetected-block fill order (step 1 of Algorithm 2): entries sorted by weight
  std::vector<int> elist, woff;
  int wmax = 0;
  int* d_elist = nullptr;
  int* d_woff = nullptr;
  mutable Timing timing;
  // hipGraph replay of whole sweeps (opt-in)
  bool use_graphs = false;
  std::vector<GraphEntry> graphs;
  hipStream_t capture_stream = nullptr;
  uint64_t graph_clock = 0;
  // reverse-sweep checkpoint interval in levels (0: the saved buffer keeps
  // every level of every family)
  int ckpt = 0;
  unsigned int* wcnt = nullptr;      // debug write counters (caller-owned device array), null: off
  size_t wcnt_n = 0;
  // blocks whose rows do not fit the LDS staging stream them from HBM, per
  // kernel: forward block units, block fill, reverse block units, reverse fill
  bool st_fwd = false, st_ufill = false, st_vjp = false, st_ufill_vjp = false;
  // wavefronts per workgroup of the block reverse kernel (kVjpWaves, or
  // kVjpWavesLds where the rows and staging of kVjpWaves do not fit the LDS)
  int vjp_waves = kVjpWavesLds;
  bool odd_for(bool b_zero) const { return !b_zero || MU > 0; }
};

size_t elem_bytes(fd_dtype dt);
// True once the library is being unloaded: releases then skip device calls.
bool unloading();
// LDS of the undetected-block fill (vjp: its reverse), one wavefront: the
// block (twice for the reverse: forward values and cotangents), A and b
// between undetected positions, the square-root tables, the entry list by
// weight and its offsets.
inline size_t ufill_lds_bytes(const Plan& P, bool vjp) {
  const size_t eb = elem_bytes(P.dt);
  return (vjp ? 2 : 1) * (size_t)P.B * eb + (size_t)(kMaxUq * kMaxUq + kMaxUq) * eb + 2 * (kMaxCut + 4) * (eb / 2) +
         (size_t)(P.B + P.wmax + 2) * sizeof(int);
}
// ... as launched: a streamed fill keeps only A, b and the square-root
// tables in LDS.
inline size_t ufill_launch_lds_bytes(const Plan& P, bool vjp) {
  const size_t eb = elem_bytes(P.dt);
  if (vjp ? P.st_ufill_vjp : P.st_ufill) return (size_t)(kMaxUq * kMaxUq + kMaxUq) * eb + 2 * (kMaxCut + 4) * (eb / 2);
  return ufill_lds_bytes(P, vjp);
}

// LDS of the block fill with tangents (forward mode): values and tangents of
// the block, of A and b between undetected positions, then the tables.
inline size_t ufill_jvp_lds_bytes(const Plan& P) {
  return ufill_lds_bytes(P, false) + (size_t)P.B * elem_bytes(P.dt) +
         (size_t)(kMaxUq * kMaxUq + kMaxUq) * elem_bytes(P.dt);
}

// level_cap >= 0: every mode with cutoff >= 2 detected, only lattice points
// with |n| <= level_cap (the levels of a total photon cutoff), F0 returned in
// level order.
fd_status build_plan(int M, const int* cutoffs, uint32_t mask, fd_dtype dt, uint32_t flags, Plan* P,
                     std::string* err, int level_cap = -1);
fd_status ensure_device(Plan* P, std::string* err);
DevPlan make_devplan(const Plan& P, bool odd);

// Workspace layouts (byte offsets from the start of the buffer).
struct FwdLayout {
  size_t prep = 0;                   // A_int, b_int, c, status scratch
  size_t f0 = 0;                     // F0 store-all (output-sized)
  std::vector<size_t> fam;           // per family (index 0 unused)
  size_t total = 0;
};
FwdLayout fwd_layout(const Plan& P, bool odd, bool store_all, size_t base);
struct VjpLayout {
  size_t prep = 0;
  size_t g0 = 0;                     // drho in level-major node order
  std::vector<size_t> gfam;          // cotangent rings per family (F0 too)
  size_t partial = 0;                // kPartialSlots x (npos x (npos+1)) complex (double)
  size_t priv = 0;                   // block plans: kPartialSlots (streamed: kStreamSlots) x vjp_private_entries
  size_t ublk = 0;                   // streamed reverse fill: the block's cotangents (B entries)
  size_t total = 0;
};
// Entries of one workgroup's private slot of the block reverse kernel: the
// pivot cotangent blocks (MD rows sets), their b-terms and the own F0
// cotangent rows, each read only by the lane that wrote it; streamed rows add
// the undetected-neighbour terms (NQ x (RC + 2) rows).
size_t vjp_private_entries(const Plan& P);
size_t vjp_lds_bytes(const Plan& P);   // dynamic LDS of the block reverse kernel (largest geometry used)
// Dynamic LDS of the forward block kernel for one chunk geometry: F0 rows
// [k0-2, k1), MD bridge pivot blocks of rows [k0-1, k1), A and b, the
// square-root tables.
size_t fwd_lds_bytes_for(const Plan& P, const ChunkGeo& G, bool jvp = false);   // jvp: values and tangents
// ... with the rows streamed from HBM (A, b and the tables only)
size_t fwd_stream_lds_bytes(const Plan& P);
// Entries of one workgroup's slot for the streamed forward block kernel: the
// bridge pivot blocks, MD x (RC + 1) rows.
size_t fwd_stream_entries(const Plan& P);
size_t prep_core_bytes(const Plan& P);   // A_int, b_int, c (the stream slots follow in prep_bytes)
size_t vjp_lds_bytes_for(const Plan& P, const ChunkGeo& G);   // ... for one chunk geometry
constexpr size_t kMaxLds = 160 * 1024;
VjpLayout vjp_layout(const Plan& P, bool odd, size_t base);
size_t prep_bytes(const Plan& P);
// Checkpointed reverse sweeps (Plan::ckpt = s > 0): the saved buffer keeps F0
// at every level and, for each segment of s levels after the first, the
// families of the level just below the segment (what the forward needs to
// restart there).  Segment c covers levels [c s, min((c + 1) s, smax + 1)).
// Levels are stored at their exact sizes; the odd-level families are left
// out when the plan promises b = 0 and every mode is detected.
struct CkptLayout {
  size_t f0 = 0;                     // F0, every level (output-sized); never 0, which means "absent"
  std::vector<size_t> ck;            // [(c - 1) * nfam + f]: family f in checkpoint c >= 1
  int nseg = 0;                      // segments; checkpoints = nseg - 1
  size_t total = 0;
};
CkptLayout ckpt_layout(const Plan& P);
// The segment buffer of a checkpointed sweep, in the workspace after the
// reverse sweep's own layout: per family, the levels seg_lo - 1 .. seg_hi of
// the largest segment, packed at their exact sizes (seg_node gives where
// level L starts); the forward's two-level ring uses slots of maxN nodes.
struct SegLayout {
  size_t base = 0;
  std::vector<size_t> fam;           // per family: start of its region (0: none)
  size_t total = 0;
};
SegLayout seg_layout(const Plan& P);
bool ckpt_keeps_family(const Plan& P, int f);
// Node offset of level L inside a segment buffer region holding levels
// seg_lo - 1 .. (group g).
int64_t seg_node(const Plan& P, int g, int seg_lo, int L);
// Bytes of the saved buffer for fock_diag_vjp (every level, or checkpoints).
size_t saved_bytes(const Plan& P);
// Workspace bytes of fock_diag_vjp with a saved buffer (and of fock_diag_fwd
// with one); includes the segment buffer of a checkpointed plan.
size_t vjp_ws_bytes(const Plan& P);
void count_work(const Plan& P, bool b_zero, int64_t* targets, int64_t* terms);
// Batched forward (one persistent sweep launch over every circuit); plans
// already on the current device, workspaces checked by the caller.
fd_status run_forward_batch(int n, Plan* const* plans, const bool* odd, const void* const* A,
                            const void* const* b, const void* const* c, void* const* rho, void* const* ws,
                            hipStream_t st, std::string* err);
void batch_forget(uint64_t plan_uid);   // drops cached batch schedules that use this plan
fd_status batch_set_tuning(const fd_batch_tuning& T);
fd_batch_tuning batch_get_tuning();

// Brackets one launch with events when its kind is enabled on the plan.
struct KTimer {
  Timing* T = nullptr;
  int kind = 0;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(const Plan& P, int k, hipStream_t st) : T(&P.timing), kind(k), s(st) {
    if (!(T->mask & (1u << k))) return;
    a = take();
    b = take();
    if (a && b) (void)hipEventRecord(a, s);
  }
  ~KTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      T->rec[kind].push_back({a, b});
    }
  }
  hipEvent_t take() {
    hipEvent_t e = nullptr;
    if (!T->pool.empty()) {
      e = T->pool.back();
      T->pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
    }
    return e;
  }
};

// kernels (kernels_fwd.hip / kernels_vjp.hip)
// Probability-sum stopping of a sweep over an all-detected plan: after every
// kStopBlock levels the masses sum_{|n| = S} p(n) of the new levels are read
// back (the stream is synchronised) and the sweep ends at the first level S*
// with sum_{S <= S*} mass >= 1 - eps; F0 above S* is cleared.
constexpr int kStopBlock = 4;
constexpr int kMassParts = 32;   // workgroups per level of the mass sum (partials added on the host in order)
struct StopRule {
  double eps = 0.0;
  int levels_done = 0;   // out: S* + 1 (smax + 1 if the sum never reaches 1 - eps)
  double mass = 0.0;     // out: sum of the returned levels' masses
};
// Forward mode (all modes detected): rho and its tangent along (dA, db, dc).
// The workspace holds two halves of jvp_half_bytes each: values, then tangents.
size_t jvp_half_bytes(const Plan& P);
hipError_t run_jvp(const Plan& P, const void* A, const void* b, const void* c, const void* dA, const void* db,
                   const void* dc, void* rho, void* drho, void* ws, hipStream_t st);
hipError_t run_forward(const Plan& P, bool odd, const void* A, const void* b, const void* c, void* rho, void* ws,
                       void* saved, hipStream_t st, StopRule* stop = nullptr);
// One forward level launch with explicit family pointers (rd: level S-1,
// wr: level S, indexed by family; F0 of levels S and S+1); Ai/bi the
// interleaved, symmetrised triple from launch_prep.
hipError_t launch_fwd_level(const Plan& P, bool odd, int S, const void* const* rd, void* const* wr,
                            const void* f0cur, void* f0nxt, const void* Ai, const void* bi, hipStream_t st);
// Copies n[f] complex entries from src[f] to dst[f] for every family f with
// a non-null src (one launch).
hipError_t launch_copy_fams(const Plan& P, const void* const* src, void* const* dst, const int64_t* n, hipStream_t st);
ChunkGeo chunk_geo(const Plan& P, int target = kBT);   // forward block kernels
ChunkGeo fwd_geo(const Plan& P, int64_t nwork);     // forward chunks on a level of nwork lattice points
struct VjpChunking {
  int target, small, small_units;
};
VjpChunking vjp_chunking(const Plan& P);
ChunkGeo vjp_geo(const Plan& P, int64_t nwork);     // reverse chunks on a level of nwork lattice points
constexpr int kSmallLevelUnits = 4096;   // below: the forward level halves its row chunks
// LDS tile of the permutations between rho's C order and node order:
// consecutive lattice points x consecutive undetected-block entries
constexpr int kOutTN = 64, kOutTK = 16;
hipError_t launch_prep(const Plan& P, const void* A, const void* b, const void* c, void* Ai, void* f0node0,
                       hipStream_t st);
// F0 in node order (level-major, prod_D C_j x B entries) -> rho in C order.
hipError_t launch_out_perm(const Plan& P, const void* f0, void* rho, hipStream_t st);
// State vectors (kernels_state.hip): workspace bytes and the forward sweep.
size_t state_ws_bytes(const Plan& P);
hipError_t run_state_fwd(const Plan& P, bool b_zero, const void* A, const void* b, const void* c, void* psi, void* ws,
                         hipStream_t st);
size_t state_vjp_ws_bytes(const Plan& P);
hipError_t run_state_jvp(const Plan& P, const void* c, const void* psi, const void* dA, const void* db, const void* dc,
                         void* dpsi, hipStream_t st);
hipError_t run_state_vjp(const Plan& P, const void* c, const void* psi, const void* g, void* dA, void* db, void* dc,
                         void* ws, hipStream_t st);
hipError_t run_vjp(const Plan& P, bool odd, const void* A, const void* b, const void* c, const void* saved,
                   const void* drho, void* dA, void* db, void* dc, void* ws, hipStream_t st);

// Error reporting of the C ABI: sets the calling thread's fd_last_error().
fd_status api_fail(fd_status s, const std::string& msg);
fd_status api_ok();

}  // namespace fd

// The opaque plan handle of the C ABI.
struct fd_plan_s {
  fd::Plan P;
};
