// extern "C" entry points declared in include/fockdiag.h: argument checks on
// the host, workspace carving, schedule choice, then the kernel launchers.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "fd_internal.h"

// A state-vector plan: the tables of the all-detected plan over the same
// modes (the lattice of n, its levels and the output permutation).
struct fd_state_plan_s {
  fd_plan inner = nullptr;
};

namespace {
thread_local std::string g_err;

fd_status fail(fd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
fd_status ok() {
  g_err.clear();
  return FD_OK;
}

// Decide the b = 0 schedule (Sec. 2.4) for this call; b has nb entries
// (2M for a density matrix, M for a state vector).
fd_status decide_b_zero(const fd::Plan& P, const void* b, hipStream_t s, bool* b_zero, int nb = -1) {
  if (nb < 0) nb = 2 * P.M;
  if (P.flags == FD_B_ZERO) {
    *b_zero = true;
    return FD_OK;
  }
  if (P.flags == FD_B_GENERAL) {
    *b_zero = false;
    return FD_OK;
  }
  const size_t eb = fd::elem_bytes(P.dt);
  std::vector<unsigned char> h((size_t)nb * eb);
  if (hipMemcpyAsync(h.data(), b, h.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(FD_ERR_HIP, "reading b for the b = 0 test failed");
  bool z = true;
  if (P.dt == FD_C64) {
    const float* v = reinterpret_cast<const float*>(h.data());
    for (size_t i = 0; i < (size_t)2 * nb; ++i) z = z && v[i] == 0.0f;
  } else {
    const double* v = reinterpret_cast<const double*>(h.data());
    for (size_t i = 0; i < (size_t)2 * nb; ++i) z = z && v[i] == 0.0;
  }
  *b_zero = z;
  return FD_OK;
}

constexpr size_t kGraphCache = 8;

// Runs `body(stream)` directly, or -- when the plan replays graphs and no
// per-kernel timing is on -- captures it once per pointer set into a graph
// (on a private capture stream) and launches the instantiated graph on `s`.
template <typename F>
hipError_t run_maybe_graph(fd::Plan& P, int kind, bool odd, std::initializer_list<const void*> ptrs, hipStream_t s,
                           F body) {
  if (!P.use_graphs || P.timing.mask != 0) return body(s);
  const void* key[12] = {};
  int n = 0;
  for (const void* q : ptrs) key[n++] = q;
  for (fd::GraphEntry& g : P.graphs) {
    if (g.kind == kind && g.odd == odd && std::equal(key, key + 12, g.ptr)) {
      g.last_use = ++P.graph_clock;
      return hipGraphLaunch(g.exec, s);
    }
  }
  hipError_t e;
  if (!P.capture_stream && (e = hipStreamCreateWithFlags(&P.capture_stream, hipStreamNonBlocking)) != hipSuccess)
    return e;
  if ((e = hipStreamBeginCapture(P.capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
  hipError_t eb = body(P.capture_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(P.capture_stream, &graph);
  if (eb != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return eb;
  }
  if (e != hipSuccess) return e;
  hipGraphExec_t exec = nullptr;
  if ((e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return e;
  }
  if (P.graphs.size() >= kGraphCache) {
    auto it = std::min_element(P.graphs.begin(), P.graphs.end(),
                               [](const fd::GraphEntry& a, const fd::GraphEntry& b) { return a.last_use < b.last_use; });
    (void)hipGraphExecDestroy(it->exec);
    (void)hipGraphDestroy(it->graph);
    P.graphs.erase(it);
  }
  fd::GraphEntry g;
  g.kind = kind;
  g.odd = odd;
  std::copy(key, key + 12, g.ptr);
  g.graph = graph;
  g.exec = exec;
  g.last_use = ++P.graph_clock;
  P.graphs.push_back(g);
  return hipGraphLaunch(exec, s);
}

void drop_graphs(fd::Plan& P) {
  for (fd::GraphEntry& g : P.graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  P.graphs.clear();
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

fd_status check_ptrs(const fd::Plan& P, std::initializer_list<const void*> ps) {
  const size_t a = P.dt == FD_C64 ? 8 : 16;
  for (const void* p : ps) {
    if (!p) return fail(FD_ERR_INVALID_ARG, "a required device pointer is NULL");
    if (!aligned(p, a)) return fail(FD_ERR_INVALID_ARG, "complex buffers must be aligned to their element size");
  }
  return FD_OK;
}
}  // namespace

namespace fd {
fd_status api_fail(fd_status s, const std::string& msg) { return fail(s, msg); }
fd_status api_ok() { return ok(); }
}  // namespace fd

extern "C" {

fd_status fd_plan_create(int M, const int* cutoffs, uint32_t detected_mask, fd_dtype dt, uint32_t flags,
                         fd_plan* out) {
  if (!out) return fail(FD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  fd_plan p = new (std::nothrow) fd_plan_s;
  if (!p) return fail(FD_ERR_OOM, "host allocation failed");
  std::string err;
  fd_status s = fd::build_plan(M, cutoffs, detected_mask, dt, flags, &p->P, &err);
  if (s != FD_OK) {
    delete p;
    return fail(s, err);
  }
  *out = p;
  return ok();
}

fd_status fd_plan_destroy(fd_plan p) {
  if (!p) return ok();
  fd::Plan& P = p->P;
  if (fd::unloading()) {   // the HIP runtime may be gone: release host memory only
    delete p;
    return ok();
  }
  if (P.d_pn) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(P.device);
    (void)hipFree(P.d_pn);
    (void)hipFree(P.d_lvl);
    (void)hipFree(P.d_status);
    (void)hipFree(P.d_elist);
    (void)hipFree(P.d_woff);
    (void)hipFree(P.d_node);
    (void)hipFree(P.d_mass);
    (void)hipSetDevice(cur);
  }
  drop_graphs(P);
  fd::batch_forget(P.uid);
  if (P.capture_stream) (void)hipStreamDestroy(P.capture_stream);
  for (auto& v : P.timing.rec)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : P.timing.pool) (void)hipEventDestroy(e);
  delete p;
  return ok();
}

fd_status fd_plan_workspace(fd_plan p, int with_vjp, size_t* fwd_bytes, size_t* saved_bytes) {
  if (!p || !fwd_bytes || !saved_bytes) return fail(FD_ERR_INVALID_ARG, "NULL argument");
  const fd::Plan& P = p->P;
  if (!with_vjp) {
    *fwd_bytes = fd::fwd_layout(P, true, false, 0).total;
    *saved_bytes = 0;
  } else {
    *saved_bytes = fd::saved_bytes(P);
    *fwd_bytes = std::max(fd::vjp_ws_bytes(P), fd::prep_bytes(P));
  }
  return ok();
}

fd_status fd_plan_set_checkpoint(fd_plan p, int every) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  if (every < 0) return fail(FD_ERR_INVALID_ARG, "the checkpoint interval must be >= 0");
  fd::Plan& P = p->P;
  if (P.ckpt != every) drop_graphs(P);
  P.ckpt = every;
  return ok();
}

fd_status fd_plan_set_write_counters(fd_plan p, unsigned int* counters, size_t n) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  if (!counters) {
    if (n != 0) return fail(FD_ERR_INVALID_ARG, "n must be 0 when the counters are NULL");
  } else {
    const size_t need = fd::saved_bytes(P) / fd::elem_bytes(P.dt);
    if (P.ckpt > 0) return fail(FD_ERR_UNSUPPORTED, "write counters need the store-all saved buffer (no checkpoints)");
    if (n < need) return fail(FD_ERR_INVALID_ARG, "fewer counters than elements of the saved buffer");
  }
  if (P.wcnt != counters || P.wcnt_n != n) drop_graphs(P);
  P.wcnt = counters;
  P.wcnt_n = n;
  return ok();
}

fd_status fd_plan_query(fd_plan p, int what, int64_t* out) {
  if (!p || !out) return fail(FD_ERR_INVALID_ARG, "NULL argument");
  fd::Plan& P = p->P;
  switch (what) {
    case FD_Q_OUT_ELEMS: *out = P.out_elems; break;
    case FD_Q_LEVELS: *out = P.smax + 1; break;
    case FD_Q_PIVOTS: *out = P.pivots; break;
    case FD_Q_STORED_NODES: {
      int64_t t = 0;
      for (int i = 0; i < 6; ++i) t += P.stored[i];
      *out = t;
      break;
    }
    case FD_Q_TARGETS:
    case FD_Q_READ_TERMS: {
      if (P.targets < 0) fd::count_work(P, P.flags == FD_B_ZERO, &P.targets, &P.terms);
      *out = what == FD_Q_TARGETS ? P.targets : P.terms;
      break;
    }
    case FD_Q_BLOCK: *out = P.B; break;
    case FD_Q_NODES_F0: *out = P.stored[fd::F_F0]; break;
    case FD_Q_NODES_F1: *out = P.stored[fd::F_F1K] + P.stored[fd::F_F1B]; break;
    case FD_Q_NODES_F2: *out = P.stored[fd::F_F2]; break;
    case FD_Q_NODES_F1010: *out = P.stored[fd::F_1010]; break;
    case FD_Q_NODES_F1001: *out = P.stored[fd::F_1001]; break;
    case FD_Q_B_SCHEDULE: *out = P.flags == FD_B_ZERO ? 1 : 0; break;
    default: return fail(FD_ERR_INVALID_ARG, "unknown query");
  }
  return ok();
}

fd_status fock_diag_fwd(fd_plan p, const void* A, const void* b, const void* c, void* rho, void* workspace,
                        size_t ws_bytes, void* saved, size_t saved_bytes, hipStream_t stream) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  fd_status s = check_ptrs(P, {A, b, c, rho, workspace});
  if (s != FD_OK) return s;
  if (saved && !aligned(saved, 256)) return fail(FD_ERR_INVALID_ARG, "saved must be 256-byte aligned");
  if (!aligned(workspace, 256)) return fail(FD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  bool b_zero = false;
  if ((s = decide_b_zero(P, b, stream, &b_zero)) != FD_OK) return s;
  const bool odd = P.odd_for(b_zero);
  if (saved) {
    if (saved_bytes < fd::saved_bytes(P)) return fail(FD_ERR_WORKSPACE, "saved buffer too small");
    // a checkpointed forward runs its ring in the reverse sweep's segment buffer
    if (ws_bytes < (P.ckpt > 0 ? fd::vjp_ws_bytes(P) : fd::prep_bytes(P)))
      return fail(FD_ERR_WORKSPACE, "workspace too small");
  } else if (ws_bytes < fd::fwd_layout(P, odd, false, 0).total) {
    return fail(FD_ERR_WORKSPACE, "workspace too small");
  }
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  hipError_t e = run_maybe_graph(P, 0, odd, {A, b, c, rho, workspace, saved}, stream, [&](hipStream_t st) {
    return fd::run_forward(P, odd, A, b, c, rho, workspace, saved, st);
  });
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return ok();
}

fd_status fd_plan_create_total(int M, const int* cutoffs, int total_cutoff, fd_dtype dt, uint32_t flags,
                               fd_plan* out) {
  if (!out) return fail(FD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (total_cutoff < 0) return fail(FD_ERR_INVALID_ARG, "total_cutoff must be >= 0");
  fd_plan p = new (std::nothrow) fd_plan_s;
  if (!p) return fail(FD_ERR_OOM, "host allocation failed");
  std::string err;
  const uint32_t all = M >= 32 ? 0xffffffffu : ((1u << M) - 1u);
  fd_status s = fd::build_plan(M, cutoffs, all, dt, flags, &p->P, &err, total_cutoff);
  if (s != FD_OK) {
    delete p;
    return fail(s, err);
  }
  *out = p;
  return ok();
}

fd_status fd_plan_level_offsets(fd_plan p, int64_t* offsets, int n) {
  if (!p || !offsets) return fail(FD_ERR_INVALID_ARG, "NULL argument");
  const fd::Plan& P = p->P;
  if (P.mask != (P.M >= 32 ? 0xffffffffu : ((1u << P.M) - 1u)))
    return fail(FD_ERR_INVALID_ARG, "level offsets are defined for plans with every mode detected");
  if (n < P.smax + 2) return fail(FD_ERR_INVALID_ARG, "offsets needs FD_Q_LEVELS + 1 entries");
  for (int S = 0; S <= P.smax + 1; ++S) offsets[S] = P.MD > 0 ? P.lvl[S] : (S == 0 ? 0 : 1);
  return ok();
}

fd_status detection_probs_until(fd_plan p, const void* A, const void* b, const void* c, void* probs, double eps,
                                int* levels_done, double* mass, void* workspace, size_t ws_bytes,
                                hipStream_t stream) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  if (P.mask != (P.M >= 32 ? 0xffffffffu : ((1u << P.M) - 1u)))
    return fail(FD_ERR_INVALID_ARG, "detection_probs_until needs a plan with every mode detected");
  if (P.MD == 0) return fail(FD_ERR_INVALID_ARG, "no mode with cutoff >= 2");
  if (!levels_done || !mass) return fail(FD_ERR_INVALID_ARG, "levels_done and mass must be host pointers");
  if (!(eps >= 0.0 && eps < 1.0)) return fail(FD_ERR_INVALID_ARG, "eps must be in [0, 1)");
  fd_status s = check_ptrs(P, {A, b, c, probs, workspace});
  if (s != FD_OK) return s;
  if (!aligned(workspace, 256)) return fail(FD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  bool b_zero = false;
  if ((s = decide_b_zero(P, b, stream, &b_zero)) != FD_OK) return s;
  const bool odd = P.odd_for(b_zero);
  if (ws_bytes < fd::fwd_layout(P, odd, false, 0).total) return fail(FD_ERR_WORKSPACE, "workspace too small");
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  fd::StopRule rule;
  rule.eps = eps;
  hipError_t e = fd::run_forward(P, odd, A, b, c, probs, workspace, nullptr, stream, &rule);
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  *levels_done = rule.levels_done;
  *mass = rule.mass;
  return ok();
}

fd_status detection_probs(fd_plan p, const void* A, const void* b, const void* c, void* probs, void* workspace,
                          size_t ws_bytes, hipStream_t stream) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  const fd::Plan& P = p->P;
  const uint32_t all = P.M >= 32 ? 0xffffffffu : ((1u << P.M) - 1u);
  if (P.mask != all) return fail(FD_ERR_INVALID_ARG, "detection_probs needs a plan with every mode detected");
  return fock_diag_fwd(p, A, b, c, probs, workspace, ws_bytes, nullptr, 0, stream);
}

fd_status fd_plan_jvp_workspace(fd_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(FD_ERR_INVALID_ARG, "NULL argument");
  *bytes = 2 * fd::jvp_half_bytes(p->P);
  return ok();
}

fd_status fock_diag_jvp(fd_plan p, const void* A, const void* b, const void* c, const void* dA, const void* db,
                        const void* dc, void* rho, void* drho, void* workspace, size_t ws_bytes,
                        hipStream_t stream) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  fd_status s = check_ptrs(P, {A, b, c, dA, db, dc, rho, drho, workspace});
  if (s != FD_OK) return s;
  if (!aligned(workspace, 256)) return fail(FD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (P.B > 1) {
    const size_t rows = std::max(fd::fwd_lds_bytes_for(P, fd::chunk_geo(P), true),
                                 fd::fwd_lds_bytes_for(P, fd::chunk_geo(P, fd::kBT / 2), true));
    if ((P.MD > 0 && rows > fd::kMaxLds) || fd::ufill_jvp_lds_bytes(P) > fd::kMaxLds)
      return fail(FD_ERR_UNSUPPORTED, "undetected block too large for the forward mode's LDS staging");
  }
  if (P.flags == FD_B_ZERO)
    return fail(FD_ERR_UNSUPPORTED, "forward mode needs the odd levels: create the plan with FD_B_AUTO or FD_B_GENERAL");
  if (ws_bytes < 2 * fd::jvp_half_bytes(P)) return fail(FD_ERR_WORKSPACE, "workspace too small");
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  const hipError_t e = run_maybe_graph(P, 2, true, {A, b, c, dA, db, dc, rho, drho, workspace}, stream,
                                      [&](hipStream_t st) {
                                        return fd::run_jvp(P, A, b, c, dA, db, dc, rho, drho, workspace, st);
                                      });
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return ok();
}

fd_status fock_diag_vjp(fd_plan p, const void* A, const void* b, const void* c, const void* saved,
                        size_t saved_bytes, const void* drho, void* dA, void* db, void* dc, void* workspace,
                        size_t ws_bytes, hipStream_t stream) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  if (P.level_cap >= 0 && P.B > 1) return fail(FD_ERR_UNSUPPORTED, "a total photon cutoff needs every mode detected");
  fd_status s = check_ptrs(P, {A, b, c, drho, dA, db, dc, workspace});
  if (s != FD_OK) return s;
  if (!aligned(workspace, 256) || (saved && !aligned(saved, 256)))
    return fail(FD_ERR_INVALID_ARG, "workspace and saved must be 256-byte aligned");
  if (P.B > 1 && (fd::vjp_lds_bytes(P) > fd::kMaxLds || fd::ufill_launch_lds_bytes(P, true) > fd::kMaxLds))
    return fail(FD_ERR_UNSUPPORTED, "undetected block too large for the reverse sweep's LDS staging");
  bool b_zero = false;
  if ((s = decide_b_zero(P, b, stream, &b_zero)) != FD_OK) return s;
  const bool odd = P.odd_for(b_zero);
  const size_t vneed = P.ckpt > 0 ? fd::vjp_ws_bytes(P) : fd::vjp_layout(P, odd, 0).total;
  const size_t sneed = fd::saved_bytes(P);
  const void* sv = saved;
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  void* region = nullptr;
  if (saved) {
    if (saved_bytes < sneed) return fail(FD_ERR_WORKSPACE, "saved buffer too small");
    if (ws_bytes < vneed) return fail(FD_ERR_WORKSPACE, "workspace too small");
  } else {
    // recompute the forward intermediates behind the reverse sweep's workspace
    const size_t off = (vneed + 255) & ~size_t(255);
    if (ws_bytes < off + sneed) return fail(FD_ERR_WORKSPACE, "workspace too small (saved == NULL)");
    region = static_cast<char*>(workspace) + off;
    sv = region;
  }
  hipError_t e = run_maybe_graph(P, 1, odd, {A, b, c, saved, drho, dA, db, dc, workspace}, stream,
                                 [&](hipStream_t st) {
                                   if (region) {
                                     hipError_t ef = fd::run_forward(P, odd, A, b, c, nullptr, workspace, region, st);
                                     if (ef != hipSuccess) return ef;
                                   }
                                   return fd::run_vjp(P, odd, A, b, c, sv, drho, dA, db, dc, workspace, st);
                                 });
  if (e != hipSuccess) return fail(FD_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return ok();
}

fd_status fock_diag_fwd_batch(int n, const fd_plan* plans, const void* const* A, const void* const* b,
                              const void* const* c, void* const* rho, void* const* workspace,
                              const size_t* ws_bytes, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!plans || !A || !b || !c || !rho || !workspace || !ws_bytes)))
    return fail(FD_ERR_INVALID_ARG, "bad batch arguments");
  if (n == 0) return ok();
  std::vector<fd::Plan*> P(n);
  std::unique_ptr<bool[]> odd(new bool[n]);
  std::vector<std::pair<uintptr_t, uintptr_t>> spans(n);
  std::string err;
  // host-side checks of every circuit first, then the device-side ones
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(FD_ERR_INVALID_ARG, "a plan of the batch is NULL");
    P[i] = &plans[i]->P;
    if (P[i]->dt != P[0]->dt) return fail(FD_ERR_INVALID_ARG, "every plan of a batch must have the same dtype");
    if (P[i]->level_cap >= 0)
      return fail(FD_ERR_UNSUPPORTED, "plans with a total photon cutoff are not batched; use fock_diag_fwd");
    fd_status s = check_ptrs(*P[i], {A[i], b[i], c[i], rho[i], workspace[i]});
    if (s != FD_OK) return s;
    if (!aligned(workspace[i], 256)) return fail(FD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  }
  for (int i = 0; i < n; ++i) {
    fd_status s;
    bool b_zero = false;
    if ((s = decide_b_zero(*P[i], b[i], stream, &b_zero)) != FD_OK) return s;
    odd[i] = P[i]->odd_for(b_zero);
    const size_t need = fd::fwd_layout(*P[i], odd[i], false, 0).total;
    if (ws_bytes[i] < need) return fail(FD_ERR_WORKSPACE, "workspace of circuit " + std::to_string(i) + " too small");
    spans[i] = {reinterpret_cast<uintptr_t>(workspace[i]), reinterpret_cast<uintptr_t>(workspace[i]) + need};
    if ((s = fd::ensure_device(P[i], &err)) != FD_OK) return fail(s, err);
    if (P[i]->device != P[0]->device) return fail(FD_ERR_INVALID_ARG, "every plan of a batch must be on one device");
  }
  std::sort(spans.begin(), spans.end());
  for (int i = 1; i < n; ++i)
    if (spans[i].first < spans[i - 1].second)
      return fail(FD_ERR_INVALID_ARG, "the workspaces of a batch must not overlap");
  fd_status s = fd::run_forward_batch(n, P.data(), odd.get(), A, b, c, rho, workspace, stream, &err);
  if (s != FD_OK) return fail(s, err);
  return ok();
}

fd_status fock_diag_vjp_batch(int n, const fd_plan* plans, const void* const* A, const void* const* b,
                              const void* const* c, const void* const* saved, const size_t* saved_bytes,
                              const void* const* drho, void* const* dA, void* const* db, void* const* dc,
                              void* const* workspace, const size_t* ws_bytes, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!plans || !A || !b || !c || !drho || !dA || !db || !dc || !workspace || !ws_bytes)))
    return fail(FD_ERR_INVALID_ARG, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    const void* sv = saved ? saved[i] : nullptr;
    const size_t sb = (saved && saved_bytes) ? saved_bytes[i] : 0;
    fd_status s = fock_diag_vjp(plans[i], A[i], b[i], c[i], sv, sb, drho[i], dA[i], db[i], dc[i], workspace[i],
                                ws_bytes[i], stream);
    if (s != FD_OK) return fail(s, "circuit " + std::to_string(i) + ": " + g_err);
  }
  return ok();
}

fd_status fd_batch_set_tuning(const fd_batch_tuning* t) {
  if (!t) return fail(FD_ERR_INVALID_ARG, "tuning is NULL");
  if (fd::batch_set_tuning(*t) != FD_OK) return fail(FD_ERR_INVALID_ARG, "batch tuning values out of range");
  return ok();
}

fd_status fd_batch_get_tuning(fd_batch_tuning* t) {
  if (!t) return fail(FD_ERR_INVALID_ARG, "tuning is NULL");
  *t = fd::batch_get_tuning();
  return ok();
}

fd_status fd_plan_use_graphs(fd_plan p, int enable) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  p->P.use_graphs = enable != 0;
  if (!enable) drop_graphs(p->P);
  return ok();
}

fd_status fd_plan_timing(fd_plan p, uint32_t kind_mask) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Timing& T = p->P.timing;
  for (auto& v : T.rec) {
    for (auto& pr : v) {
      T.pool.push_back(pr.first);
      T.pool.push_back(pr.second);
    }
    v.clear();
  }
  T.mask = kind_mask;
  return ok();
}

fd_status fd_plan_kernel_times(fd_plan p, int kind, int64_t* launches, double* total_ms) {
  if (!p || !launches || !total_ms || kind < 0 || kind >= fd::KK_COUNT)
    return fail(FD_ERR_INVALID_ARG, "bad timing query");
  fd::Timing& T = p->P.timing;
  double tot = 0.0;
  for (auto& pr : T.rec[kind]) {
    if (hipEventSynchronize(pr.second) != hipSuccess) return fail(FD_ERR_HIP, "hipEventSynchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess)
      return fail(FD_ERR_HIP, "hipEventElapsedTime failed");
    tot += ms;
  }
  *launches = (int64_t)T.rec[kind].size();
  *total_ms = tot;
  for (auto& pr : T.rec[kind]) {
    T.pool.push_back(pr.first);
    T.pool.push_back(pr.second);
  }
  T.rec[kind].clear();
  return ok();
}

const char* fd_last_error(void) { return g_err.c_str(); }

fd_status fd_state_plan_create(int M, const int* cutoffs, fd_dtype dt, uint32_t flags, fd_state_plan* out) {
  if (!out) return fail(FD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (M < 1 || M > 16) return fail(FD_ERR_INVALID_ARG, "M must be in [1, 16]");
  fd_state_plan sp = new (std::nothrow) fd_state_plan_s;
  if (!sp) return fail(FD_ERR_OOM, "host allocation failed");
  const uint32_t all = M >= 32 ? 0xffffffffu : ((1u << M) - 1u);
  fd_status s = fd_plan_create(M, cutoffs, all, dt, flags, &sp->inner);
  if (s != FD_OK) {
    delete sp;
    return s;
  }
  *out = sp;
  return ok();
}

fd_status fd_state_plan_destroy(fd_state_plan sp) {
  if (!sp) return ok();
  fd_status s = fd_plan_destroy(sp->inner);
  delete sp;
  return s;
}

fd_status fd_state_plan_workspace(fd_state_plan sp, size_t* bytes) {
  if (!sp || !bytes) return fail(FD_ERR_INVALID_ARG, "NULL argument");
  *bytes = fd::state_ws_bytes(sp->inner->P);
  return ok();
}

fd_status fock_state_fwd(fd_state_plan sp, const void* A, const void* b, const void* c, void* psi, void* workspace,
                         size_t ws_bytes, hipStream_t stream) {
  if (!sp) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = sp->inner->P;
  fd_status s = check_ptrs(P, {A, b, c, psi, workspace});
  if (s != FD_OK) return s;
  if (!aligned(workspace, 256)) return fail(FD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < fd::state_ws_bytes(P)) return fail(FD_ERR_WORKSPACE, "workspace too small");
  bool b_zero = false;
  if ((s = decide_b_zero(P, b, stream, &b_zero, P.M)) != FD_OK) return s;
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  if (fd::run_state_fwd(P, b_zero, A, b, c, psi, workspace, stream) != hipSuccess)
    return fail(FD_ERR_HIP, "kernel launch failed");
  return ok();
}

fd_status fd_state_plan_vjp_workspace(fd_state_plan sp, size_t* bytes) {
  if (!sp || !bytes) return fail(FD_ERR_INVALID_ARG, "NULL argument");
  *bytes = fd::state_vjp_ws_bytes(sp->inner->P);
  return ok();
}

fd_status fock_state_vjp(fd_state_plan sp, const void* c, const void* psi, const void* dpsi, void* dA, void* db,
                         void* dc, void* workspace, size_t ws_bytes, hipStream_t stream) {
  if (!sp) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = sp->inner->P;
  fd_status s = check_ptrs(P, {c, psi, dpsi, dA, db, dc, workspace});
  if (s != FD_OK) return s;
  if (!aligned(workspace, 256)) return fail(FD_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < fd::state_vjp_ws_bytes(P)) return fail(FD_ERR_WORKSPACE, "workspace too small");
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  if (fd::run_state_vjp(P, c, psi, dpsi, dA, db, dc, workspace, stream) != hipSuccess)
    return fail(FD_ERR_HIP, "kernel launch failed");
  return ok();
}

fd_status fock_state_jvp(fd_state_plan sp, const void* c, const void* psi, const void* dA, const void* db,
                         const void* dc, void* dpsi, hipStream_t stream) {
  if (!sp) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = sp->inner->P;
  fd_status s = check_ptrs(P, {c, psi, dA, db, dc, dpsi});
  if (s != FD_OK) return s;
  std::string err;
  if ((s = fd::ensure_device(&P, &err)) != FD_OK) return fail(s, err);
  if (fd::run_state_jvp(P, c, psi, dA, db, dc, dpsi, stream) != hipSuccess)
    return fail(FD_ERR_HIP, "kernel launch failed");
  return ok();
}

fd_status fd_state_device_status(fd_state_plan sp, hipStream_t stream) {
  if (!sp) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  return fd_device_status(sp->inner, stream);
}

fd_status fd_state_plan_timing(fd_state_plan sp, uint32_t kind_mask) {
  if (!sp) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  return fd_plan_timing(sp->inner, kind_mask);
}

fd_status fd_state_plan_kernel_times(fd_state_plan sp, int kind, int64_t* launches, double* total_ms) {
  if (!sp) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  return fd_plan_kernel_times(sp->inner, kind, launches, total_ms);
}

fd_status fd_device_status(fd_plan p, hipStream_t stream) {
  if (!p) return fail(FD_ERR_INVALID_ARG, "plan is NULL");
  fd::Plan& P = p->P;
  if (!P.d_status) return ok();
  int h = 0;
  if (hipMemcpyAsync(&h, P.d_status, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipMemsetAsync(P.d_status, 0, sizeof(int), stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
    return fail(FD_ERR_HIP, "reading the device status failed");
  if (h & 1) return fail(FD_ERR_NONFINITE, "non-finite value seen on the device");
  if (h & 2) return fail(FD_ERR_INVALID_ARG, "plan made with FD_B_ZERO received a non-zero b");
  if (h & 4) return fail(FD_ERR_HIP, "a batched sweep gave up waiting at a step barrier (results invalid)");
  return ok();
}

}  // extern "C"
