// Host paths of the C ABI under AddressSanitizer / UndefinedBehaviorSanitizer:
// plans over many shapes (box and total cutoffs, undetected modes, cutoff-1
// modes), every query, the workspace layouts with and without checkpoints,
// level offsets, state plans, and argument errors.  No call reaches the GPU.
// The pivot count of Algorithm 1 with equal cutoffs is checked against the
// closed form 2 C^M - C^(M-1) - 1.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "fockdiag.h"

static int failures = 0;
#define CHECK(cond)                                                       \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                         \
    }                                                                     \
  } while (0)

static void exercise(fd_plan p, int M) {
  int64_t v = 0;
  for (int q = 0; q <= FD_Q_B_SCHEDULE; ++q) CHECK(fd_plan_query(p, q, &v) == FD_OK);
  CHECK(fd_plan_query(p, 99, &v) == FD_ERR_INVALID_ARG);
  size_t a = 0, b = 0;
  CHECK(fd_plan_workspace(p, 0, &a, &b) == FD_OK && b == 0);
  size_t ws0 = 0, sv0 = 0;
  CHECK(fd_plan_workspace(p, 1, &ws0, &sv0) == FD_OK);
  int64_t levels = 0;
  CHECK(fd_plan_query(p, FD_Q_LEVELS, &levels) == FD_OK);
  for (int every : {1, 2, 3, (int)levels, (int)levels + 2}) {
    CHECK(fd_plan_set_checkpoint(p, every) == FD_OK);
    size_t ws = 0, sv = 0;
    CHECK(fd_plan_workspace(p, 1, &ws, &sv) == FD_OK && sv > 0 && ws > 0);
  }
  CHECK(fd_plan_set_checkpoint(p, -1) == FD_ERR_INVALID_ARG);
  CHECK(fd_plan_set_checkpoint(p, 0) == FD_OK);
  size_t ws1 = 0, sv1 = 0;
  CHECK(fd_plan_workspace(p, 1, &ws1, &sv1) == FD_OK && ws1 == ws0 && sv1 == sv0);
  size_t jb = 0;
  CHECK(fd_plan_jvp_workspace(p, &jb) == FD_OK);
  std::vector<int64_t> off((size_t)levels + 1);
  const fd_status so = fd_plan_level_offsets(p, off.data(), (int)off.size());
  CHECK(so == FD_OK || so == FD_ERR_INVALID_ARG);
  // argument errors return before any device work
  CHECK(fock_diag_fwd(p, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr) == FD_ERR_INVALID_ARG);
  CHECK(fock_diag_vjp(p, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                      nullptr) != FD_OK);
  CHECK(fd_plan_use_graphs(p, 1) == FD_OK && fd_plan_use_graphs(p, 0) == FD_OK);
  CHECK(fd_plan_timing(p, 0) == FD_OK);
  (void)M;
}

int main() {
  std::mt19937 rng(12345);
  int made = 0;
  for (int t = 0; t < 400; ++t) {
    const int M = 1 + (int)(rng() % 8);
    std::vector<int> cut(M);
    for (int j = 0; j < M; ++j) cut[j] = 1 + (int)(rng() % 7);
    uint32_t mask = (uint32_t)(rng() % (1u << M));
    // at most two undetected modes with cutoff >= 2 (the compiled limit); others refused
    fd_plan p = nullptr;
    const fd_status s = fd_plan_create(M, cut.data(), mask, (t & 1) ? FD_C64 : FD_C128, (uint32_t)(t % 3), &p);
    if (s == FD_OK) {
      ++made;
      exercise(p, M);
      CHECK(fd_plan_destroy(p) == FD_OK);
    } else {
      CHECK(p == nullptr && fd_last_error()[0] != 0);
    }
  }
  CHECK(made > 100);
  for (int M = 1; M <= 6; ++M)
    for (int C = 2; C <= 6; ++C) {
      std::vector<int> cut(M, C);
      fd_plan p = nullptr;
      CHECK(fd_plan_create(M, cut.data(), (1u << M) - 1, FD_C128, FD_B_ZERO, &p) == FD_OK);
      int64_t piv = 0, cm = 1;
      for (int j = 0; j < M; ++j) cm *= C;
      CHECK(fd_plan_query(p, FD_Q_PIVOTS, &piv) == FD_OK && piv == 2 * cm - cm / C - 1);
      exercise(p, M);
      fd_plan_destroy(p);
      fd_plan q = nullptr;
      CHECK(fd_plan_create_total(M, cut.data(), C + 1, FD_C128, FD_B_AUTO, &q) == FD_OK);
      exercise(q, M);
      fd_plan_destroy(q);
      fd_state_plan sp = nullptr;
      CHECK(fd_state_plan_create(M, cut.data(), FD_C64, FD_B_AUTO, &sp) == FD_OK);
      size_t b1 = 0, b2 = 0;
      CHECK(fd_state_plan_workspace(sp, &b1) == FD_OK && fd_state_plan_vjp_workspace(sp, &b2) == FD_OK);
      CHECK(fd_state_plan_destroy(sp) == FD_OK);
    }
  // invalid shapes
  int bad[3] = {0, 4, 4};
  fd_plan p = nullptr;
  CHECK(fd_plan_create(3, bad, 7, FD_C128, 0, &p) == FD_ERR_INVALID_ARG);
  CHECK(fd_plan_create(0, bad, 0, FD_C128, 0, &p) == FD_ERR_INVALID_ARG);
  CHECK(fd_plan_create(3, nullptr, 7, FD_C128, 0, &p) == FD_ERR_INVALID_ARG);
  CHECK(fd_plan_create(3, bad + 1, 7, FD_C128, 0, nullptr) == FD_ERR_INVALID_ARG);
  CHECK(fd_plan_destroy(nullptr) == FD_OK);
  std::printf("host sanitizer driver: %d plans exercised, %d failures\n", made, failures);
  return failures ? 1 : 0;
}
