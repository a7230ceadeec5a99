// Host-side argument validation for the libedm C ABI.
//
// Plain C++ (no HIP), so it runs before anything touches the device and can be
// exercised on a machine without a GPU.  Each check returns EDM_OK or an
// EDM_E_* code and fills `msg` with a human-readable reason.
#pragma once

#include <cstdint>
#include <string>

#include "../../include/edm.h"

namespace edm {

// Number of query points (= candidate neighbours) of a series of length L.
inline int64_t n_query(int64_t L, int32_t E, int32_t tau, int32_t Tp) {
  return L - static_cast<int64_t>(E - 1) * tau - Tp;
}

inline int fail(std::string &msg, int code, const std::string &why) {
  msg = why;
  return code;
}

inline int check_embedding(int64_t L, int32_t E, int32_t tau, int32_t Tp, int32_t k,
                           std::string &msg) {
  if (E < 1) return fail(msg, EDM_E_ARG, "E must be >= 1");
  if (tau < 1) return fail(msg, EDM_E_ARG, "tau must be >= 1");
  if (Tp < 0) return fail(msg, EDM_E_ARG, "Tp must be >= 0");
  if (k < 1 || k > EDM_K_MAX) return fail(msg, EDM_E_ARG, "k must be in 1..32 (0 means E+1)");
  if (L < 1) return fail(msg, EDM_E_ARG, "L must be >= 1");
  if (L > EDM_L_MAX) return fail(msg, EDM_E_ARG, "series longer than EDM_L_MAX");
  const int64_t nq = n_query(L, E, tau, Tp);
  if (nq - 1 < k) return fail(msg, EDM_E_SHORT, "series too short: need L-(E-1)*tau-Tp-1 >= k");
  return EDM_OK;
}

inline int check_embed(const void *x, int64_t L, int32_t E, int32_t tau, const void *out,
                       std::string &msg) {
  if (!x || !out) return fail(msg, EDM_E_ARG, "NULL pointer");
  if (E < 1) return fail(msg, EDM_E_ARG, "E must be >= 1");
  if (tau < 1) return fail(msg, EDM_E_ARG, "tau must be >= 1");
  if (L - static_cast<int64_t>(E - 1) * tau < 1) return fail(msg, EDM_E_SHORT, "series shorter than one embedded point");
  return EDM_OK;
}

inline int check_knn(const void *x, int64_t L, int32_t E, int32_t tau, int32_t Tp, int32_t k,
                     const void *idx, std::string &msg) {
  if (!x || !idx) return fail(msg, EDM_E_ARG, "NULL pointer (x and idx are required)");
  if (E > EDM_E_MAX) return fail(msg, EDM_E_ARG, "E must be <= 20");
  return check_embedding(L, E, tau, Tp, k == 0 ? E + 1 : k, msg);
}

inline int check_lookup(const void *idx, const void *w, int64_t nq, int32_t k, int32_t E,
                        int32_t tau, int32_t Tp, const void *Y, int64_t N, int64_t ldy,
                        const void *pred, const void *rho, std::string &msg) {
  if (!idx || !w || !Y) return fail(msg, EDM_E_ARG, "NULL pointer (idx, w and Y are required)");
  if (!pred && !rho) return fail(msg, EDM_E_ARG, "nothing to compute: pred and rho are both NULL");
  if (k < 1 || k > EDM_K_MAX) return fail(msg, EDM_E_ARG, "k must be in 1..32");
  if (E < 1 || tau < 1 || Tp < 0) return fail(msg, EDM_E_ARG, "E, tau >= 1 and Tp >= 0 required");
  if (N < 0) return fail(msg, EDM_E_ARG, "N must be >= 0");
  if (nq < 2 || nq - 1 < k) return fail(msg, EDM_E_SHORT, "table too short: need nq-1 >= k");
  const int64_t need = nq + static_cast<int64_t>(E - 1) * tau + Tp;
  if (need > EDM_L_MAX) return fail(msg, EDM_E_ARG, "series longer than EDM_L_MAX");
  if (ldy < need) return fail(msg, EDM_E_ARG, "ldy shorter than nq+(E-1)*tau+Tp");
  return EDM_OK;
}

inline int check_lengths(const int64_t *L, int64_t N, int64_t ld, std::string &msg) {
  if (N > 0 && !L) return fail(msg, EDM_E_ARG, "NULL length array");
  for (int64_t i = 0; i < N; ++i) {
    if (L[i] < 1) return fail(msg, EDM_E_ARG, "length < 1");
    if (L[i] > ld) return fail(msg, EDM_E_ARG, "length exceeds the leading dimension");
    if (L[i] > EDM_L_MAX) return fail(msg, EDM_E_ARG, "series longer than EDM_L_MAX");
  }
  return EDM_OK;
}

inline int check_sweep(const void *X, const int64_t *L, int64_t N, int64_t ldx, int32_t E_max,
                       int32_t tau, int32_t Tp, const void *rho, const void *E_opt,
                       std::string &msg) {
  if (N < 0) return fail(msg, EDM_E_ARG, "N must be >= 0");
  if (N > 0 && (!X || !rho || !E_opt)) return fail(msg, EDM_E_ARG, "NULL pointer");
  if (E_max < 1 || E_max > EDM_E_MAX) return fail(msg, EDM_E_ARG, "E_max must be in 1..20");
  if (tau < 1 || Tp < 0) return fail(msg, EDM_E_ARG, "tau >= 1 and Tp >= 0 required");
  return check_lengths(L, N, ldx, msg);
}

inline int check_ccm(const void *X, const int64_t *Lx, int64_t Nl, int64_t ldx, const void *Y,
                     const int64_t *Ly, int64_t Nt, int64_t ldy, const void *E_tgt, int32_t tau,
                     int32_t Tp, const void *rho, std::string &msg) {
  if (Nl < 0 || Nt < 0) return fail(msg, EDM_E_ARG, "Nl and Nt must be >= 0");
  if ((Nl > 0 && !X) || (Nt > 0 && (!Y || !E_tgt)) || (Nl > 0 && Nt > 0 && !rho))
    return fail(msg, EDM_E_ARG, "NULL pointer");
  if (tau < 1 || Tp < 0) return fail(msg, EDM_E_ARG, "tau >= 1 and Tp >= 0 required");
  int rc = check_lengths(Lx, Nl, ldx, msg);
  if (rc != EDM_OK) return rc;
  return check_lengths(Ly, Nt, ldy, msg);
}

}  // namespace edm
