// Private host-side helpers shared by the libedm host files: the context
// structure, error reporting, the workspace and the pinned staging buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/edm.h"

struct edm_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int form = EDM_FORM_PLAIN;
  int32_t excl = 0;            // exclusion radius of the neighbour search (0: self only)
  std::string err;
  char *ws = nullptr;          // device workspace
  size_t ws_bytes = 0;
  int *status = nullptr;       // device status word
  float *dmat = nullptr;       // distance matrices of the two-kernel form
  size_t dmat_bytes = 0;
  char *pinned = nullptr;      // host staging buffer
  size_t pinned_bytes = 0;
  hipEvent_t pinned_ready = nullptr;  // recorded after the last copy out of `pinned`
  bool pinned_pending = false;
  // kernel timing (edm_ctx_set_timing): event pairs recorded around launches
  bool timing = false;
  struct TimedRange {
    int family;
    hipEvent_t start, stop;
  };
  std::vector<TimedRange> ranges;
  std::vector<hipEvent_t> spare_events;
};

namespace edm {
namespace host {

int set_err(edm_ctx *ctx, int code, const std::string &msg);
int hip_err(edm_ctx *ctx, hipError_t e, const char *what);
size_t align_up(size_t v, size_t a);
size_t workspace_limit();
int ws_reserve(edm_ctx *ctx, size_t bytes);
int upload(edm_ctx *ctx, const void *host, size_t bytes, void *dev);
int check_ctx(edm_ctx *ctx);
// Resolves this device's copy of the allocation-free entry point's static
// scratch (once per device; called by edm_ctx_create).
int noalloc_scratch_init(edm_ctx *ctx);

// While alive, kernel launches of this thread are timed on ctx (when its
// timing is on); one of these opens every C ABI call that launches kernels.
struct TimingScope {
  explicit TimingScope(edm_ctx *ctx);
  ~TimingScope();
  edm_ctx *prev;
};

// Sub-allocation plan inside a buffer.
struct Plan {
  size_t bytes = 0;
  size_t take(size_t n) {
    const size_t at = align_up(bytes, 256);
    bytes = at + n;
    return at;
  }
};

}  // namespace host
}  // namespace edm

#define EDM_HIP(ctx, call)                                            \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) return ::edm::host::hip_err(ctx, e_, #call); \
  } while (0)

#define EDM_RC(expr)               \
  do {                             \
    const int rc_ = (expr);        \
    if (rc_ != EDM_OK) return rc_; \
  } while (0)
