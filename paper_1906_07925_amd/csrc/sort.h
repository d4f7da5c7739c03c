// Host interface of the stable LSD radix sort used for the cell keys.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpsph {

// Optional per-launch hook (event timing); begin() before a launch, end() after it.
struct LaunchHook {
  virtual void begin(const char *name) = 0;
  virtual void end() = 0;
  virtual ~LaunchHook() = default;
};

// Words of the histogram buffer for n keys.
size_t radix_hist_words(int n);
int radix_passes(int key_bits);

// Sort n keys (the low key_bits bits are significant) with the identity permutation as payload.
// k0/v0/k1/v1 are n-word ping-pong buffers; on return *keys_out / *perm_out point at the sorted
// keys and, for each sorted position, the input index it came from (stable).  Requires
// key_bits >= 1.  Enqueued on stream; no synchronisation.
hipError_t radix_sort(const uint32_t *keys_in, uint32_t *k0, uint32_t *v0, uint32_t *k1,
                      uint32_t *v1, uint32_t *hist, int n, int key_bits, hipStream_t stream,
                      const uint32_t **keys_out, const uint32_t **perm_out, LaunchHook *hook);

}  // namespace mpsph
