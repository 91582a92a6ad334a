// Key of a captured iteration graph in the per-engine and per-batch graph caches (host only).
#pragma once

#include <cstdint>

namespace psara {

// The adaptive flag, the primal mode and the iteration count, each in its own bits, so that no
// two (adaptive, mode, count) triples share a key for any count in [0, 2^31) and mode in
// [0, 2^31).
inline uint64_t graph_key(bool adaptive, int mode, int count) {
  return ((uint64_t)(adaptive ? 1u : 0u) << 63) | ((uint64_t)(uint32_t)mode << 32) | (uint64_t)(uint32_t)count;
}

}  // namespace psara
