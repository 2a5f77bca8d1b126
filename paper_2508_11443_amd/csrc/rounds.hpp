// The flattened round schedule of the level-two search (rounds.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fks_internal.hpp"

namespace fks {

// Trial index of every bucket by the sortless rounds: keys (any order), the
// level-one constants, the 4-bit size words of the attempt, the host copy of
// the T level-two triples.  t_out (n bytes, zeroed by the caller) receives the
// trial of every bucket that finishes; *exhausted reports keys left after T
// rounds.  S bounds the flat cell space of a round.
int rounds_search(const uint64_t* keys, uint64_t n, uint64_t S, const Triple& A, uint64_t magic,
                  const uint32_t* words, const Triple* Ch, uint32_t T, uint8_t* t_out, bool* exhausted,
                  hipStream_t st);

}  // namespace fks
