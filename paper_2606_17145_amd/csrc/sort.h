// Device radix sort shared by the tree build and the particle-mesh assignment.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

// Words of the histogram buffer that sr_sort_keys64 needs for n keys.
int64_t sr_sort_hist_words(int64_t n);

// Stable LSD radix sort of n 64-bit keys with a 32-bit payload on `st`, 8 bits a
// pass over the low `passes` bytes of the keys.  keys[0] and idx[0] hold the
// input; the two buffers alternate, so the result is in buffer (passes & 1).
int sr_sort_keys64(uint64_t* const keys[2], uint32_t* const idx[2], int64_t n, int passes, uint32_t* hist,
                   hipStream_t st);
