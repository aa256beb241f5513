// Philox4x32-10 through PyTorch's ATen engine (an independent, open-source
// implementation), for cross-checking the oracle's Philox.  Reads records of
// six little-endian uint32 (c0 c1 c2 c3 k0 k1) from stdin, writes four uint32
// per record to stdout.  The engine's seed is the key, its subsequence the
// counter's upper half and its offset the counter's lower half.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>
int main() {
  uint32_t r[6];
  while (fread(r, sizeof(uint32_t), 6, stdin) == 6) {
    uint64_t seed = (uint64_t)r[4] | ((uint64_t)r[5] << 32);
    uint64_t sub = (uint64_t)r[2] | ((uint64_t)r[3] << 32);
    uint64_t off = (uint64_t)r[0] | ((uint64_t)r[1] << 32);
    at::philox_engine e(seed, sub, off);
    uint32_t o[4];
    for (int i = 0; i < 4; ++i) o[i] = e();
    fwrite(o, sizeof(uint32_t), 4, stdout);
  }
  return 0;
}
