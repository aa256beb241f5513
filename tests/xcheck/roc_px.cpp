// Philox4x32-10 through rocRAND's engine (an independent, open-source
// implementation), for cross-checking the oracle's Philox.  The engine's
// ten-round block function is protected, so a derived struct exposes it.
// Reads records of six little-endian uint32 (c0 c1 c2 c3 k0 k1) from stdin,
// writes four uint32 per record to stdout.  Host-only use of the header.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdint>
#include <cstdio>
struct block_probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};
int main() {
  uint32_t r[6];
  block_probe p;
  while (fread(r, sizeof(uint32_t), 6, stdin) == 6) {
    uint4 c = {r[0], r[1], r[2], r[3]};
    uint2 k = {r[4], r[5]};
    uint4 o = p.block(c, k);
    uint32_t w[4] = {o.x, o.y, o.z, o.w};
    fwrite(w, sizeof(uint32_t), 4, stdout);
  }
  return 0;
}
