// Device twin of the Chung-Lu draw of gen.c, for filling device memory with a
// graph's draws directly. It reads copies of the host generator's tables and
// performs only integer arithmetic (Philox4x32-10 blocks, Lemire's
// multiply-shift, alias lookups, the splitmix64-based domain test), so draw i
// equals the host's draw i bit for bit. Input generation only: nothing here
// evaluates a query.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint32_t kPhM0 = 0xD2511F53u, kPhM1 = 0xCD9E8D57u, kPhW0 = 0x9E3779B9u, kPhW1 = 0xBB67AE85u;
constexpr uint32_t kTagCL = 2;

__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                       uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += kPhW0; k1 += kPhW1; }
    const uint64_t p0 = (uint64_t)kPhM0 * c0, p1 = (uint64_t)kPhM1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

struct Tables {
  const uint32_t *vthr; const int32_t *valias; int64_t n;
  const uint32_t *lthr; const int32_t *lalias; int32_t P;
  const int32_t *perm;
  uint64_t seed; int32_t dom_mod;
};

__device__ __forceinline__ int64_t alias_draw(const uint32_t *thr, const int32_t *alias, int64_t n, uint32_t r_idx,
                                              uint32_t r_coin) {
  const int64_t i = (int64_t)(((uint64_t)r_idx * (uint64_t)n) >> 32);
  return r_coin < thr[i] ? i : alias[i];
}

__global__ __launch_bounds__(256) void k_cl_draws(const Tables T, uint64_t idx0, int64_t count, int32_t *out) {
  const uint32_t k0 = (uint32_t)T.seed, k1 = (uint32_t)(T.seed >> 32);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t idx = idx0 + (uint64_t)i;
    uint32_t r[4];
    philox((uint32_t)idx, (uint32_t)(idx >> 32), kTagCL, 0, k0, k1, r);
    const int32_t s = T.perm[alias_draw(T.vthr, T.valias, T.n, r[0], r[1])];
    const int32_t p = 1 + (int32_t)alias_draw(T.lthr, T.lalias, T.P, r[2], r[3]);
    int32_t o = -1;
    for (uint32_t blk = 1; blk <= 48 && o < 0; ++blk) {   // up to 96 object attempts
      philox((uint32_t)idx, (uint32_t)(idx >> 32), kTagCL, blk, k0, k1, r);
      for (int t = 0; t < 2 && o < 0; ++t) {
        const int32_t v = T.perm[alias_draw(T.vthr, T.valias, T.n, r[2 * t], r[2 * t + 1])];
        const bool dom = T.dom_mod <= 1 ||
                         mix64(T.seed * 0x2545F4914F6CDD1Dull + (uint64_t)p * 0x100000001B3ull + (uint64_t)(uint32_t)v) %
                                 (uint64_t)T.dom_mod == 0;
        if (dom) o = v;
      }
    }
    int32_t *w = out + 3 * i;
    w[0] = o < 0 ? -1 : s;
    w[1] = o < 0 ? -1 : p;
    w[2] = o;
  }
}

}  // namespace

extern "C" {

// Draws [idx0, idx0 + count) into out (device, count * 3 int32), in draw order;
// a draw whose object rejection failed is written as (-1, -1, -1). Tables are
// device copies of the host generator's (gsw_cl_tables). Returns a hipError_t.
int gsw_dev_cl_draws(const uint32_t *vthr, const int32_t *valias, int64_t n, const uint32_t *lthr,
                     const int32_t *lalias, int32_t P, const int32_t *perm, uint64_t seed, int32_t dom_mod,
                     uint64_t idx0, int64_t count, int32_t *out, void *stream) {
  if (count <= 0) return 0;
  Tables T{vthr, valias, n, lthr, lalias, P, perm, seed, dom_mod};
  int64_t g = (count + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_cl_draws, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream, T, idx0, count, out);
  return (int)hipGetLastError();
}

}  // extern "C"
