// Plain records shared by the device kernels and the host-side table builder
// (no HIP dependencies, so the host code that fills them can be built and
// tested by a plain C++ compiler).
#pragma once
#include <stdint.h>

namespace hentt {

// Moduli constants used by the butterflies.
struct ModQ {
  uint64_t q, nq, q2, nq2, q4, nq4;  // q, 2q, 4q and their negations mod 2^64
};

struct LimbConst {
  ModQ m;                   // q, 2q, 4q and their negations mod 2^64
  uint64_t ninv, ninv_s;    // N^-1 mod q and its Shoup quotient
  uint64_t ninvw, ninvw_s;  // N^-1 * psi^-brv(1) mod q and its Shoup quotient
  uint64_t mu;              // floor(2^(2k) / q), k = bit length of q (Barrett)
  uint32_t k, pad;
};

static_assert(sizeof(LimbConst) == 96, "limb records are 12 words (documented in the C ABI)");

// Montgomery constants of a limb (R = 2^64).
struct MontLimb {
  uint64_t qinv;   // -q^-1 mod 2^64
  uint64_t r, rs;  // R mod q and its Shoup quotient
  uint64_t pad;
};

// A root power and its Shoup quotient (W, W' = floor(W 2^64 / q)), Algorithm 1.
struct alignas(16) Tw { uint64_t w, ws; };

}  // namespace hentt
