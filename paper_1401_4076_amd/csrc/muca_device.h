// muca_device.h -- device-side building blocks of libmuca (gfx950).
//
// Philox4x32-10 streams, the lattice geometry of the lattice gas (paper
// Sec. 3, eq. (5)), and binary64 exp/log built from IEEE-754 operations only,
// so that the acceptance thresholds and the weight recursion are reproducible
// bit for bit on any IEEE-754 machine.  Everything here is compiled with
// floating-point contraction off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace muca {

// Per-group constants, read by every kernel.  One entry per group.
struct GroupDesc {
  int32_t d, L, N, V;
  int32_t e_lo, e_hi, nbins, nd;  // nd = 4d + 1 columns of the threshold table
  int32_t bin_off;                // first bin in lnW / H / P
  int32_t thr_off;                // first entry of this group's threshold table
  int32_t first_walker, walkers;
  int32_t words;                  // 32-bit occupation words per walker
  int32_t LL;                     // L * L
  float invL;                     // 1/L rounded, used with an exact fix-up
  int32_t brick8;                 // L / 8 for a bricked bit layout, 0 for linear
  int64_t bits_off;               // first occupation word of the group's walker 0
  int64_t pos_off;                // first particle entry of the group's walker 0
};

// A set of walkers of the cooperative sweep: walkers [first, first + count)
// (global walker indices) of one group, placed in every spread-th 16-lane row
// of the block (spread 1 with 64 lanes per walker).
struct SweepTask {
  int32_t group, first, count, spread;
};

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): 10 rounds of two 32x32->64 products
// with the Weyl-sequence key schedule.
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    // one 32x32->64 product gives both halves (a single v_mad_u64_u32)
    const uint64_t pa = (uint64_t)0xD2511F53u * c0, pb = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t a = (uint32_t)pa, ah = (uint32_t)(pa >> 32);
    const uint32_t b = (uint32_t)pb, bh = (uint32_t)(pb >> 32);
    c0 = bh ^ c1 ^ k0;
    c1 = b;
    c2 = ah ^ c3 ^ k1;
    c3 = a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// {0..n-1} from a 32-bit word: floor(u n / 2^32).
__device__ __forceinline__ uint32_t draw(uint32_t u, uint32_t n) { return __umulhi(u, n); }

// ---------------------------------------------------------------- geometry
// Exact q = s / L for s < 2^24 via a float estimate and one correction.
__device__ __forceinline__ uint32_t div_L(uint32_t s, int32_t L, float invL) {
  int32_t q = (int32_t)((float)s * invL);
  int32_t r = (int32_t)s - q * L;
  q += (r >= L) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return (uint32_t)q;
}

// Packed coordinates x | y << 10 | z << 20 of site s = x + L y + L^2 z.
constexpr uint32_t kXyzBits = 10;
constexpr uint32_t kXyzMask = (1u << kXyzBits) - 1u;

__device__ __forceinline__ uint32_t site_xyz(const GroupDesc& g, uint32_t s) {
  const uint32_t q = div_L(s, g.L, g.invL);
  const uint32_t x = s - q * (uint32_t)g.L;
  if (g.d == 2) return x | (q << kXyzBits);
  const uint32_t z = div_L(q, g.L, g.invL);
  const uint32_t y = q - z * (uint32_t)g.L;
  return x | (y << kXyzBits) | (z << (2 * kXyzBits));
}

// ---------------------------------------------------------------- bit layout
// Where the occupation bit of a site lives in a walker's bit array.
// Linear: bit s % 32 of word s / 32.  Bricked (3D groups with L % 8 == 0
// whose state is too large for LDS, brick8 = L / 8): 8x8x8 bricks of 512
// bits (16 words, 64 bytes) in x-fastest brick order, inside a brick x
// fastest, then y, then z.  A site and its six neighbours then share one
// brick unless a neighbour crosses a face, where the linear layout puts the
// z neighbours 2 L^2 / 8 bytes apart: fewer lines fetched per gather.
struct BitRef {
  uint32_t word, bit;
};

__device__ __forceinline__ BitRef bit_ref(const GroupDesc& g, uint32_t s, uint32_t xyz) {
  if (g.brick8 == 0) return BitRef{s >> 5, s & 31u};
  const uint32_t x = xyz & kXyzMask, y = (xyz >> kXyzBits) & kXyzMask, z = xyz >> (2 * kXyzBits);
  const uint32_t nb = (uint32_t)g.brick8;
  const uint32_t b = ((z >> 3) * nb + (y >> 3)) * nb + (x >> 3);
  return BitRef{(b << 4) | ((z & 7u) << 1) | ((y & 7u) >> 2), (x & 7u) | ((y & 3u) << 3)};
}

__device__ __forceinline__ BitRef bit_of(const GroupDesc& g, uint32_t s) {
  if (g.brick8 == 0) return BitRef{s >> 5, s & 31u};
  return bit_ref(g, s, site_xyz(g, s));
}

// Occupation of site s in a walker's bit array, and the two single-bit updates.
__device__ __forceinline__ uint32_t occupied(const GroupDesc& g, const uint32_t* wb, uint32_t s) {
  const BitRef r = bit_of(g, s);
  return (wb[r.word] >> r.bit) & 1u;
}
__device__ __forceinline__ void set_site(const GroupDesc& g, uint32_t* wb, uint32_t s) {
  const BitRef r = bit_of(g, s);
  wb[r.word] |= 1u << r.bit;
}
__device__ __forceinline__ void clear_site(const GroupDesc& g, uint32_t* wb, uint32_t s) {
  const BitRef r = bit_of(g, s);
  wb[r.word] &= ~(1u << r.bit);
}

// The 2d neighbours of site s on the periodic lattice.
__device__ __forceinline__ void neighbours(const GroupDesc& g, uint32_t s, uint32_t nb[6]) {
  const int32_t L = g.L;
  const uint32_t q = div_L(s, L, g.invL);
  const uint32_t x = s - q * (uint32_t)L;
  nb[0] = (x == (uint32_t)(L - 1)) ? s - (uint32_t)(L - 1) : s + 1;
  nb[1] = (x == 0) ? s + (uint32_t)(L - 1) : s - 1;
  if (g.d == 2) {
    const uint32_t y = q;
    const uint32_t row = (uint32_t)L * (uint32_t)(L - 1);
    nb[2] = (y == (uint32_t)(L - 1)) ? s - row : s + (uint32_t)L;
    nb[3] = (y == 0) ? s + row : s - (uint32_t)L;
    nb[4] = nb[5] = 0;
  } else {
    const uint32_t z = div_L(q, L, g.invL);
    const uint32_t y = q - z * (uint32_t)L;
    const uint32_t row = (uint32_t)L * (uint32_t)(L - 1);
    const uint32_t slab = (uint32_t)g.LL * (uint32_t)(L - 1);
    nb[2] = (y == (uint32_t)(L - 1)) ? s - row : s + (uint32_t)L;
    nb[3] = (y == 0) ? s + row : s - (uint32_t)L;
    nb[4] = (z == (uint32_t)(L - 1)) ? s - slab : s + (uint32_t)g.LL;
    nb[5] = (z == 0) ? s + slab : s - (uint32_t)g.LL;
  }
}

// Neighbour of site s in direction dir: axis dir/2, +1 for even dir, -1 for odd.
__device__ __forceinline__ uint32_t neighbour1(const GroupDesc& g, uint32_t s, int dir) {
  const uint32_t L = (uint32_t)g.L;
  const uint32_t q = div_L(s, g.L, g.invL);
  const int axis = dir >> 1;
  const bool up = (dir & 1) == 0;
  uint32_t c, stride;
  if (axis == 0) {
    c = s - q * L;
    stride = 1;
  } else if (axis == 1) {
    c = (g.d == 2) ? q : q - div_L(q, g.L, g.invL) * L;
    stride = L;
  } else {
    c = div_L(q, g.L, g.invL);
    stride = (uint32_t)g.LL;
  }
  if (up) return (c == L - 1) ? s - (L - 1) * stride : s + stride;
  return (c == 0) ? s + (L - 1) * stride : s - stride;
}

// ---------------------------------------------------------------- exp / log
// Binary64 constants: ln 2 = HI + LO with HI carrying 29 significant bits
// (k * HI exact for |k| < 2^24), 1/ln 2 and sqrt(1/2), each the double
// nearest the exact value.
constexpr double kLn2Hi = 0x1.62e42ff000000p-1;
constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

constexpr double factorial(int n) { return n <= 1 ? 1.0 : (double)n * factorial(n - 1); }

// exp(x) for -23 <= x < 0: Cody-Waite reduction x = k ln2 + r, |r| <= ln2/2,
// Taylor polynomial of degree 13 with coefficients 1/n! (each the correctly
// rounded quotient), evaluated by Horner's rule, then scaled by 2^k.
__device__ __forceinline__ double exp_ieee(double x) {
  const double k = floor(x * kInvLn2 + 0.5);
  const double r = (x - k * kLn2Hi) - k * kLn2Lo;
  double q = 1.0 / factorial(13);
  q = q * r + 1.0 / factorial(12);
  q = q * r + 1.0 / factorial(11);
  q = q * r + 1.0 / factorial(10);
  q = q * r + 1.0 / factorial(9);
  q = q * r + 1.0 / factorial(8);
  q = q * r + 1.0 / factorial(7);
  q = q * r + 1.0 / factorial(6);
  q = q * r + 1.0 / factorial(5);
  q = q * r + 1.0 / factorial(4);
  q = q * r + 1.0 / factorial(3);
  q = q * r + 1.0 / factorial(2);
  q = q * r + 1.0;
  q = q * r + 1.0;
  return ldexp(q, (int)k);
}

// ln(h) for an integer h >= 1: h = m 2^e, m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(s), s = (m - 1)/(m + 1), odd series through s^21.
__device__ __forceinline__ double log_ieee(int32_t h) {
  int e;
  double m = frexp((double)h, &e);
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double q = 1.0 / 21.0;
  q = q * z + 1.0 / 19.0;
  q = q * z + 1.0 / 17.0;
  q = q * z + 1.0 / 15.0;
  q = q * z + 1.0 / 13.0;
  q = q * z + 1.0 / 11.0;
  q = q * z + 1.0 / 9.0;
  q = q * z + 1.0 / 7.0;
  q = q * z + 1.0 / 5.0;
  q = q * z + 1.0 / 3.0;
  q = q * z + 1.0;
  const double ln_m = (2.0 * s) * q;
  const double de = (double)e;
  return de * kLn2Hi + (de * kLn2Lo + ln_m);
}

// Threshold of the Metropolis rule min(1, exp(x)) for a 32-bit uniform u:
// 0xFFFFFFFF = always accept, otherwise accept iff u < T.
constexpr uint32_t kAlways = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t threshold(double x) {
  if (x >= 0.0) return kAlways;
  if (!(x >= -23.0)) return 0u;  // also NaN
  const double v = floor(ldexp(exp_ieee(x), 32));
  if (v >= 4294967295.0) return kAlways;
  return (uint32_t)v;
}

__device__ __forceinline__ bool accepts(uint32_t T, uint32_t u) {
  return (T == kAlways) | (u < T);
}

// ---------------------------------------------------------------- tunnelling
// Sec. 4 counts convergence in tunnelling events: trips of a walker from the
// top of the energy window to its bottom or back.  A walker's state packs
// the window end it visited last (bits 0-1: 0 none yet, 1 bottom, 2 top) and
// its completed trips (bits 2-31).  It is updated once per sweep, where the
// histogram entry is taken, with the walker's bin b (0 = e_lo, top = e_hi).
// A window of one bin never completes a trip.
__device__ __forceinline__ uint32_t tunnel_step(uint32_t st, int32_t b, int32_t top) {
  const uint32_t end = b == 0 ? 1u : (b == top ? 2u : 0u);
  const uint32_t last = st & 3u;
  if (end == 0u || end == last) return st;
  return ((st & ~3u) + (last != 0u ? 4u : 0u)) | end;
}

}  // namespace muca
