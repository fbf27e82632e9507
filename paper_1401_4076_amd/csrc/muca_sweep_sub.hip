// muca_sweep_sub.hip -- equilibrium sweep with G lanes cooperating on one
// walker (paper Sec. 2: fixed weights, Metropolis acceptance
// min(1, W(E_n)/W(E_o)); Sec. 4: a sweep is L^d attempts).
//
// A Markov chain is sequential, so a walker's attempts are decided one after
// the other.  The G lanes of a walker share the work around each decision:
//  * batch phase (lane-parallel): lane l takes attempt t + l of the next G:
//    its Philox block, the particle k, the candidate sites c2, c3 with their
//    coordinates, and s_o = pos[k] read from the walker state;
//  * per attempt: the attempt's values are broadcast (DPP row broadcast for
//    16 lanes, readlane for 64), and one lane-parallel gather reads the
//    occupation of the 2d neighbours of s_o, of c2, c3 and of the 2d
//    neighbours of c2; each lane computes its site from per-lane constants
//    (axis, direction, periodic wrap), without branches;
//  * the threshold row T[E][.] stays in lanes 0..4d; every lane tests the
//    attempt's uniform u against its entry and a ballot picks the entry of
//    the attempt's dE;
//  * an accepted move is written to the walker state and patched into the
//    prefetched s_o of the later attempts of the batch that chose the same
//    particle, so the prefetch always equals pos[k] at decision time.
// Random-number consumption, candidate order and decisions are those of the
// one-walker-per-lane kernel, so all layouts give identical results.
//
// kLds: walker state (occupation bits, particle sites and their packed
// coordinates) lives in LDS for the whole launch; otherwise occupation bits
// and sites stay in device memory (workgroup-coherent accesses, the group's
// bit layout: linear or bricked, see bit_ref) and the coordinates of s_o are
// recomputed in the batch phase.  kPipe (device memory only; the 16-lane
// layouts): the gathers of the next kPipe attempts (1 or 2) are issued before
// the current one is decided.
// spread (16 lanes only, per task): walkers sit in every spread-th 16-lane
// row, so a small population fills more wavefronts (layouts SUB16X2, SUB16X1,
// and per group in SUB16MIX).
#include "muca_kernels.h"

#pragma clang fp contract(off)

namespace muca {

namespace {

template <bool kLds>
__device__ __forceinline__ uint32_t ld(const uint32_t* p) {
  if constexpr (kLds) return *p;
  else return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <bool kLds>
__device__ __forceinline__ void st(uint32_t* p, uint32_t v) {
  if constexpr (kLds) *p = v;
  else __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bit `bit` (only its low 5 bits count) of word w.  v_bfe_u32 reads only the
// low 5 bits of its offset, so a linear site can be passed unmasked.
__device__ __forceinline__ uint32_t bit_at(uint32_t w, uint32_t bit) {
  return __builtin_amdgcn_ubfe(w, bit, 1u);
}

// Word and bit of a linear site; the site itself serves as the bit (see
// bit_at).
__device__ __forceinline__ BitRef linear_ref(uint32_t s) {
  return BitRef{__builtin_amdgcn_ubfe(s, 5u, 27u), s};
}

// Word and bit of a site: linear in LDS; in device memory the group's layout
// (linear or bricked, see bit_ref).
template <bool kLds>
__device__ __forceinline__ BitRef locate(const GroupDesc& g, uint32_t s, uint32_t xyz) {
  if constexpr (kLds) return linear_ref(s);
  else return bit_ref(g, s, xyz);
}

// The move s_o -> s_n: s_o is occupied and s_n empty, so toggling both bits
// clears the one and sets the other.
template <bool kLds>
__device__ __forceinline__ void flip(const GroupDesc& g, uint32_t* bits, uint32_t so,
                                     uint32_t sox, uint32_t sn, uint32_t snx) {
  const BitRef a = locate<kLds>(g, so, sox), b = locate<kLds>(g, sn, snx);
  if constexpr (kLds) {
    atomicXor(&bits[a.word], 1u << (a.bit & 31u));
    atomicXor(&bits[b.word], 1u << (b.bit & 31u));
  } else {
    __hip_atomic_fetch_xor(&bits[a.word], 1u << (a.bit & 31u), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_xor(&bits[b.word], 1u << (b.bit & 31u), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Word i (0..3) of a Philox block, as two selects (no indexed array).
__device__ __forceinline__ uint32_t pick4(const U4& q, int i) {
  const uint32_t lo = (i & 1) ? q.y : q.x;
  const uint32_t hi = (i & 1) ? q.w : q.z;
  return (i & 2) ? hi : lo;
}

// Per-lane constants of one neighbour role: coordinate field, edge value,
// step and wrapped step along the lane's axis and direction.
struct NbrRole {
  uint32_t shift, edge;
  int32_t step, wrap;    // of the linear index
  uint32_t cstep, cwrap;  // of the packed coordinates (mod 2^32)
};

__device__ __forceinline__ NbrRole make_role(const GroupDesc& g, int dir) {
  NbrRole r{0u, 0xFFFFFFFFu, 0, 0, 0u, 0u};  // dir < 0: the site itself
  if (dir < 0) return r;
  const int axis = dir >> 1;
  const int32_t stride = axis == 0 ? 1 : (axis == 1 ? g.L : g.LL);
  r.shift = kXyzBits * (uint32_t)axis;
  const uint32_t unit = 1u << r.shift;
  if ((dir & 1) == 0) {
    r.edge = (uint32_t)(g.L - 1);
    r.step = stride;
    r.wrap = -(g.L - 1) * stride;
    r.cstep = unit;
    r.cwrap = 0u - (uint32_t)(g.L - 1) * unit;
  } else {
    r.edge = 0u;
    r.step = -stride;
    r.wrap = (g.L - 1) * stride;
    r.cstep = 0u - unit;
    r.cwrap = (uint32_t)(g.L - 1) * unit;
  }
  return r;
}

// Linear index and bit location of the role's site.
template <bool kLds>
__device__ __forceinline__ uint32_t role_locate(const GroupDesc& g, const NbrRole& r,
                                                uint32_t lin, uint32_t xyz, BitRef& at) {
  const bool edge = ((xyz >> r.shift) & kXyzMask) == r.edge;
  const uint32_t s = lin + (uint32_t)(edge ? r.wrap : r.step);
  if constexpr (kLds) {
    at = linear_ref(s);
  } else {
    at = bit_ref(g, s, xyz + (edge ? r.cwrap : r.cstep));
  }
  return s;
}

template <int G>
__device__ __forceinline__ uint32_t sub_mask(uint64_t ballot, int base) {
  if constexpr (G == 64) return (uint32_t)ballot;
  else return (uint32_t)(ballot >> base) & ((1u << G) - 1u);
}

// Broadcast of lane A of each 16-lane row: one 64-bit DPP move (row_newbcast
// is among the DPP controls of gfx950's 64-bit moves) carries two values.
// Every lane of every row is written, so no old value is needed.
template <int A>
__device__ __forceinline__ uint64_t row_bcast64(uint64_t v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + A, 0xF, 0xF, true);
}

__device__ __forceinline__ uint64_t pair(uint32_t low, uint32_t high) {
  return (uint64_t)low | ((uint64_t)high << 32);
}
__device__ __forceinline__ uint32_t lo(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t hi(uint64_t v) { return (uint32_t)(v >> 32); }

// One attempt's broadcast values, this lane's gather site, the site's bit in
// the loaded word, and the word (pipelined device-memory path).
struct Pend {
  uint32_t k, u, c2, c2x, c3, c3x, so, sox, site, sh, v;
};

constexpr uint32_t kNone = 0xFFFFFFFFu;  // no particle index or site (V <= 2^24)

// Walker state and per-lane constants of one cooperative walker.
template <int G, bool kLds, bool kTbl>
struct Walker {
  const GroupDesc* g;
  uint32_t* bits;
  uint32_t* plin;  // particle sites (device-memory mode)
  uint64_t* pp;    // LDS mode: (site, packed coordinates) of every particle
  const uint32_t* th;  // threshold table (LDS copy or device memory)
  int32_t* hist;
  int ls, base, d2, nd;
  uint32_t V, N, key0, seed32;
  int32_t E;  // energy minus the window's e_lo (bin index) during the launch
  uint64_t t;
  uint32_t tun;  // tunnelling state (see tunnel_step)
  uint32_t Trow;
  // lane roles of the main gather: [0,2d) nbr(s_o), 2d: c2, 2d+1: c3,
  // [2d+2, 4d+2) nbr(c2) and, when 6d+2 lanes are available (full), also
  // [4d+2, 6d+2) nbr(c3).  With state in device memory the gather is bound
  // by line fetches, so c3 and its neighbours (needed only when c2 is
  // occupied, probability ~rho) are not read speculatively: lane 2d+1 reads
  // c2's word again and c3 is read in the rare path.
  NbrRole role;
  bool role_so, role_c3, full;
  NbrRole role2;  // lanes [0, 2d): nbr of s_n in the second gather
  // batch values of lane ls (attempt t + ls)
  // kept in pairs (low word, high word) so that one 64-bit DPP broadcast
  // moves two values: (k, u), (c2, c2x), (c3, c3x), (s_o, s_o coordinates)
  uint64_t b_ku, b_c2p, b_c3p, b_sop;
  // device-memory path: the previous attempt's move (particle, old and new
  // site; kNone if rejected), the one before it (pm2_*, read by the two-deep
  // pipeline) and the fetch of the next batch's first attempt
  uint32_t pm_k, pm_so, pm_sn, pm_snx;
  uint32_t pm2_k, pm2_so, pm2_sn, pm2_snx;
  Pend next;
};

template <int G, bool kLds, bool kTbl>
__device__ __forceinline__ void batch_phase(Walker<G, kLds, kTbl>& W, uint64_t t0) {
  const GroupDesc& g = *W.g;
  const uint64_t tl = t0 + (uint64_t)W.ls;
  const U4 r = philox((uint32_t)tl, (uint32_t)(tl >> 32), 0u, 0u, W.key0, W.seed32);
  const uint32_t k = draw(r.x, W.N);
  const uint32_t c2 = draw(r.z, W.V), c3 = draw(r.w, W.V);
  W.b_ku = pair(k, r.y);
  W.b_c2p = pair(c2, site_xyz(g, c2));
  W.b_c3p = pair(c3, site_xyz(g, c3));
  if constexpr (kLds) {
    W.b_sop = W.pp[k];
  } else {
    const uint32_t so = ld<kLds>(&W.plin[k]);
    W.b_sop = pair(so, site_xyz(g, so));
  }
}

// This lane's site in the main gather of an attempt and its bit location.
// (Plain values, not a struct reference: a select between fields of one
// struct can be turned into an indexed stack load.)
template <int G, bool kLds, bool kTbl>
__device__ __forceinline__ uint32_t gather_site(const Walker<G, kLds, kTbl>& W, uint32_t so,
                                                uint32_t sox, uint32_t c2, uint32_t c2x,
                                                uint32_t c3, uint32_t c3x, BitRef& at) {
  const uint32_t blin = W.role_so ? so : (W.role_c3 ? c3 : c2);
  const uint32_t bxyz = W.role_so ? sox : (W.role_c3 ? c3x : c2x);
  return role_locate<kLds>(*W.g, W.role, blin, bxyz, at);
}

// The decision of attempt ta from the occupancy masks of its main gather
// (m: occupied role sites, nm: occupied and not s_o; bit i = role lane i of
// the walker), then the move.
template <int G, bool kLds, bool kTbl>
__device__ __forceinline__ void resolve(Walker<G, kLds, kTbl>& W, uint32_t k, uint32_t u,
                                        uint32_t c2, uint32_t c2x, uint32_t c3, uint32_t c3x,
                                        uint32_t so, uint32_t sox, uint64_t ta, uint32_t m,
                                        uint32_t nm, uint64_t ok) {
  const GroupDesc& g = *W.g;
  const int d2 = W.d2;
  const uint32_t dmask = (1u << d2) - 1u;
  const int ko = __popc(m & dmask);
  const bool c2free = !((m >> d2) & 1u);
  bool c3free = !((m >> (d2 + 1)) & 1u);  // LDS state only (speculative c3)
  uint32_t sn = c2free ? c2 : c3;
  uint32_t snx = c2free ? c2x : c3x;
  int kn = __popc((nm >> (c2free ? d2 + 2 : 2 * d2 + 2)) & dmask);
  if (!c2free && !(W.full && c3free)) {
    if constexpr (!kLds) {
      const BitRef a3 = locate<kLds>(g, c3, c3x);
      const uint32_t w3 = ld<kLds>(&W.bits[a3.word]);
      c3free = !bit_at(w3, a3.bit);
    }
    if (!c3free) {
      // both candidates occupied: words 0..3 of blocks 1, 2, ... in order
      uint32_t blk = 0;
      for (;;) {
        blk += 1;
        const U4 q = philox((uint32_t)ta, (uint32_t)(ta >> 32), blk, 0u, W.key0, W.seed32);
        const int l4 = W.ls & 3;
        const uint32_t word = pick4(q, l4);
        const uint32_t cand = draw(word, W.V);
        uint32_t vv = 0;
        BitRef ac = linear_ref(cand);
        if constexpr (!kLds) ac = bit_of(g, cand);
        if (W.ls < 4) vv = ld<kLds>(&W.bits[ac.word]);
        const bool fr = (W.ls < 4) && !bit_at(vv, ac.bit);
        const uint32_t fm = sub_mask<G>(__ballot(fr), W.base) & 0xFu;
        if (fm) {
          const int first = __ffs(fm) - 1;
          sn = draw(pick4(q, first), W.V);
          snx = site_xyz(g, sn);
          break;
        }
      }
    }
    // second gather: neighbours of s_n, not counting s_o
    BitRef at3;
    const uint32_t s3 = role_locate<kLds>(g, W.role2, sn, snx, at3);
    uint32_t v3 = 0;
    const bool on3 = W.ls < d2;
    if (on3) v3 = ld<kLds>(&W.bits[at3.word]);
    const bool occ3 = on3 && bit_at(v3, at3.bit) && (s3 != so);
    kn = __popc(sub_mask<G>(__ballot(occ3), W.base));
  }
  const int dE = ko - kn;
  const bool acc = (ok >> (W.base + dE + d2)) & 1u;
  if (acc && W.ls == 0) {
    if constexpr (kLds) W.pp[k] = pair(sn, snx);
    else st<kLds>(&W.plin[k], sn);
    flip<kLds>(g, W.bits, so, sox, sn, snx);
  }
  if constexpr (!kLds) {
    if (acc) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  }
  if constexpr (!kLds) {
    W.pm2_k = W.pm_k;
    W.pm2_so = W.pm_so;
    W.pm2_sn = W.pm_sn;
    W.pm2_snx = W.pm_snx;
    W.pm_k = acc ? k : kNone;
    W.pm_so = acc ? so : kNone;
    W.pm_sn = acc ? sn : kNone;
    W.pm_snx = snx;
  }
  // later attempts of this batch that chose the same particle see its new site
  const bool take = acc && (lo(W.b_ku) == k);
  W.b_sop = take ? pair(sn, snx) : W.b_sop;
  W.E += acc ? dE : 0;
  // W.E = E - e_lo < 2^24 and nd <= 13: a full-rate 24-bit product
  if (acc && dE != 0 && W.ls < W.nd)
    W.Trow = W.th[__umul24((uint32_t)W.E, (uint32_t)W.nd) + (uint32_t)W.ls];
}

// One attempt with the broadcast values of attempt ta (state in LDS).
template <int G, bool kLds, bool kTbl>
__device__ __forceinline__ void attempt(Walker<G, kLds, kTbl>& W, uint32_t k, uint32_t u,
                                        uint32_t c2, uint32_t c2x, uint32_t c3, uint32_t c3x,
                                        uint32_t so, uint32_t sox, uint64_t ta) {
  BitRef at;
  const uint32_t site = gather_site(W, so, sox, c2, c2x, c3, c3x, at);
  // Every lane loads (a lane without a role reads its base site, a valid
  // word) and the masks only look at bits of lanes with roles, so the
  // ballots need no lane predicate.  Bits above the walker's 16 may belong
  // to the next walker of the wave; every use selects its own bits.
  const uint32_t v = ld<kLds>(&W.bits[at.word]);
  __builtin_amdgcn_sched_barrier(0);  // issue the gather before waiting on the row below
  // while the gather is in flight: every lane of the threshold row tests u
  // (accepts(): T = kAlways or u < T; lanes past the row hold 0, never); the
  // entry of the attempt's dE decides
  const uint64_t ok = __ballot(u < W.Trow) | __ballot(W.Trow == kAlways);
  const uint32_t m = (uint32_t)(__ballot(bit_at(v, at.bit) != 0u) >> W.base);
  const uint32_t nm = m & ~(uint32_t)(__ballot(site == so) >> W.base);  // occupied, not s_o
  resolve<G, kLds, kTbl>(W, k, u, c2, c2x, c3, c3x, so, sox, ta, m, nm, ok);
}

// ---- device-memory state: the gather of attempt a + 1 is issued before
// attempt a is decided, so its memory latency overlaps the decision.  When
// a + 1 is decided, the gathered bits are corrected for a's move (s_o empty,
// s_n occupied; either value of the word is corrected the same way), and if
// that move displaced a + 1's particle, its neighbourhood is read again.
// (With state in LDS the extra instructions cost more than the LDS latency
// they hide, so that path decides each attempt after its own gather.)

template <int G, bool kLds, bool kTbl>
__device__ __forceinline__ void gather(const Walker<G, kLds, kTbl>& W, Pend& p) {
  BitRef at;
  p.site = gather_site(W, p.so, p.sox, p.c2, p.c2x, p.c3, p.c3x, at);
  p.sh = at.bit;
  p.v = ld<kLds>(&W.bits[at.word]);
}

template <int A, int G, bool kLds, bool kTbl>
__device__ __forceinline__ Pend fetch16(const Walker<G, kLds, kTbl>& W) {
  Pend p;
  const uint64_t ku = row_bcast64<A>(W.b_ku), c2p = row_bcast64<A>(W.b_c2p);
  const uint64_t c3p = row_bcast64<A>(W.b_c3p), sop = row_bcast64<A>(W.b_sop);
  p.k = lo(ku);
  p.u = hi(ku);
  p.c2 = lo(c2p);
  p.c2x = hi(c2p);
  p.c3 = lo(c3p);
  p.c3x = hi(c3p);
  p.so = lo(sop);
  p.sox = hi(sop);
  gather(W, p);
  return p;
}

template <int G, bool kLds, bool kTbl>
__device__ __forceinline__ Pend fetch64(const Walker<G, kLds, kTbl>& W, int a) {
  Pend p;
  p.k = __builtin_amdgcn_readlane(lo(W.b_ku), a);
  p.u = __builtin_amdgcn_readlane(hi(W.b_ku), a);
  p.c2 = __builtin_amdgcn_readlane(lo(W.b_c2p), a);
  p.c2x = __builtin_amdgcn_readlane(hi(W.b_c2p), a);
  p.c3 = __builtin_amdgcn_readlane(lo(W.b_c3p), a);
  p.c3x = __builtin_amdgcn_readlane(hi(W.b_c3p), a);
  p.so = __builtin_amdgcn_readlane(lo(W.b_sop), a);
  p.sox = __builtin_amdgcn_readlane(hi(W.b_sop), a);
  gather(W, p);
  return p;
}

// Decision of a fetched attempt.  Its gather was issued D decisions earlier
// (D = 1 or 2), so the moves of those D attempts (pm2_* the older, pm_* the
// newer) are applied to the gathered bits, oldest first; if one of them moved
// this attempt's particle, its neighbourhood is read again from the new site.
template <int D, int G, bool kLds, bool kTbl>
__device__ __forceinline__ void decide(Walker<G, kLds, kTbl>& W, Pend p, uint64_t ta) {
  const uint64_t ok = __ballot(p.u < W.Trow) | __ballot(W.Trow == kAlways);  // as in attempt()
  uint32_t bit = bit_at(p.v, p.sh);
  if constexpr (D == 2) bit = (p.site == W.pm2_sn) ? 1u : ((p.site == W.pm2_so) ? 0u : bit);
  bit = (p.site == W.pm_sn) ? 1u : ((p.site == W.pm_so) ? 0u : bit);
  const bool moved1 = p.k == W.pm_k;
  bool moved = moved1;
  if constexpr (D == 2) moved = moved1 || (p.k == W.pm2_k);
  if (__ballot(moved) != 0ull) {
    uint32_t nso = W.pm_sn, nsox = W.pm_snx;
    if constexpr (D == 2) {
      nso = moved1 ? W.pm_sn : W.pm2_sn;
      nsox = moved1 ? W.pm_snx : W.pm2_snx;
    }
    p.so = moved ? nso : p.so;
    p.sox = moved ? nsox : p.sox;
    BitRef at;
    const uint32_t site = gather_site(W, p.so, p.sox, p.c2, p.c2x, p.c3, p.c3x, at);
    const uint32_t v = ld<kLds>(&W.bits[at.word]);
    bit = moved ? bit_at(v, at.bit) : bit;
    p.site = moved ? site : p.site;
  }
  const uint32_t m = (uint32_t)(__ballot(bit != 0u) >> W.base);
  const uint32_t nm = m & ~(uint32_t)(__ballot(p.site == p.so) >> W.base);
  resolve<G, kLds, kTbl>(W, p.k, p.u, p.c2, p.c2x, p.c3, p.c3x, p.so, p.sox, ta, m, nm, ok);
}

// Attempts A..nb-2 of a 16-lane batch; cur holds attempt A's fetch.  Returns
// the fetch of the batch's last attempt, still undecided.
template <int A, int G, bool kLds, bool kTbl>
__device__ __forceinline__ Pend run16(Walker<G, kLds, kTbl>& W, Pend cur, int nb) {
  if constexpr (A == 15) {
    return cur;
  } else {
    if (A + 1 == nb) return cur;
    const Pend nxt = fetch16<A + 1, G, kLds, kTbl>(W);
    decide<1, G, kLds, kTbl>(W, cur, W.t + (uint64_t)A);
    return run16<A + 1, G, kLds, kTbl>(W, nxt, nb);
  }
}

// Two-deep pipeline over a full batch of 16: attempt A is decided after the
// gather of A + 2 is issued.  a, b hold the fetches of attempts A and A + 1;
// on return they hold those of attempts 14 and 15, still undecided.
template <int A, int G, bool kLds, bool kTbl>
__device__ __forceinline__ void run16x2(Walker<G, kLds, kTbl>& W, Pend& a, Pend& b) {
  if constexpr (A < 14) {
    const Pend c = fetch16<A + 2, G, kLds, kTbl>(W);
    decide<2, G, kLds, kTbl>(W, a, W.t + (uint64_t)A);
    a = b;
    b = c;
    run16x2<A + 1, G, kLds, kTbl>(W, a, b);
  }
}

template <int A, int G, bool kLds, bool kTbl>
__device__ __forceinline__ void unrolled16(Walker<G, kLds, kTbl>& W, int nb) {
  if constexpr (A < 16) {
    if (A < nb) {
      const uint64_t ku = row_bcast64<A>(W.b_ku), c2p = row_bcast64<A>(W.b_c2p);
      const uint64_t c3p = row_bcast64<A>(W.b_c3p), sop = row_bcast64<A>(W.b_sop);
      attempt<G, kLds, kTbl>(W, lo(ku), hi(ku), lo(c2p), hi(c2p), lo(c3p), hi(c3p), lo(sop),
                             hi(sop), W.t + (uint64_t)A);
      unrolled16<A + 1, G, kLds, kTbl>(W, nb);
    }
  }
}

// One set of walkers (one task) for `sweeps` sweeps, by the whole block.
// kPipe: 0 = each attempt decided after its own gather (LDS state, or the
// 64-lane layout), 1 or 2 = that many gathers ahead (device-memory state,
// 16 lanes; 2 needs every group's V to be a multiple of 16).
template <int G, bool kLds, bool kTbl, int kPipe>
__device__ __forceinline__ void run_set(
    const GroupDesc* __restrict__ groups, const SweepTask task, uint32_t* smem,
    uint32_t* __restrict__ gbits, uint32_t* __restrict__ gpos, int32_t* __restrict__ gE,
    uint64_t* __restrict__ gT, uint32_t* __restrict__ gtun, const uint32_t* __restrict__ thr,
    int32_t* __restrict__ H, const int32_t* __restrict__ active, int sweeps, uint32_t first_id,
    uint32_t seed32, int tbl_words, int hist_words) {
  if (active && !active[task.group]) return;  // uniform per block
  const int spread = task.spread;
  const GroupDesc g = groups[task.group];
  Walker<G, kLds, kTbl> W;
  W.g = &g;
  W.ls = threadIdx.x & (G - 1);
  W.base = (threadIdx.x & 63) & ~(G - 1);
  // spread > 1 (16 lanes per walker only): a walker in every spread-th row,
  // the other rows idle, so that a small population fills more wavefronts
  const int row = threadIdx.x / G;
  const int slot = row / spread;
  const bool has = (row % spread) == 0 && slot < task.count;
  const int w = task.first + slot;
  const int64_t j = w - g.first_walker;
  W.d2 = 2 * g.d;
  W.nd = g.nd;
  W.V = (uint32_t)g.V;
  W.N = (uint32_t)g.N;
  uint32_t* sb = gbits + g.bits_off + j * g.words;
  uint32_t* sp = gpos + g.pos_off + j * g.N;
  // the group's threshold table goes to LDS when the launch reserved room
  if constexpr (kTbl) {
    const uint32_t* src = thr + g.thr_off;
    const int n = g.nbins * g.nd;
    for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = src[i];
  }
  int32_t* lhist = reinterpret_cast<int32_t*>(smem + tbl_words);
  if constexpr (kLds) {
    for (int i = threadIdx.x; i < g.nbins; i += blockDim.x) lhist[i] = 0;
    // walker slots start 8-byte aligned: (site, coordinates) pairs, then bits
    uint32_t* state = smem + (((size_t)tbl_words + (size_t)hist_words + 1) & ~(size_t)1);
    const size_t stride = 2 * (size_t)g.N + (((size_t)g.words + 1) & ~(size_t)1);
    W.pp = reinterpret_cast<uint64_t*>(state + (size_t)slot * stride);
    W.bits = state + (size_t)slot * stride + 2 * (size_t)g.N;
    W.plin = nullptr;
    if (has) {
      for (int i = W.ls; i < g.words; i += G) W.bits[i] = sb[i];
      for (int i = W.ls; i < g.N; i += G) {
        const uint32_t s = sp[i];
        W.pp[i] = pair(s, site_xyz(g, s));
      }
    }
  } else {
    W.bits = sb;
    W.plin = sp;
    W.pp = nullptr;
  }
  __syncthreads();

  if (has) {
    const int d2 = W.d2;
    const int ls = W.ls;
    W.full = kLds && 3 * d2 + 2 <= G;
    const int nroles = W.full ? 3 * d2 + 2 : 2 * d2 + 2;
    W.role_so = ls < d2;
    W.role_c3 = kLds && ((ls == d2 + 1) || (ls >= 2 * d2 + 2 && ls < nroles));
    int dir = -1;
    if (ls < d2) dir = ls;
    else if (ls >= d2 + 2 && ls < 2 * d2 + 2) dir = ls - d2 - 2;
    else if (ls >= 2 * d2 + 2 && ls < nroles) dir = ls - 2 * d2 - 2;
    W.role = make_role(g, dir);
    W.role2 = make_role(g, ls < d2 ? ls : -1);
    if constexpr (kTbl) W.th = smem;
    else W.th = thr + g.thr_off;
    if constexpr (kLds) W.hist = lhist;  // summed over the block, flushed at the end
    else W.hist = H + g.bin_off;
    W.key0 = first_id + (uint32_t)w;
    W.seed32 = seed32;
    W.E = gE[w] - g.e_lo;
    W.t = gT[w];
    W.tun = gtun[w];
    W.Trow = (ls < W.nd) ? W.th[W.E * W.nd + ls] : 0u;
    // A batch never straddles the end of a sweep (the last batch of a sweep
    // may be short; its spare lanes compute attempts that the next batch
    // redoes), so the histogram entry is taken after the batch.
    if constexpr (kPipe == 0) {
      for (int sw = 0; sw < sweeps; ++sw) {
        for (uint32_t done = 0; done < W.V; done += G) {
          const int nb = (int)((W.V - done) < (uint32_t)G ? (W.V - done) : (uint32_t)G);
          batch_phase<G, kLds>(W, W.t);
          if constexpr (G == 16) {
            unrolled16<0, G, kLds, kTbl>(W, nb);
          } else {
            for (int a = 0; a < nb; ++a) {
              attempt<G, kLds, kTbl>(W, __builtin_amdgcn_readlane(lo(W.b_ku), a),
                                     __builtin_amdgcn_readlane(hi(W.b_ku), a),
                                     __builtin_amdgcn_readlane(lo(W.b_c2p), a),
                                     __builtin_amdgcn_readlane(hi(W.b_c2p), a),
                                     __builtin_amdgcn_readlane(lo(W.b_c3p), a),
                                     __builtin_amdgcn_readlane(hi(W.b_c3p), a),
                                     __builtin_amdgcn_readlane(lo(W.b_sop), a),
                                     __builtin_amdgcn_readlane(hi(W.b_sop), a),
                                     W.t + (uint64_t)a);
            }
          }
          W.t += (uint64_t)nb;
        }
        if (ls == 0) atomicAdd(&W.hist[W.E], 1);
        W.tun = tunnel_step(W.tun, W.E, g.nbins - 1);
      }
    } else if constexpr (kPipe == 2) {
      static_assert(G == 16, "the two-deep pipeline is for 16 lanes per walker");
      W.pm_k = W.pm_so = W.pm_sn = W.pm2_k = W.pm2_so = W.pm2_sn = kNone;
      W.pm_snx = W.pm2_snx = 0u;
      batch_phase<G, kLds>(W, W.t);
      Pend a = fetch16<0, G, kLds, kTbl>(W);
      Pend b = fetch16<1, G, kLds, kTbl>(W);
      for (int sw = 0; sw < sweeps; ++sw) {
        for (uint32_t done = 0; done < W.V; done += 16) {  // V % 16 == 0: full batches
          const bool more = (done + 16u < W.V) || (sw + 1 < sweeps);
          run16x2<0, G, kLds, kTbl>(W, a, b);  // attempts 0..13; a, b = 14, 15
          Pend n0 = a, n1 = b;
          // the next batch's values, then its first gathers, ahead of 14 and 15
          if (more) {
            batch_phase<G, kLds>(W, W.t + 16u);
            n0 = fetch16<0, G, kLds, kTbl>(W);
          }
          decide<2, G, kLds, kTbl>(W, a, W.t + 14u);
          if (more) n1 = fetch16<1, G, kLds, kTbl>(W);
          decide<2, G, kLds, kTbl>(W, b, W.t + 15u);
          W.t += 16u;
          a = n0;
          b = n1;
        }
        if (ls == 0) atomicAdd(&W.hist[W.E], 1);
        W.tun = tunnel_step(W.tun, W.E, g.nbins - 1);
      }
    } else {
      W.pm_k = W.pm_so = W.pm_sn = W.pm2_k = W.pm2_so = W.pm2_sn = kNone;
      W.pm_snx = W.pm2_snx = 0u;
      batch_phase<G, kLds>(W, W.t);
      if constexpr (G == 16) W.next = fetch16<0, G, kLds, kTbl>(W);
      else W.next = fetch64<G, kLds, kTbl>(W, 0);
      for (int sw = 0; sw < sweeps; ++sw) {
        for (uint32_t done = 0; done < W.V; done += G) {
          const int nb = (int)((W.V - done) < (uint32_t)G ? (W.V - done) : (uint32_t)G);
          const bool more = (done + (uint32_t)nb < W.V) || (sw + 1 < sweeps);
          Pend cur;
          if constexpr (G == 16) {
            cur = run16<0, G, kLds, kTbl>(W, W.next, nb);
          } else {
            cur = W.next;
            for (int a = 0; a + 1 < nb; ++a) {
              const Pend nxt = fetch64<G, kLds, kTbl>(W, a + 1);
              decide<1, G, kLds, kTbl>(W, cur, W.t + (uint64_t)a);
              cur = nxt;
            }
          }
          // the batch's last attempt; the next batch is fetched before it is decided
          if (more) {
            batch_phase<G, kLds>(W, W.t + (uint64_t)nb);
            if constexpr (G == 16) W.next = fetch16<0, G, kLds, kTbl>(W);
            else W.next = fetch64<G, kLds, kTbl>(W, 0);
          }
          decide<1, G, kLds, kTbl>(W, cur, W.t + (uint64_t)(nb - 1));
          W.t += (uint64_t)nb;
        }
        if (ls == 0) atomicAdd(&W.hist[W.E], 1);
        W.tun = tunnel_step(W.tun, W.E, g.nbins - 1);
      }
    }
    if (ls == 0) {
      gE[w] = W.E + g.e_lo;
      gT[w] = W.t;
      gtun[w] = W.tun;
    }
  }

  if constexpr (kLds) {
    __syncthreads();
    if (has) {
      for (int i = W.ls; i < g.words; i += G) sb[i] = W.bits[i];
      for (int i = W.ls; i < g.N; i += G) sp[i] = lo(W.pp[i]);
    }
    for (int i = threadIdx.x; i < g.nbins; i += blockDim.x)
      if (lhist[i]) atomicAdd(&H[g.bin_off + i], lhist[i]);
  }
}

}  // namespace

// Block b runs tasks [first[b], first[b + 1]) one after the other.
template <int G, bool kLds, bool kTbl, int kPipe>
__global__ void __launch_bounds__(256) k_sweep_sub(
    const GroupDesc* __restrict__ groups, const SweepTask* __restrict__ tasks,
    const int32_t* __restrict__ first, uint32_t* __restrict__ gbits,
    uint32_t* __restrict__ gpos, int32_t* __restrict__ gE, uint64_t* __restrict__ gT,
    uint32_t* __restrict__ gtun, const uint32_t* __restrict__ thr, int32_t* __restrict__ H,
    const int32_t* __restrict__ active, int sweeps, uint32_t first_id, uint32_t seed32,
    int tbl_words, int hist_words) {
  static_assert(G == 16 || G == 64, "16 or 64 lanes per walker");
  static_assert(!(kLds && kPipe), "the pipelined gather is for device-memory state");
  static_assert(kPipe >= 0 && kPipe <= 2 && (G == 16 || kPipe == 0), "pipeline depth");
  // LDS: [threshold table (tbl_words)] [block histogram (hist_words, LDS-state mode)]
  //      [walker slots]
  extern __shared__ uint32_t smem[];
  const int t0 = first[blockIdx.x], t1 = first[blockIdx.x + 1];
  for (int ti = t0; ti < t1; ++ti) {
    if (ti > t0) __syncthreads();  // the previous set is out of LDS
    run_set<G, kLds, kTbl, kPipe>(groups, tasks[ti], smem, gbits, gpos, gE, gT, gtun, thr, H,
                                  active, sweeps, first_id, seed32, tbl_words, hist_words);
  }
}

template __global__ void k_sweep_sub<16, true, true, 0>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<16, true, false, 0>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<16, false, true, 1>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<16, false, false, 1>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<16, false, true, 2>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<16, false, false, 2>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<64, true, true, 0>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<64, true, false, 0>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<64, false, true, 0>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);
template __global__ void k_sweep_sub<64, false, false, 0>(
    const GroupDesc*, const SweepTask*, const int32_t*, uint32_t*, uint32_t*, int32_t*,
    uint64_t*, uint32_t*, const uint32_t*, int32_t*, const int32_t*, int, uint32_t, uint32_t, int,
    int);

}  // namespace muca
