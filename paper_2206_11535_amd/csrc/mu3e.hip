// HIP kernels (gfx950) and C ABI of the online event selection.
//
// Plain form of the selection, per batch of frames:
//   k_cuts     one wave64 per frame, frames dealt cyclically to a static grid
//              (Section V-B, Alg. 1 and Alg. 2): the frame's layer-0..2 hits
//              are staged in LDS; per layer-1 hit a 128-bit mask of layer-0
//              partners passing the Phi01 window is built; (h1, h2) pairs
//              passing Phi12 are streamed through an LDS queue and each full
//              wave of pairs joins against its Phi01 partners (Delta lambda,
//              then r_tc); survivors are compacted with ballot/popcount into
//              the wave's chunks of a global triplet list.
//   k_scount / k_splace  tables of the 64-entry slices of the list's chunks.
//   k_tracks   one wave per slice, one lane per selected triplet (Alg. 3):
//              fit, layer-3 extension, second fit, weighted curvature,
//              chi2 < 32; the result is stored at the triplet's own index.
//   k_vcount / k_vplace  per frame: track cap; frames able to form an
//              e+e+e- triple get a slice of the candidate track table.
//   k_vprep    per accepted track of such frames: float64 refit.
//   k_vframes  one wave per candidate frame: energy test over the triples,
//              combination cap, vertex estimate and signal tests (Alg. 4).
// The batched form runs the cuts (and optionally the fits) in one
// persistent kernel and captures the whole sequence in a HIP graph.
//
// Decisions taken on float32 values are certain with respect to the exact
// value unless the value lies within a bound of its own rounding error around
// the edge; then the candidate is re-evaluated in float64.
//
// No shared counter is updated per frame or per triplet: device-scope
// atomics on one address serialise across the chip, so lists are handed out
// in chunks, results are stored in place and reservations are made per wave
// or by prefix sums.

#include "mu3e.h"
#include "mu3e_math.hpp"
#include "mu3e_window.hpp"
#include "mu3e_adjoint.hpp"

#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

// Workspace of mu3e_select_frames_static: one copy per device, held by each
// device the library runs on until the process ends.  Host code never passes
// this name to a kernel or a copy (on the host it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returns for the current
// device.
static __device__ __align__(256) unsigned char scratch[MU3E_STATIC_SCRATCH_BYTES];

using namespace mu3e;

namespace {

constexpr int kWave = 64;
constexpr int kCounters = 64;                // int32 counters at the workspace head
constexpr int kMinChunk = 64;                // triplet-list chunk sizes lie in [64, 4096]
constexpr int kMaxChunk = 4096;
constexpr int kMaxTripletCapacity = 1 << 30; // keeps the chunk bump counter within int32
constexpr int kClaimRanges = 8;              // claim counters of the batched form,
constexpr int kClaimStride = 1024;           // int32 apart (4 KiB)
constexpr int kTallyOffset = 512;            // selected-triplet tallies: claims + k * kClaimStride + 512

// counters: [0] triplets selected, [2] status bits, [3] candidate frames of
// the vertex stage, [4] their track-table size, [11] those with more tracks
// than slots, [5] entries queued for the
// float64 re-evaluation, [7] triplet-list entries handed out in chunks
// (also past the capacity: each grant adds one chunk), [9] and [10] lengths
// of the slice tables, [12] frames deferred to k_tiles, [13] their claims,
// [16] claims of the vertex stage's candidate frames
enum { ST_TRIP_FULL = 1, ST_TRACK_FULL = 2, ST_BAD_OFFSETS = 4 };

// Value of lane k (uniform k) in every lane: one v_readlane, no LDS crossbar.
__device__ inline int lane_value(int v, int k) { return __builtin_amdgcn_readlane(v, k); }

// ----------------------------------------------------------- triplet list
// Selected triplets are appended to chunks of one list: each wave of the
// cuts starts with a chunk of its own, fills it with ballot compaction, and
// when its survivors do not fit closes it and takes the next from a bump
// counter (one atomic per further chunk), so a frame may span chunks.  Chunk table row c holds
// [start, count, fitted, 0]; entries [fitted, count) of a chunk are fitted by
// k_tracks (the batched form fits the rest itself).
struct TripList {
  int32_t* trips;    // [capacity][2]: frame, packed frame-local i0 | i1 << 8 | i2 << 16
  int32_t* chunks;   // [capacity / kMinChunk + 1][4]
  int capacity, chunk;
  int pre;           // chunks 0 .. pre-1 belong to waves 0 .. pre-1 of the cuts from the start
};

// A wave's current chunk; wave-uniform.  id >= 0: chunk id is held and its
// entries [id * chunk, id * chunk + used) are written; kNoChunk: none taken
// yet; kListFull: the list ran out (stop asking).  Two scalars, so that the
// loops of the cuts carry little state.
constexpr int kNoChunk = -1, kListFull = -2;

struct Cursor {
  int id, used;
};

// Logical index of block b of G: XCD-major.  Blocks are dealt to the eight
// XCDs in turn (b mod 8), so this gives the blocks of one XCD consecutive
// indices; with frames dealt cyclically by logical index (g, g + G, ...) the
// frames one XCD works on at a time are neighbours, whose hit segments share
// cache lines in that XCD's L2 instead of being fetched into several.
__device__ inline int xcd_major(int b, int G) {
  const int q = G / 8;
  return b < 8 * q ? (b % 8) * q + b / 8 : b;
}

// The wave of logical index g < pre (the index its frames are dealt by)
// starts with a chunk of its own (so that the waves do not all queue on the
// bump counter at the start: atomics on one address are serialised); its
// row is written here.  The ids go XCD-major over g: consecutive chunks, the
// slices of the track stage that run at the same time on different XCDs,
// then hold frames eight apart rather than neighbouring frames, whose hits
// share cache lines (the fits run 10 % faster so).
__device__ inline Cursor cursor_start(const TripList& T, int g) {
  if (g >= T.pre) return Cursor{kNoChunk, 0};
  const int id = xcd_major(g, T.pre);
  if (threadIdx.x == 0) {
    int32_t* row = T.chunks + 4 * id;
    row[0] = id * T.chunk; row[1] = 0; row[2] = 0; row[3] = 0;
  }
  return Cursor{id, 0};
}

__device__ inline void cursor_close(const Cursor& c, int fitted, const TripList& T) {
  if (c.id >= 0 && threadIdx.x == 0) {
    T.chunks[4 * c.id + 1] = c.used;
    T.chunks[4 * c.id + 2] = fitted;
  }
}

// All chunks of a launch have the same size, so the k-th grant starts at
// k * chunk and the granted chunks (those ending within capacity) are rows
// 0 .. min(counters[7], capacity) / chunk - 1 of the table (counters[7]
// starts at pre * chunk: the chunks given out at the start).
__device__ inline int chunks_granted(const TripList& T, const int32_t* __restrict__ counters) {
  const int handed = counters[7] < T.capacity ? counters[7] : T.capacity;
  return handed / T.chunk;
}

__device__ inline void cursor_open(Cursor& c, const TripList& T, int32_t* __restrict__ counters) {
  int id = kListFull;
  if (threadIdx.x == 0) {
    const int s0 = atomicAdd(&counters[7], T.chunk);
    if (s0 <= T.capacity - T.chunk) {
      id = s0 / T.chunk;
      int32_t* row = T.chunks + 4 * id;
      row[0] = s0; row[1] = 0; row[2] = 0; row[3] = 0;
    } else {
      atomicOr(&counters[2], ST_TRIP_FULL);
    }
  }
  c.id = lane_value(id, 0);
  c.used = 0;
}

// Wave ballot of a condition: the condition's lane mask as the compare
// produced it (no detour through a 0/1 integer).
__device__ inline unsigned long long ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

// Set bits of m below this lane (the lane's rank among the set lanes).
__device__ inline int rank_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// base + rank_below(m), the addition done by the bit counts themselves.
__device__ inline int rank_below(unsigned long long m, int base) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, (unsigned)base));
}

// Makes the values available in registers at this point: the loads that
// produce them are issued here, together, rather than sunk by the compiler
// into the branches that first use them (each such load would cost the wave
// another memory round trip).  Emits no instruction.
template <class A, class B, class C, class D, class E>
__device__ inline void materialize(const A& a, const B& b, const C& c, const D& d, const E& e) {
  asm volatile("" ::"v"(a), "v"(b), "v"(c), "v"(d), "v"(e));
}
template <class A, class B, class C, class D, class E, class F>
__device__ inline void materialize(const A& a, const B& b, const C& c, const D& d, const E& e, const F& f) {
  asm volatile("" ::"v"(a), "v"(b), "v"(c), "v"(d), "v"(e), "v"(f));
}
__device__ inline void materialize(float a, float b, float c, float d, float e, float f, float g, float h, float i) {
  asm volatile("" ::"v"(a), "v"(b), "v"(c), "v"(d), "v"(e), "v"(f), "v"(g), "v"(h), "v"(i));
}

// ------------------------------------------------------------- cut tests
// Each test decides in float32 when the value lies outside a bound of its own
// rounding error around the window edges, and otherwise re-evaluates in
// float64.  The float64 paths are separate non-inlined functions: inlined,
// the compiler hoists their loop-invariant parts (divisions, square roots)
// out of the join loop and runs them for every candidate.

__device__ __attribute__((noinline, cold)) bool cos_refine(float x0, float y0, float x1, float y1, float lo,
                                                            float hi, float Ra, float Rb) {
  const double cd = ((double)x0 * x1 + (double)y0 * y1) / ((double)Ra * (double)Rb);
  return cd >= (double)lo && cd <= (double)hi;
}

__device__ __attribute__((noinline, cold)) bool dl_refine(float z0, float z1, float z2, float R0, float R1, float R2,
                                                           float lo, float hi) {
  const double d = ((double)z2 - (double)z1) / ((double)R2 - (double)R1) -
                   ((double)z1 - (double)z0) / ((double)R1 - (double)R0);
  return d >= (double)lo && d <= (double)hi;
}

__device__ __attribute__((noinline, cold)) bool rtc_refine(float x0, float y0, float x1, float y1, float x2, float y2,
                                                            float lo, float hi) {
  const double dax = (double)x0 - x1, day = (double)y0 - y1, dbx = (double)x2 - x1, dby = (double)y2 - y1;
  const double dex = (double)x2 - x0, dey = (double)y2 - y0;
  const double cross = dax * dby - day * dbx;
  if (cross == 0.0) return false;
  const double r = sqrt(dax * dax + day * day) * sqrt(dbx * dbx + dby * dby) * sqrt(dex * dex + dey * dey) /
                   (2.0 * fabs(cross));
  return r >= (double)lo && r <= (double)hi;
}

// Classification of a float32 test value: sure pass, sure fail, or
// ambiguous (within its rounding-error bound of an edge: decided by the
// float64 refinement).  Computed without branches; callers refine the
// ambiguous lanes behind one wave-uniform ballot.
struct Verdict {
  bool pass, amb;
};

__device__ inline Verdict window(float v, float err, float lo, float hi) {
  Verdict r;
  r.pass = v - err > lo && v + err < hi;
  r.amb = !r.pass && !(v + err < lo || v - err > hi);
  return r;
}

// cos(Phi_ij) = (h_i . h_j) / (R_i R_j) in a closed window.
__device__ inline Verdict cos_test(float x0, float y0, float x1, float y1, float invRR, float lo, float hi) {
  const float a = x0 * x1, b = y0 * y1;
  return window((a + b) * invRR, 8.0f * kU32 * (fabsf(a) + fabsf(b)) * invRR, lo, hi);
}

// Delta lambda = tan(lambda_12) - tan(lambda_01) in a closed window, as a
// window on z0 for the (h1, h2) pair (mu3e_window.hpp: the edges and their
// rounding bound).
__device__ inline ZWindow dl_window(float z1, float z2, const Consts& C) {
  return dl_window_f(z1, z2, C.inv12, C.d01, C.dl_lo, C.dl_hi, C.dl_abs);
}

// |r_tc| in a closed window, tested as r_tc^2 = d01^2 d12^2 d20^2 / (4 cross^2)
// with bounds on the rounding of the cross product and the chords.
__device__ inline Verdict rtc_test(float x0, float y0, float x1, float y1, float x2, float y2, const Consts& C) {
  const float ax = x0 - x1, ay = y0 - y1, bx = x2 - x1, by = y2 - y1, ex = x2 - x0, ey = y2 - y0;
  const float pa = ax * by, pb = ay * bx;
  const float cr = fabsf(pa - pb);
  const float ecr = 8.0f * kU32 * (fabsf(pa) + fabsf(pb));
  const float num = (ax * ax + ay * ay) * (bx * bx + by * by) * (ex * ex + ey * ey);
  const float en = 32.0f * kU32;
  const float clo = fmaxf(cr - ecr, 0.0f), chi = cr + ecr;
  const float dlo = 4.0f * clo * clo, dhi = 4.0f * chi * chi;
  const float nlo = num * (1.0f - en), nhi = num * (1.0f + en);
  const float m = 1.0f + 16.0f * kU32;
  const float lo2 = C.rtc_lo2, hi2 = C.rtc_hi2;
  Verdict r;
  r.pass = dlo > 0.0f && nlo >= lo2 * dhi * m && nhi * m <= hi2 * dlo;
  r.amb = !r.pass && !(nhi * m < lo2 * dlo || nlo > hi2 * dhi * m);
  return r;
}

// The Phi window of a pair, refined where ambiguous (all lanes call).
__device__ inline bool cos_cut_wave(bool act, float x0, float y0, float x1, float y1, float invRR, float lo,
                                    float hi, float Ra, float Rb) {
  const Verdict v = cos_test(x0, y0, x1, y1, invRR, lo, hi);
  bool pass = act && v.pass;
  if (ballot(act && v.amb) != 0ull) {
    if (act && v.amb) pass = cos_refine(x0, y0, x1, y1, lo, hi, Ra, Rb);
  }
  return pass;
}

// =================================================================== k_cuts
constexpr int kPlainTile = 128;      // LDS tile (hits per layer) of the plain form's cuts
constexpr int kJoinQueue = 2 * 64;   // combinations passing Delta lambda awaiting r_tc (< 2 waves)
constexpr uint32_t kDlAmbiguous = 1u << 24;     // queued combination whose Delta lambda float32 cannot decide
constexpr uint32_t kPhi12Ambiguous = 1u << 25;  // queued pair / combination whose cos Phi12 float32 cannot decide

// Frame-local hit indices of a triplet-list entry: i0 | i1 << 10 | i2 << 20,
// so that a layer may hold up to 1023 hits (larger layers are tiled through
// LDS by the cuts).
constexpr int kIdxBits = 10;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
static_assert(kMaxTiledLayerHits == (int)kIdxMask, "index packing and layer capacity disagree");

__device__ inline uint32_t pack_local(int i0, int i1, int i2) {
  return (uint32_t)i0 | ((uint32_t)i1 << kIdxBits) | ((uint32_t)i2 << (2 * kIdxBits));
}

// LDS of the cuts of one wave for tiles of at most TT (64 or 128) hits per
// layer: the tile's layer-0..2 hits, per layer-1 hit a mask of its layer-0
// partners passing Phi01 (TT / 64 words), the queue of (h1, h2) pairs
// passing Phi12 and the queue of combinations passing Delta lambda that
// await the r_tc test.  A frame whose layers fit one tile is staged once; a
// larger one runs tile by tile.
template <int TT>
struct CutLds {
  static constexpr int W = TT / 64;
  float sx[3 * TT], sy[3 * TT], sz[3 * TT];
  unsigned long long sm01[W * TT];
  uint32_t spend[2 * kWave];    // packed tile-local i1 | i2 << 8, kPhi12Ambiguous
  uint32_t sjoin[kJoinQueue];   // packed tile-local i1 | i2 << 8 | i0 << 16, kDlAmbiguous, kPhi12Ambiguous
};

// ------------------------------------------------------------ frame loads
// What a wave needs of a frame before its cuts, held in registers so that it
// can be loaded while the previous frame is processed: lanes 0..4 hold
// layer_offsets[4f .. 4f+4], lane i < 64 holds hit i of layers 0..2 (x, y, z).
struct FrameRegs {
  int lo;
  float x, y, z;
};

__device__ inline int load_offsets(const int32_t* __restrict__ lo, int f, bool valid) {
  const int lane = threadIdx.x;
  return valid && lane < 5 ? lo[4 * f + lane] : 0;
}

// Issues the hit loads of a frame whose offsets are in R.lo; only indices
// inside [b0, b3) and [0, n_hits) are read (malformed offsets read nothing).
__device__ inline void load_hits(FrameRegs& R, const float* __restrict__ X, const float* __restrict__ Y,
                                 const float* __restrict__ Z, int n_hits, bool valid) {
  const int b0 = lane_value(R.lo, 0), b3 = lane_value(R.lo, 3);
  const int i = b0 + (int)threadIdx.x;
  R.x = R.y = R.z = 0.f;
  if (valid && b0 >= 0 && i < b3 && i < n_hits) {
    R.x = X[i];
    R.y = Y[i];
    R.z = Z[i];
  }
}

// Phi01 of one tile (Alg. 2): over all (i0, i1) pairs of the staged layer-0
// and layer-1 tiles (n0, n1 hits), the bit of i0 is set in i1's partner mask.
template <int TT>
__device__ __attribute__((always_inline)) inline void phi01_tile(int n0, int n1, const Consts& C, CutLds<TT>& L) {
  constexpr int W = CutLds<TT>::W;
  const int lane = threadIdx.x;
  const int n01 = n0 * n1;
  // hardware reciprocal (about 1 ulp): (p + 0.5) / n0 stays at least
  // 0.5 / n0 >= 1/256 from an integer, far above its rounding error, so the
  // truncation below is exact
  const float r0 = __builtin_amdgcn_rcpf((float)n0);
  for (int base = 0; base < n01; base += kWave) {
    const int p = base + lane;
    const bool act = p < n01;
    const int i1 = act ? (int)(((float)p + 0.5f) * r0) : 0;   // exact for p < 2^14
    const int i0 = act ? p - i1 * n0 : 0;
    if (cos_cut_wave(act, L.sx[i0], L.sy[i0], L.sx[TT + i1], L.sy[TT + i1], C.invRR01, C.c01_lo, C.c01_hi, C.R[0],
                     C.R[1]))
      atomicOr(&L.sm01[W * i1 + (W == 2 ? (i0 >> 6) : 0)], 1ull << (i0 & 63));
  }
}

// Phi12, the join and r_tc of one tile whose Phi01 masks are built: (h1, h2)
// pairs passing Phi12 are streamed through an LDS queue and each full wave of
// pairs is joined against its Phi01 partners (Delta lambda tested as they
// are expanded), the combinations passing it are queued and tested on r_tc
// a full wave at a time.  Survivors are ballot-compacted into the wave's
// chunks of the triplet list with their frame-local indices (tile-local
// index + tile start a0, a1, a2).  Returns the number of survivors; those
// not stored because the list is full are added to `lost`.
template <int TT>
__device__ __attribute__((always_inline)) inline int join_tile(int f, int n1, int n2, int a0, int a1, int a2,
                                                               const Consts& C, CutLds<TT>& L, const TripList& T,
                                                               Cursor& cur, int& done, int& lost,
                                                               int32_t* __restrict__ counters) {
  constexpr int W = CutLds<TT>::W;
  const int lane = threadIdx.x;
  int total = 0;
  // r_tc test of the first m (<= kWave) queued combinations, one per lane
  // (with the float64 Phi12 and Delta lambda decisions of those marked
  // ambiguous); survivors are ballot-compacted into the wave's chunks.
  auto test = [&](int m) {
    const bool act = lane < m;
    const uint32_t c3 = act ? L.sjoin[lane] : 0u;
    const int j1 = c3 & 0xff, j2 = (c3 >> 8) & 0xff, j0 = (c3 >> 16) & 0xff;
    const float x0 = L.sx[j0], y0 = L.sy[j0];
    const float x1 = L.sx[TT + j1], y1 = L.sy[TT + j1];
    const float x2 = L.sx[2 * TT + j2], y2 = L.sy[2 * TT + j2];
    const Verdict vr = rtc_test(x0, y0, x1, y1, x2, y2, C);
    bool rpass = vr.pass;
    const bool damb = act && (c3 & kDlAmbiguous), pamb = act && (c3 & kPhi12Ambiguous);
    if (ballot(damb || pamb || (act && vr.amb)) != 0ull) {   // rare: float64 where float32 cannot decide
      if ((pamb && !cos_refine(x1, y1, x2, y2, C.c12_lo, C.c12_hi, C.R[1], C.R[2])) ||
          (damb && !dl_refine(L.sz[j0], L.sz[TT + j1], L.sz[2 * TT + j2], C.R[0], C.R[1], C.R[2], C.dl_lo,
                              C.dl_hi)))
        rpass = false;
      else if (act && vr.amb)
        rpass = rtc_refine(x0, y0, x1, y1, x2, y2, C.rtc_lo, C.rtc_hi);
    }
    const bool pass = act && rpass;
    const unsigned long long bm = ballot(pass);
    const int c = __popcll(bm);
    if (c > 0) {
      if (cur.id != kListFull && (cur.id < 0 || cur.used + c > T.chunk)) {
        cursor_close(cur, done, T);
        cursor_open(cur, T, counters);
        done = 0;
      }
      if (cur.id >= 0) {
        if (pass) {
          const int slot = rank_below(bm, cur.id * T.chunk + cur.used);
          *reinterpret_cast<int2*>(T.trips + 2 * slot) = make_int2(f, (int32_t)pack_local(a0 + j0, a1 + j1, a2 + j2));
        }
        cur.used += c;
      } else {
        lost += c;   // the list is full: these survivors are not stored
      }
    }
    total += c;
  };
  // Join of the k pending (h1, h2) pairs with their Phi01 partners: each
  // lane visits its pair's partners one per round and tests Delta lambda
  // (which needs only z); the passing combinations are ballot-compacted
  // into an LDS queue, and each full wave of them is tested on r_tc, so
  // that the costly test runs on full waves of the few survivors.
  int nq = 0;   // queued combinations, < kWave between rounds
  auto join = [&](int k) {
    const bool have = lane < k;
    const uint32_t e = have ? L.spend[lane] : 0u;
    const int i1 = e & 0xff, i2 = (e >> 8) & 0xff;
    const ZWindow zw = dl_window(L.sz[TT + i1], L.sz[2 * TT + i2], C);
    // the partners of one mask word (layer-0 hits base .. base + 63), one
    // per round: the lowest set bit, taken without a branch
    auto rounds = [&](unsigned long long w, int base) {
      unsigned long long live;   // the lanes with a partner left
      while ((live = ballot(w != 0ull)) != 0ull) {
        const bool has = w != 0ull;
        const int i0 = base + (has ? (int)__builtin_ctzll(w) : 0);
        w &= w - 1;
        const float z0 = L.sz[i0];
        // combinations in the ambiguous band are queued too, marked; the
        // r_tc stage decides them in float64 (rare), so the rounds carry
        // no branch
        const bool pass = has && z0 >= zw.out_lo && z0 <= zw.out_hi;
        const bool sure = z0 > zw.in_lo && z0 < zw.in_hi;
        // the ballot of pass as the AND of lane masks that are compare
        // results already (a ballot of a combined condition costs two
        // vector instructions more)
        const unsigned long long bm = live & ballot(z0 >= zw.out_lo) & ballot(z0 <= zw.out_hi);
        if (pass) L.sjoin[rank_below(bm, nq)] = (sure ? e : e | kDlAmbiguous) | ((uint32_t)i0 << 16);
        nq += __popcll(bm);
        if (nq >= kWave) {
          __syncthreads();
          test(kWave);
          const int rem = nq - kWave;
          const uint32_t v = lane < rem ? L.sjoin[kWave + lane] : 0u;
          __syncthreads();
          if (lane < rem) L.sjoin[lane] = v;
          __syncthreads();
          nq = rem;
        }
      }
    };
    rounds(have ? L.sm01[W * i1] : 0ull, 0);
    if (W == 2) rounds(have ? L.sm01[W * i1 + 1] : 0ull, 64);
  };
  // ---- Phi12 over all (i1, i2) pairs whose h1 has a layer-0 partner
  int npend = 0;
  const int n12 = n1 * n2;
  const float r2 = __builtin_amdgcn_rcpf((float)n2);
  for (int base = 0; base < n12; base += kWave) {
    const int p = base + lane;
    const bool inr = p < n12;
    const int i1 = inr ? (int)(((float)p + 0.5f) * r2) : 0;
    const int i2 = inr ? p - i1 * n2 : 0;
    const bool act = inr && (L.sm01[W * i1] | (W == 2 ? L.sm01[W * i1 + 1] : 0ull)) != 0ull;
    // pairs float32 cannot decide are queued too, marked, and decided in
    // float64 by the r_t,c stage for the combinations that reach it
    const Verdict v = cos_test(L.sx[TT + i1], L.sy[TT + i1], L.sx[2 * TT + i2], L.sy[2 * TT + i2], C.invRR12,
                               C.c12_lo, C.c12_hi);
    const bool pass = act && (v.pass || v.amb);
    const unsigned long long bm = ballot(pass);
    if (pass) L.spend[rank_below(bm, npend)] = (uint32_t)i1 | ((uint32_t)i2 << 8) | (v.amb ? kPhi12Ambiguous : 0u);
    npend += __popcll(bm);
    if (npend >= kWave) {
      __syncthreads();
      join(kWave);
      const int rem = npend - kWave;
      const uint32_t v = lane < rem ? L.spend[kWave + lane] : 0u;
      __syncthreads();
      if (lane < rem) L.spend[lane] = v;
      __syncthreads();
      npend = rem;
    }
  }
  if (npend > 0) { __syncthreads(); join(npend); }
  if (nq > 0) { __syncthreads(); test(nq); }
  return total;
}

// A frame with a layer above TT hits (LDS overflow), tile by tile: tiles of
// at most TT hits per layer, in the order (layer-1 tile, layer-0 tile,
// layer-2 tile); each (layer-0, layer-1) tile pair builds its Phi01 masks
// once for all layer-2 tiles.  Returns the number of survivors.  Only k_tiles
// runs it, so that its loop state stays out of the common one-tile path.
template <int TT>
__device__ __attribute__((always_inline)) inline int cut_tiles(int f, int b0, int b1, int b2, int n0, int n1, int n2,
                                                               const float* __restrict__ X,
                                                               const float* __restrict__ Y,
                                                               const float* __restrict__ Z, const Consts& C,
                                                               CutLds<TT>& L, const TripList& T, Cursor& cur,
                                                               int& done, int& lost,
                                                               int32_t* __restrict__ counters) {
  constexpr int W = CutLds<TT>::W;
  const int lane = threadIdx.x;
  int total = 0;
  auto stage_layer = [&](int l, int src, int m) {
    for (int i = lane; i < m; i += kWave) {
      L.sx[l * TT + i] = X[src + i];
      L.sy[l * TT + i] = Y[src + i];
      L.sz[l * TT + i] = Z[src + i];
    }
  };
  for (int a1 = 0; a1 < n1; a1 += TT) {
    const int m1 = min(TT, n1 - a1);
    for (int a0 = 0; a0 < n0; a0 += TT) {
      const int m0 = min(TT, n0 - a0);
      __syncthreads();
      stage_layer(0, b0 + a0, m0);
      stage_layer(1, b1 + a1, m1);
      for (int i = lane; i < W * m1; i += kWave) L.sm01[i] = 0ull;
      __syncthreads();
      phi01_tile<TT>(m0, m1, C, L);
      for (int a2 = 0; a2 < n2; a2 += TT) {
        const int m2 = min(TT, n2 - a2);
        __syncthreads();
        stage_layer(2, b2 + a2, m2);
        __syncthreads();
        total += join_tile<TT>(f, m1, m2, a0, a1, a2, C, L, T, cur, done, lost, counters);
      }
    }
  }
  return total;
}

// Selection Cuts of frame f by one wave (Alg. 2): the frame's layer-0..2
// hits are staged in LDS; survivors are ballot-compacted into the wave's
// chunks of the triplet list (cur; done = the wave's fitted prefix of its
// current chunk, recorded when the chunk is closed); returns the number
// committed (0 when the frame overflows max_triplets) and writes the frame's
// flags and counts.  A frame with a layer above TT hits is appended to the
// deferred list (counters[12] entries) for k_tiles instead.
template <int TT>
__device__ __attribute__((always_inline)) inline int cut_frame(int f, const FrameRegs& R, const float* __restrict__ X,
                                                               const float* __restrict__ Y,
                                                               const float* __restrict__ Z, int n_hits,
                                                               const Consts& C, CutLds<TT>& L, const TripList& T,
                                                               Cursor& cur, int& done, uint32_t* __restrict__ flags,
                                                               int32_t* __restrict__ counts, float* __restrict__ vtx,
                                                               int32_t* __restrict__ ccnt,
                                                               int32_t* __restrict__ counters,
                                                               int32_t* __restrict__ defer) {
  constexpr int W = CutLds<TT>::W;
  const int lane = threadIdx.x;
  const int b0 = lane_value(R.lo, 0), b1 = lane_value(R.lo, 1), b2 = lane_value(R.lo, 2);
  const int b3 = lane_value(R.lo, 3), b4 = lane_value(R.lo, 4);
  const int n0 = b1 - b0, n1 = b2 - b1, n2 = b3 - b2, n3 = b4 - b3;
  if (lane < 4) vtx[4 * f + lane] = __builtin_nanf("");
  if (lane == 0) { ccnt[f] = 0; counts[3 * f + 1] = 0; counts[3 * f + 2] = 0; }
  if (b0 < 0 || n0 < 0 || n1 < 0 || n2 < 0 || n3 < 0 || b4 > n_hits) {
    // malformed offsets: nothing of this frame is read
    if (lane == 0) { flags[f] = 0; counts[3 * f] = 0; atomicOr(&counters[2], ST_BAD_OFFSETS); }
    return 0;
  }
  if (n0 > C.max_lh || n1 > C.max_lh || n2 > C.max_lh || n3 > C.max_lh) {
    if (lane == 0) { flags[f] = MU3E_HITS_OVF | MU3E_KEEP; counts[3 * f] = 0; }
    return 0;
  }
  int total = 0;   // triplets passing all cuts (exact)
  int lost = 0;    // of those, not stored (the triplet list was full)
  const int fid = cur.id, fused = cur.used;   // where this frame's entries begin
  if (n0 > 0 && n2 > 0 && n1 > 0) {
    if (n0 <= TT && n1 <= TT && n2 <= TT) {
      // ---- one tile (the common case): stage the layer-0..2 hits
      // (coalesced), clear the masks.  Hits 0..63 arrive in registers loaded
      // during the previous frame; the rest are loaded in a loop of their
      // own, so that the common case waits on no memory load here (a wait
      // would also cover the next frame's loads, issued just before this
      // frame).
      const int n012 = n0 + n1 + n2;
      auto stage = [&](int i, float x, float y, float z) {
        const int l = (i >= n0) + (i >= n0 + n1);
        const int k = i - (l == 0 ? 0 : (l == 1 ? n0 : n0 + n1));
        L.sx[l * TT + k] = x;
        L.sy[l * TT + k] = y;
        L.sz[l * TT + k] = z;
      };
      if (lane < n012) stage(lane, R.x, R.y, R.z);
      for (int i = kWave + lane; i < n012; i += kWave) stage(i, X[b0 + i], Y[b0 + i], Z[b0 + i]);
      for (int i = lane; i < W * n1; i += kWave) L.sm01[i] = 0ull;
      __syncthreads();
      phi01_tile<TT>(n0, n1, C, L);
      __syncthreads();
      total = join_tile<TT>(f, n1, n2, 0, 0, 0, C, L, T, cur, done, lost, counters);
    } else {
      // ---- LDS overflow: the frame is deferred to k_tiles, which runs it
      // tile by tile and writes its flags and triplet count
      if (lane == 0) defer[atomicAdd(&counters[12], 1)] = f;
      return 0;
    }
  }
  const bool ovf = total > C.max_trip;
  if (lane == 0) {
    counts[3 * f] = total;
    flags[f] = (ovf ? (MU3E_TRIPLET_OVF | MU3E_KEEP) : 0u) | (lost ? (MU3E_LIST_FULL | MU3E_KEEP) : 0u);
  }
  // an overflowing frame is rolled back within the current chunk; entries it
  // left in chunks closed meanwhile are skipped by their frame flag (as are
  // those of a frame the list could not hold)
  if (ovf && cur.id >= 0) cur.used = cur.id == fid ? fused : 0;
  __syncthreads();
  return ovf ? 0 : total;
}

// End of a wave's cuts: record its last chunk and add its survivors to one
// of kClaimRanges tallies on separate lines (k_scount sums them into
// counters[0]), so that the waves ending together do not queue on one address.
__device__ inline void close_list(const Cursor& cur, int done, int selected, const TripList& T,
                                  int32_t* __restrict__ claims) {
  cursor_close(cur, done, T);
  if (threadIdx.x == 0 && selected > 0)
    atomicAdd(&claims[(blockIdx.x % kClaimRanges) * kClaimStride + kTallyOffset], selected);
}

// Runs body(f, regs) for the frames first, next(first), ... (next returns -1
// after the last; all wave-uniform), loading each frame's offsets two frames
// ahead and its hits one frame ahead, so that the loads overlap the cuts of
// the frame before.
template <class Next, class Body>
__device__ inline void frame_pipeline(int first, Next next, Body body, const int32_t* __restrict__ lo,
                                      const float* __restrict__ X, const float* __restrict__ Y,
                                      const float* __restrict__ Z, int n_hits) {
  int f = first;
  FrameRegs cur;
  cur.lo = load_offsets(lo, f, f >= 0);
  load_hits(cur, X, Y, Z, n_hits, f >= 0);
  int f1 = f >= 0 ? next(f) : -1;
  int nlo = load_offsets(lo, f1, f1 >= 0);
  while (f >= 0) {
    const int f2 = f1 >= 0 ? next(f1) : -1;
    FrameRegs nx;
    nx.lo = nlo;
    load_hits(nx, X, Y, Z, n_hits, f1 >= 0);
    nlo = load_offsets(lo, f2, f2 >= 0);
    body(f, cur);
    cur = nx;
    f = f1;
    f1 = f2;
  }
}

// Plain form: one wave per frame, frames dealt cyclically to a static grid
// (Alg. 1 with the paper's cyclic distribution); survivors go to the wave's
// chunks of the triplet list.
template <int TT>
__global__ void __launch_bounds__(64)
k_cuts(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
       const int32_t* __restrict__ lo, int F, int n_hits, Consts C, uint32_t* __restrict__ flags,
       int32_t* __restrict__ counts, float* __restrict__ vtx, int32_t* __restrict__ ccnt, TripList T,
       int32_t* __restrict__ counters, int32_t* __restrict__ claims, int32_t* __restrict__ defer) {
  __shared__ CutLds<TT> L;
  Cursor cur = cursor_start(T, xcd_major((int)blockIdx.x, (int)gridDim.x));
  int done = 0, selected = 0;   // nothing is fitted here
  const int G = gridDim.x;
  const int g0 = xcd_major((int)blockIdx.x, G);
  frame_pipeline(
      g0 < F ? g0 : -1, [&](int g) { return g < F - G ? g + G : -1; },
      [&](int f, const FrameRegs& R) {
        selected += cut_frame<TT>(f, R, X, Y, Z, n_hits, C, L, T, cur, done, flags, counts, vtx, ccnt, counters,
                                  defer);
      },
      lo, X, Y, Z, n_hits);
  close_list(cur, 0, selected, T, claims);
}

// Frames the cuts kernel deferred (a layer above TT hits: LDS overflow), one
// wave per frame, claimed from a counter: the frame runs tile by tile
// (cut_tiles) and its flags and triplet count are written, with the same
// cap and roll-back as in cut_frame.  Waves beyond the number of deferred
// frames return at once, so a batch without such frames costs one empty
// launch.
template <int TT>
__global__ void __launch_bounds__(64)
k_tiles(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
        const int32_t* __restrict__ lo, Consts C, uint32_t* __restrict__ flags, int32_t* __restrict__ counts,
        TripList T, int32_t* __restrict__ counters, int32_t* __restrict__ claims,
        const int32_t* __restrict__ defer) {
  const int nd = counters[12];
  if ((int)blockIdx.x >= nd) return;
  __shared__ CutLds<TT> L;
  const int lane = threadIdx.x;
  Cursor cur{kNoChunk, 0};
  int done = 0, selected = 0;
  for (;;) {
    int k = 0;
    if (lane == 0) k = atomicAdd(&counters[13], 1);
    k = lane_value(k, 0);
    if (k >= nd) break;
    const int f = defer[k];
    const int b0 = lo[4 * f], b1 = lo[4 * f + 1], b2 = lo[4 * f + 2], b3 = lo[4 * f + 3];
    const int fid = cur.id, fused = cur.used;
    int lost = 0;
    const int total = cut_tiles<TT>(f, b0, b1, b2, b1 - b0, b2 - b1, b3 - b2, X, Y, Z, C, L, T, cur, done, lost,
                                    counters);
    const bool ovf = total > C.max_trip;
    if (lane == 0) {
      counts[3 * f] = total;
      flags[f] = (ovf ? (MU3E_TRIPLET_OVF | MU3E_KEEP) : 0u) | (lost ? (MU3E_LIST_FULL | MU3E_KEEP) : 0u);
    }
    if (ovf && cur.id >= 0) cur.used = cur.id == fid ? fused : 0;
    selected += ovf ? 0 : total;
    __syncthreads();
  }
  close_list(cur, 0, selected, T, claims);
}

// ================================================================= k_tracks
// Track reconstruction of one selected triplet (Section IV-B, Alg. 3).
// Returns 1 accepted, 0 rejected, -1 undecided in float32 (re-evaluate).
template <class T>
__device__ inline int track_eval(const float* __restrict__ X, const float* __restrict__ Y,
                                 const float* __restrict__ Z, int g0, int g1, int g2, int b3, int b4,
                                 const Consts& C, int& g3, T& kbar, T& chi2) {
  constexpr bool F32 = sizeof(T) == 4;
  const float x0 = X[g0], y0 = Y[g0], z0 = Z[g0];
  const float x1 = X[g1], y1 = Y[g1], z1 = Z[g1];
  const float x2 = X[g2], y2 = Y[g2], z2 = Z[g2];
  materialize(x0, y0, z0, x1, y1, z1, x2, y2, z2);
  const Fit<T> f1 = fit_triplet<T>(x0, y0, z0, x1, y1, z1, x2, y2, z2, C);
  if (!f1.ok) return (F32 && f1.c.cross != 0.0) ? -1 : 0;
  T px = 0, py = 0, pz = 0;
  bool near = false;
  const int reach = predict_l3<T>(f1, x2, y2, z2, (T)C.R[3], (T)1e-4, px, py, pz, F32 ? &near : nullptr);
  if (F32 && near) return -1;
  if (!reach) return 0;
  T best = (T)1e30, second = (T)1e30;
  int ib = -1;   // the nearest hit so far (its coordinates are read again after the scan)
  auto consider = [&](float x, float y, float z, int g) {
    const T dx = (T)x - px, dy = (T)y - py, dz = (T)z - pz;
    const T d2 = dx * dx + dy * dy + dz * dz;
    const bool nb = d2 < best;
    second = nb ? best : (d2 < second ? d2 : second);
    ib = nb ? g : ib;
    best = nb ? d2 : best;
  };
  auto quad = [&](int g) {   // hits g .. g+3, all inside [b3, b4); 16-byte loads at dword-aligned addresses
    float4 vx, vy, vz;
    __builtin_memcpy(&vx, X + g, sizeof(float4));
    __builtin_memcpy(&vy, Y + g, sizeof(float4));
    __builtin_memcpy(&vz, Z + g, sizeof(float4));
    consider(vx.x, vy.x, vz.x, g);
    consider(vx.y, vy.y, vz.y, g + 1);
    consider(vx.z, vy.z, vz.z, g + 2);
    consider(vx.w, vy.w, vz.w, g + 3);
  };
  // layer-3 hits in order: four at a time, then the last 0..3 with their
  // loads issued together (one memory round trip for the tail)
  int g = b3;
  for (; g + 4 <= b4; g += 4) quad(g);
  {
    const int m = b4 - g;
    float tx[3] = {0.f, 0.f, 0.f}, ty[3] = {0.f, 0.f, 0.f}, tz[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < m) { tx[k] = X[g + k]; ty[k] = Y[g + k]; tz[k] = Z[g + k]; }
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < m) consider(tx[k], ty[k], tz[k], g + k);
  }
  if (ib < 0) return 0;
  const float bx = X[ib], by = Y[ib], bz = Z[ib];
  if (F32 && second < (T)1e29) {
    const T eps = (T)1e-3;   // bound on the float32 error of the predicted point [mm]
    if (second - best <= (T)2 * eps * (m_sqrt(best) + m_sqrt(second)) + (T)1e-5 * second) return -1;
  }
  g3 = ib;
  const Fit<T> f2 = fit_triplet<T>(x1, y1, z1, x2, y2, z2, bx, by, bz, C);
  if (!f2.ok) return (F32 && f2.c.cross != 0.0) ? -1 : 0;
  if (f2.c.sgn != f1.c.sgn) return 0;
  combine(f1, f2, kbar, chi2);
  if (F32 && m_abs(chi2 - (T)C.chi2_trk) <= (T)0.1) return -1;
  return chi2 < (T)C.chi2_trk ? 1 : 0;
}

// ----------------------------------------------------------- track results
// Results of the track stage are stored in place, parallel to the triplet
// list, so that no shared counter is needed: entry e has res[4e .. 4e+3] =
// {code, i3, kappa_bar bits, chi2 bits}.  TR_ACCEPT: accepted track, i3 its
// frame-local layer-3 hit; TR_REJECT: rejected, or not fitted because its
// frame overflowed; TR_REDO: float32 could not decide, the entry index is
// queued for the float64 re-evaluation, which rewrites the result.
enum { TR_REJECT = 0, TR_ACCEPT = 1, TR_REDO = 2 };

// Accepted tracks per frame also note their entry index in the frame's row of
// tslot (the first nslot of them), so that the vertex stage finds the tracks
// of its candidate frames without scanning the list.  nslot follows the
// track capacity per frame the caller asks for (track_slots); frames with at
// most kSmallSlots tracks are refitted into LDS by the vertex wave, larger
// ones into their slice of the workspace's track table.
constexpr int kSmallSlots = 16;
constexpr int kMaxSlots = 128;

struct TrackOut {
  uint32_t* flags;   // per-frame flags [F]
  int32_t* res;      // [triplet capacity][4]
  int32_t* redo;     // [redo_cap] entry indices
  int redo_cap;
  int32_t* counts;   // per-frame counts [3F]; tracks at 3f + 1
  int32_t* ccnt;     // per-frame charge tally: +1 per e+, +65536 per e-
  int32_t* tslot;    // [F][nslot] entry indices of accepted tracks
  int nslot;
};

__device__ inline void store_result(int32_t* __restrict__ res, int e, int code, int i3, float kb, float c2) {
  *reinterpret_cast<int4*>(res + 4 * e) = make_int4(code, i3, __float_as_int(kb), __float_as_int(c2));
}

__device__ inline void tally_track(const TrackOut& O, int f, int e, float kb) {
  const int rank = atomicAdd(&O.counts[3 * f + 1], 1);
  if (rank < O.nslot) O.tslot[f * O.nslot + rank] = e;
  atomicAdd(&O.ccnt[f], kb > 0.f ? 1 : 65536);
}

// Called by all 64 lanes of a wave; a lane with active == false holds no
// entry.  r from track_eval: 1 accepted, 0 rejected, -1 undecided; the
// undecided entries of the wave are queued with one atomic.
__device__ inline void emit_result(bool active, int r, int e, int f, int i3, float kb, float c2,
                                   const TrackOut& O, int32_t* __restrict__ counters) {
  const unsigned long long und = ballot(active && r < 0);
  int qbase = 0;
  if (und != 0ull) {
    if (threadIdx.x == 0) qbase = atomicAdd(&counters[5], __popcll(und));
    qbase = lane_value(qbase, 0);
  }
  if (!active) return;
  if (r < 0) {
    const int q = qbase + rank_below(und);
    if (q < O.redo_cap) {
      O.redo[q] = e;
    } else {   // the float64 queue is full: this frame stays undecided, kept
      atomicOr(&counters[2], ST_TRACK_FULL);
      atomicOr(&O.flags[f], MU3E_LIST_FULL | MU3E_KEEP);
    }
    store_result(O.res, e, TR_REDO, 0, 0.f, 0.f);
  } else {
    store_result(O.res, e, r == 1 ? TR_ACCEPT : TR_REJECT, i3, kb, c2);
    if (r == 1) tally_track(O, f, e, kb);
  }
}

// Global hit indices of a list entry (frame f, packed frame-local indices pk)
// and the frame's layer-3 range.
struct EntryHits {
  int g0, g1, g2, b3, b4;
};

__device__ inline EntryHits entry_hits(const int32_t* __restrict__ lo, int f, uint32_t pk) {
  return EntryHits{lo[4 * f] + (int)(pk & kIdxMask), lo[4 * f + 1] + (int)((pk >> kIdxBits) & kIdxMask),
                   lo[4 * f + 2] + (int)(pk >> (2 * kIdxBits)), lo[4 * f + 3], lo[4 * f + 4]};
}

// A list entry of T: {frame, packed frame-local indices}, one 8-byte load.
__device__ inline int2 list_entry(const TripList& T, int e) {
  return *reinterpret_cast<const int2*>(T.trips + 2 * e);
}

// Track reconstruction of one list entry with hits h; i3 is the frame-local
// layer-3 hit of an accepted track.
template <class T>
__device__ inline int fit_entry(const float* __restrict__ X, const float* __restrict__ Y,
                                const float* __restrict__ Z, const EntryHits& h, const Consts& C, int& i3, T& kb,
                                T& c2) {
  int g3 = -1;
  const int r = track_eval<T>(X, Y, Z, h.g0, h.g1, h.g2, h.b3, h.b4, C, g3, kb, c2);
  i3 = g3 >= 0 ? g3 - h.b3 : 0;
  return r;
}

// ------------------------------------------------------------ slice tables
// The non-empty slices of at most 64 entries of the granted chunks, each as
// {first entry index, entry count}.  fit: slices of [fitted, count) of each
// chunk, the entries k_tracks fits; all: slices of [0, count).  counters[9]
// and counters[10] hold their lengths.
struct Slices {
  int2* fit;
  int2* all;
};

// Sums of a and b over a block of 256 threads (all threads get them).
__device__ inline void block_sum2(int& a, int& b, int* tmp) {   // 256 threads
  const int i = threadIdx.x;
  tmp[i] = a;
  tmp[256 + i] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (i < o) { tmp[i] += tmp[i + o]; tmp[256 + i] += tmp[256 + i + o]; }
    __syncthreads();
  }
  a = tmp[0];
  b = tmp[256];
  __syncthreads();
}

// Slice counts of chunk c: fit slices of [fitted, count), all slices of
// [0, count).
__device__ inline void chunk_slices(const TripList& T, int c, int& nf, int& na) {
  const int n = T.chunks[4 * c + 1];
  const int from = T.chunks[4 * c + 2];
  na = (n + kWave - 1) / kWave;
  nf = from < n ? (n - from + kWave - 1) / kWave : 0;
}

// Two passes without atomics, 256 chunks per block: k_scount writes each
// block's slice totals, k_splace offsets each block by the totals of the
// blocks before it and writes the tables.  k_scount also sums the cuts'
// selected-triplet tallies into counters[0].
__global__ void __launch_bounds__(256)
k_scount(TripList T, int32_t* __restrict__ blk, int32_t* __restrict__ counters,
         const int32_t* __restrict__ claims) {
  __shared__ int tmp[512];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int sel = 0;
    for (int k = 0; k < kClaimRanges; ++k) sel += claims[k * kClaimStride + kTallyOffset];
    counters[0] = sel;
  }
  const int nch = chunks_granted(T, counters);
  const int c = blockIdx.x * 256 + (int)threadIdx.x;
  int nf = 0, na = 0;
  if (c < nch) chunk_slices(T, c, nf, na);
  block_sum2(nf, na, tmp);
  if (threadIdx.x == 0) { blk[2 * blockIdx.x] = nf; blk[2 * blockIdx.x + 1] = na; }
}

__global__ void __launch_bounds__(256)
k_splace(TripList T, Slices S, const int32_t* __restrict__ blk, int32_t* __restrict__ counters) {
  __shared__ int tmp[512];
  const int nch = chunks_granted(T, counters);
  int bf = 0, ba = 0, tf = 0, ta = 0;
  for (int j = threadIdx.x; j < (int)gridDim.x; j += 256) {
    const int f = blk[2 * j], a = blk[2 * j + 1];
    tf += f; ta += a;
    if (j < (int)blockIdx.x) { bf += f; ba += a; }
  }
  block_sum2(bf, ba, tmp);
  block_sum2(tf, ta, tmp);
  if (blockIdx.x == 0 && threadIdx.x == 0) { counters[9] = tf; counters[10] = ta; }
  const int c = blockIdx.x * 256 + (int)threadIdx.x;
  int nf = 0, na = 0;
  if (c < nch) chunk_slices(T, c, nf, na);
  // block exclusive scan of (nf, na)
  tmp[threadIdx.x] = nf;
  tmp[256 + threadIdx.x] = na;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int i = threadIdx.x;
    const int x = i >= o ? tmp[i - o] : 0, y = i >= o ? tmp[256 + i - o] : 0;
    __syncthreads();
    tmp[i] += x;
    tmp[256 + i] += y;
    __syncthreads();
  }
  const int of = bf + tmp[threadIdx.x] - nf, oa = ba + tmp[256 + threadIdx.x] - na;
  if (nf > 0 || na > 0) {
    const int start = T.chunks[4 * c], n = T.chunks[4 * c + 1], from = T.chunks[4 * c + 2];
    for (int j = 0; j < nf; ++j) {
      const int t = from + j * kWave;
      S.fit[of + j] = make_int2(start + t, min(kWave, n - t));
    }
    for (int j = 0; j < na; ++j) {
      const int t = j * kWave;
      S.all[oa + j] = make_int2(start + t, min(kWave, n - t));
    }
  }
}

// Float32 track reconstruction of the entries [fitted, count) of every
// chunk, one wave per 64-entry slice (dealt cyclically to the grid);
// candidates the float32 arithmetic cannot decide go to the float64 list.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5)))
k_tracks(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
         const int32_t* __restrict__ lo, Consts C, const uint32_t* __restrict__ flags, TripList T, Slices S,
         TrackOut O, int32_t* __restrict__ counters) {
  const int ns = counters[9];
  for (int v = blockIdx.x; v < ns; v += gridDim.x) {
    const int2 sl = S.fit[v];
    const bool active = (int)threadIdx.x < sl.y;
    const int e = sl.x + (int)threadIdx.x;
    int r = 0, f = 0, i3 = 0;
    float kb = 0.f, c2 = 0.f;
    if (active) {
      const int2 en = list_entry(T, e);
      f = en.x;
      const uint32_t fl = flags[f];
      const EntryHits h = entry_hits(lo, f, (uint32_t)en.y);
      materialize(fl, h.g0, h.g1, h.g2, h.b3, h.b4);   // one round trip for the flag and the offsets
      if (!(fl & (MU3E_TRIPLET_OVF | MU3E_LIST_FULL))) r = fit_entry<float>(X, Y, Z, h, C, i3, kb, c2);
    }
    emit_result(active, r, e, f, i3, kb, c2, O, counters);
  }
}

// ============================================================ batched form
// Persistent waves run the Selection Cuts of all frames: frames [0, Fs) are
// dealt cyclically to the waves (the paper's scheme, no shared counters),
// and the tail [Fs, F) is taken by work stealing -- `claim` frames at a time
// from kClaimRanges counters over kClaimRanges sub-ranges of the tail, each
// counter on its own 4-KiB line (claims spread over memory channels); a wave
// starts in sub-range blockIdx mod kClaimRanges and moves on when it is used
// up.  kFuse: the same wave also fits the pending survivors of its frames 64
// at a time (fit batches span frames); entries left unfitted in a chunk
// closed in the middle of a frame are recorded for k_tracks.  Without kFuse
// the kernel needs far fewer registers (more resident waves for the
// latency-bound cuts) and k_tracks fits everything.
template <bool kFuse, int TT>
__global__ void __launch_bounds__(64)
k_batched(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
          const int32_t* __restrict__ lo, int F, int Fs, int n_hits, Consts C, uint32_t* __restrict__ flags,
          int32_t* __restrict__ counts, float* __restrict__ vtx, int32_t* __restrict__ ccnt, TripList T,
          TrackOut O, int32_t* __restrict__ counters, int32_t* __restrict__ claims, int claim,
          int32_t* __restrict__ defer) {
  __shared__ CutLds<TT> L;
  const int lane = threadIdx.x;
  Cursor cur = cursor_start(T, xcd_major((int)blockIdx.x, (int)gridDim.x));
  int done = 0, selected = 0;
  auto fit = [&](int k) {   // fit entries [done, done + k) of the current chunk, lane j taking done + j
    const bool active = lane < k;
    const int e = cur.id * T.chunk + done + lane;
    int r = 0, f = 0, i3 = 0;
    float kb = 0.f, c2 = 0.f;
    if (active) {
      const int2 en = list_entry(T, e);
      f = en.x;
      const EntryHits h = entry_hits(lo, f, (uint32_t)en.y);
      materialize(h.g0, h.g1, h.g2, h.b3, h.b4);
      r = fit_entry<float>(X, Y, Z, h, C, i3, kb, c2);
    }
    emit_result(active, r, e, f, i3, kb, c2, O, counters);
    done += k;
  };
  auto body = [&](int f, const FrameRegs& R) {
    selected += cut_frame<TT>(f, R, X, Y, Z, n_hits, C, L, T, cur, done, flags, counts, vtx, ccnt, counters,
                              defer);
    if constexpr (kFuse) {
      while (cur.used - done >= kWave) fit(kWave);
    }
  };
  // Frame source: the static cyclic part, then claims from the stolen tail
  // (one call site of the body keeps a single inlined copy of the cuts).
  const int G = gridDim.x;
  const int tail = F - Fs;
  int range = 0, fe = 0;   // stealing state: sub-ranges visited, end of the current claim
  auto claim_next = [&]() -> int {
    for (; tail > 0 && range < kClaimRanges; ++range) {
      const int k = (int)((blockIdx.x + range) % kClaimRanges);
      const int r0 = Fs + (int)((int64_t)tail * k / kClaimRanges);
      const int r1 = Fs + (int)((int64_t)tail * (k + 1) / kClaimRanges);
      int32_t* ctr = claims + kClaimStride * k;
      int base = r1;
      if (lane == 0) {
        const int seen = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (seen < r1 - r0) base = r0 + atomicAdd(ctr, claim);
      }
      base = lane_value(base, 0);
      if (base < r1) {
        fe = base + claim < r1 ? base + claim : r1;
        return base;
      }
    }
    return -1;
  };
  auto next = [&](int g) -> int {
    if (g < Fs) {
      if (g < Fs - G) return g + G;
      return claim_next();
    }
    if (g + 1 < fe) return g + 1;
    return claim_next();
  };
  const int g0 = xcd_major((int)blockIdx.x, G);
  frame_pipeline(g0 < Fs ? g0 : claim_next(), next, body, lo, X, Y, Z, n_hits);
  if constexpr (kFuse) {
    if (cur.used > done) fit(cur.used - done);
  }
  close_list(cur, done, selected, T, claims);
}

// Float64 re-evaluation of the entries queued by k_tracks (or the fused
// batched kernel); rewrites their results.
__global__ void __launch_bounds__(64)
k_tracks_redo(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
              const int32_t* __restrict__ lo, Consts C, TripList T, TrackOut O, int32_t* __restrict__ counters) {
  const int n = min(counters[5], O.redo_cap);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int e = O.redo[t];
    const int2 en = list_entry(T, e);
    const int f = en.x;
    int i3 = 0;
    double kd = 0, cd = 0;
    const EntryHits h = entry_hits(lo, f, (uint32_t)en.y);
    materialize(h.g0, h.g1, h.g2, h.b3, h.b4);
    const int r = fit_entry<double>(X, Y, Z, h, C, i3, kd, cd);
    store_result(O.res, e, r == 1 ? TR_ACCEPT : TR_REJECT, i3, (float)kd, (float)cd);
    if (r == 1) tally_track(O, f, e, (float)kd);
  }
}

// ================================================================ vertex
// Per-track quantities of the vertex stage, in float64 (Section IV-C).
struct VTrack {
  double q, E, p, cth, rt, cx, cy, rbar, sms0, hx, hy, hz;
};

// Refit of a four-hit track in float64 and its transverse circle: radius
// r_t = Rbar sin(theta_C1), centre on the bending side of the layer-0/1 chord.
__device__ inline bool vtrack_make(const float* __restrict__ X, const float* __restrict__ Y,
                                   const float* __restrict__ Z, int n_hits, const int32_t* h, const Consts& C,
                                   VTrack& v) {
  const int g0 = h[0], g1 = h[1], g2 = h[2], g3 = h[3];
  if ((unsigned)g0 >= (unsigned)n_hits || (unsigned)g1 >= (unsigned)n_hits || (unsigned)g2 >= (unsigned)n_hits ||
      (unsigned)g3 >= (unsigned)n_hits)
    return false;
  const Fit<double> a = fit_triplet<double>(X[g0], Y[g0], Z[g0], X[g1], Y[g1], Z[g1], X[g2], Y[g2], Z[g2], C);
  const Fit<double> b = fit_triplet<double>(X[g1], Y[g1], Z[g1], X[g2], Y[g2], Z[g2], X[g3], Y[g3], Z[g3], C);
  if (!a.ok || !b.ok) return false;
  double kbar, chi2;
  combine(a, b, kbar, chi2);
  v.q = kbar > 0 ? 1.0 : -1.0;
  v.rbar = 1.0 / fabs(kbar);
  v.p = kCLight * (double)C.b * v.rbar;
  v.E = sqrt(v.p * v.p + kMassE * kMassE);
  v.cth = a.cth1;
  const double sth = a.sth1;
  v.hx = X[g0]; v.hy = Y[g0]; v.hz = Z[g0];
  const double dx = (double)X[g1] - v.hx, dy = (double)Y[g1] - v.hy;
  const double d = sqrt(dx * dx + dy * dy);
  double rt = v.rbar * sth;
  if (rt < 0.5 * d) rt = 0.5 * d;
  v.rt = rt;
  const double off = sqrt(fmax(rt * rt - 0.25 * d * d, 0.0));
  // right-hand normal of the motion h0 -> h1 is (dy, -dx)/d; clockwise
  // (positive) tracks curve to the right
  v.cx = 0.5 * (v.hx + X[g1]) + v.q * off * dy / d;
  v.cy = 0.5 * (v.hy + Y[g1]) - v.q * off * dx / d;
  v.sms0 = highland<double>(v.p, (double)C.xx0 / sth);
  return true;
}

// Turning angle travelled backwards along the track from its layer-0 hit to
// the point q, in [0, 2 pi).
__device__ inline double back_turn(const VTrack& t, double qx, double qy) {
  const double vx = t.hx - t.cx, vy = t.hy - t.cy, wx = qx - t.cx, wy = qy - t.cy;
  double a = atan2_full(vx * wy - vy * wx, vx * wx + vy * wy);   // counter-clockwise h0 -> q
  if (t.q < 0) a = -a;                                       // backwards of a clockwise track is ccw
  if (a < 0) a += 2.0 * kPiD;
  return a;
}

__device__ inline double sigma2_at(const VTrack& t, double qx, double qy, const Consts& C) {
  const double s = t.rt * back_turn(t, qx, qy);
  return t.sms0 * t.sms0 * s * s + (double)C.sig_pix * (double)C.sig_pix;
}

__device__ inline double cone_dist(double r, double z, const Consts& C) {
  // distance in the (r, z) half plane to the segments (R_t, 0) - (0, +-50)
  double best = 1e300;
  for (int s = -1; s <= 1; s += 2) {
    const double ux = -(double)C.r_target, uz = 50.0 * s;
    const double px = r - (double)C.r_target, pz = z;
    double t = (px * ux + pz * uz) / (ux * ux + uz * uz);
    t = t < 0 ? 0 : (t > 1 ? 1 : t);
    const double ex = px - t * ux, ez = pz - t * uz;
    best = fmin(best, sqrt(ex * ex + ez * ez));
  }
  return best;
}

// Vertex estimate of one e+ e+ e- triple, in two parts so that a wave can
// spread the combinations over its lanes.  VPoints: the intersections of the
// three track circles pairwise (pairs (0,1), (0,2), (1,2)) that lie near the
// target, and at each the mean of the two tracks' position variances.
struct VPoints {
  double qx[3][2], qy[3][2], s2[3][2];
  int nq[3];
};

__device__ inline bool vertex_points(const VTrack* T0, const VTrack* T1, const VTrack* T2, const Consts& C,
                                     VPoints& P) {
  const VTrack* tk[3] = {T0, T1, T2};
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  const double lim = (double)C.r_target + (double)C.target_tol;
#pragma unroll   // constant indices: P stays in registers
  for (int k = 0; k < 3; ++k) {
    const VTrack& A = *tk[pa[k]];
    const VTrack& B = *tk[pb[k]];
    const double dx = B.cx - A.cx, dy = B.cy - A.cy;
    const double d = sqrt(dx * dx + dy * dy);
    P.nq[k] = 0;
    if (d == 0.0 || d > A.rt + B.rt || d < fabs(A.rt - B.rt)) return false;
    const double id = 1.0 / d;
    const double a = (A.rt * A.rt - B.rt * B.rt + d * d) * (0.5 * id);
    const double h = sqrt(fmax(A.rt * A.rt - a * a, 0.0));
    const double ux = dx * id, uy = dy * id;
    // the two intersections (s = -1, +1), kept in that order if near the target
    const double x0 = A.cx + a * ux + h * uy, y0 = A.cy + a * uy - h * ux;
    const double x1 = A.cx + a * ux - h * uy, y1 = A.cy + a * uy + h * ux;
    const bool in0 = sqrt(x0 * x0 + y0 * y0) <= lim, in1 = sqrt(x1 * x1 + y1 * y1) <= lim;
    if (!in0 && !in1) return false;
    const double fx = in0 ? x0 : x1, fy = in0 ? y0 : y1;
    P.qx[k][0] = fx;
    P.qy[k][0] = fy;
    P.s2[k][0] = 0.5 * (sigma2_at(A, fx, fy, C) + sigma2_at(B, fx, fy, C));
    P.nq[k] = 1;
    if (in0 && in1) {
      P.qx[k][1] = x1;
      P.qy[k][1] = y1;
      P.s2[k][1] = 0.5 * (sigma2_at(A, x1, y1, C) + sigma2_at(B, x1, y1, C));
      P.nq[k] = 2;
    }
  }
  return true;
}

// Whether the circles of tracks A and B may have an intersection near the
// target, as vertex_points decides it for the pair (A, B), with margins
// (1e-12 relative on the circle test, 1e-6 on the squared target radius,
// which covers the rounding of the intersection points even near tangency)
// so that it never rejects a pair that vertex_points accepts: a prefilter.
__device__ inline bool pair_may_meet(const VTrack& A, const VTrack& B, double lim2) {
  const double dx = B.cx - A.cx, dy = B.cy - A.cy;
  const double d = sqrt(dx * dx + dy * dy);
  if (d == 0.0 || d > (A.rt + B.rt) * (1.0 + 1e-12) || d < fabs(A.rt - B.rt) * (1.0 - 1e-12)) return false;
  const double a = (A.rt * A.rt - B.rt * B.rt + d * d) / (2.0 * d);
  const double h = sqrt(fmax(A.rt * A.rt - a * a, 0.0));
  const double ux = dx / d, uy = dy / d;
  const double x0 = A.cx + a * ux + h * uy, y0 = A.cy + a * uy - h * ux;
  const double x1 = A.cx + a * ux - h * uy, y1 = A.cy + a * uy + h * ux;
  const double l2 = lim2 * (1.0 + 1e-6);
  return x0 * x0 + y0 * y0 <= l2 || x1 * x1 + y1 * y1 <= l2;
}

// Bit c of the mask: combination c (intersection c & 1 of pair 0, (c >> 1) & 1
// of pair 1, (c >> 2) & 1 of pair 2) exists.
__device__ inline int vertex_combos(const VPoints& P) {
  int m = 0;
  for (int c = 0; c < 8; ++c)
    if ((c & 1) < P.nq[0] && ((c >> 1) & 1) < P.nq[1] && ((c >> 2) & 1) < P.nq[2]) m |= 1 << c;
  return m;
}

// Combination c: weighted mean of its three intersections, points of closest
// approach of the tracks, z back-projection, chi2 and the three signal tests;
// v[4] = (x, y, z, chi2) when all pass.
__device__ inline bool vertex_combo(const VTrack* T0, const VTrack* T1, const VTrack* T2, const Consts& C,
                                    const VPoints& P, int c, double* v) {
  const VTrack* tk[3] = {T0, T1, T2};
  double w = 0, mx = 0, my = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool second = (c >> k) & 1;   // selects without a dynamic index (no scratch)
    const double x = second ? P.qx[k][1] : P.qx[k][0], y = second ? P.qy[k][1] : P.qy[k][0];
    const double s2 = second ? P.s2[k][1] : P.s2[k][0];
    const double iw = 1.0 / s2;
    w += iw; mx += x * iw; my += y * iw;
  }
  const double iwt = 1.0 / w;
  mx *= iwt; my *= iwt;
  // per track: the point of closest approach, its turning angle, z and the
  // inverse variance (one division each), and the unit radial direction
  // (reused for the momentum below)
  double px[3], py[3], pz[3], ws[3], ux[3], uy[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const VTrack& t = *tk[k];
    const double ex = mx - t.cx, ey = my - t.cy;
    const double en = sqrt(ex * ex + ey * ey);
    if (en == 0.0) return false;
    const double ien = 1.0 / en;
    ux[k] = ex * ien;
    uy[k] = ey * ien;
    px[k] = t.cx + t.rt * ux[k];
    py[k] = t.cy + t.rt * uy[k];
    const double dphi = back_turn(t, px[k], py[k]);
    pz[k] = t.hz - dphi * t.rbar * t.cth;
    const double s = t.rt * dphi;
    ws[k] = 1.0 / (t.sms0 * t.sms0 * s * s + (double)C.sig_pix * (double)C.sig_pix);
  }
  const double wz = ws[0] + ws[1] + ws[2];
  const double mz = (pz[0] * ws[0] + pz[1] * ws[1] + pz[2] * ws[2]) / wz;
  double chi2 = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double ex = px[k] - mx, ey = py[k] - my, ez = pz[k] - mz;
    chi2 += (ex * ex + ey * ey + ez * ez) * ws[k];
  }
  const double dt = cone_dist(sqrt(mx * mx + my * my), mz, C);
  double sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const VTrack& t = *tk[k];
    const double pt = kCLight * (double)C.b * t.rt;
    // travel direction: clockwise (positive) -> (uy, -ux)
    sx += pt * t.q * uy[k];
    sy -= pt * t.q * ux[k];
    sz += t.p * t.cth;
  }
  const double ps = sqrt(sx * sx + sy * sy + sz * sz);
  if (!(chi2 <= (double)C.chi2_v && dt <= (double)C.d_target && ps <= (double)C.p_sum)) return false;
  v[0] = mx; v[1] = my; v[2] = mz; v[3] = chi2;
  return true;
}

// All combinations of one triple in order: the passing one with the lowest
// chi2 (the first of equal ones) in v[4].
__device__ __forceinline__ bool vertex_triple_inline(const VTrack* T0, const VTrack* T1, const VTrack* T2,
                                                     const Consts& C, double* v) {
  VPoints P;
  if (!vertex_points(T0, T1, T2, C, P)) return false;
  const int m = vertex_combos(P);
  bool found = false;
  for (int c = 0; c < 8; ++c) {
    double u[4];
    if ((m >> c & 1) && vertex_combo(T0, T1, T2, C, P, c, u) && (!found || u[3] < v[3])) {
      for (int k = 0; k < 4; ++k) v[k] = u[k];
      found = true;
    }
  }
  return found;
}

__device__ bool vertex_triple(const VTrack* T0, const VTrack* T1, const VTrack* T2, const Consts& C, double* v) {
  return vertex_triple_inline(T0, T1, T2, C, v);
}

// ================================================================ refined vertex
// The more precise vertex reconstruction that Section VII names as the next
// step: the point v minimising J(v, phi) = sum_k w_k |H_k(phi_k) - v|^2 jointly
// over v and one backward turning angle phi_k per track (H_k the helix of
// track k), with 1/w_k eq. track-error's variance at the track's closest
// approach to the rough estimate, held fixed.  Gauss-Newton in float64 from
// the rough estimate.  For a fixed vertex step each angle's linearised
// optimum is explicit, so a step solves only the 3x3 system
//   sum_k w_k (I - u_k u_k^T) dv = sum_k w_k (I - u_k u_k^T) d_k
// (u_k the unit tangent T_k / |T_k|, d_k = H_k - v), and then
//   dphi_k = T_k . (dv - d_k) / |T_k|^2.
// A step that does not lower J is halved (up to kRefineHalvings times) until
// it does, unless it is below 1e-6 mm; converged once a step is below
// 1e-10 mm and 1e-12 rad, within kRefineIters steps (a wave runs as long as
// its slowest lane, so both limits bound the kernel's tail).
constexpr int kRefineIters = 16;
constexpr int kRefineHalvings = 8;

struct Helix {
  double cx, cy, rt, ps0, q, dz, hz;   // z = hz - phi * dz
};

__device__ inline Helix helix_of(const VTrack& t) {
  return Helix{t.cx, t.cy, t.rt, atan2(t.hy - t.cy, t.hx - t.cx), t.q, t.rbar * t.cth, t.hz};
}

// d = H(phi) - v and the tangent dH/dphi
__device__ inline void helix_eval(const Helix& h, double phi, double vx, double vy, double vz, double* d,
                                  double* tg) {
  double s, c;
  sincos(h.ps0 + h.q * phi, &s, &c);   // backwards of a clockwise (positive) track is counter-clockwise
  d[0] = h.cx + h.rt * c - vx;
  d[1] = h.cy + h.rt * s - vy;
  d[2] = h.hz - phi * h.dz - vz;
  tg[0] = -h.q * h.rt * s;
  tg[1] = h.q * h.rt * c;
  tg[2] = -h.dz;
}

// o[8] = refined x, y, z, J, rough x, y, z, chi2.  Returns the iterations
// used (converged), 0 if the rough estimate does not pass, -1 if no
// convergence within kRefineIters (o[0..3] then hold the last iterate).
__device__ int refine_vertex(const VTrack& A, const VTrack& B, const VTrack& E, const Consts& C, double* o) {
  double rv[4];
  if (!vertex_triple_inline(&A, &B, &E, C, rv)) return 0;
  o[4] = rv[0]; o[5] = rv[1]; o[6] = rv[2]; o[7] = rv[3];
  const Helix h[3] = {helix_of(A), helix_of(B), helix_of(E)};
  const VTrack* tk[3] = {&A, &B, &E};
  double phi[3], w[3];
  double vx = rv[0], vy = rv[1], vz = rv[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const VTrack& t = *tk[k];
    const double ex = vx - t.cx, ey = vy - t.cy, en = sqrt(ex * ex + ey * ey);   // en > 0: the estimate passed
    const double px = t.cx + t.rt * ex / en, py = t.cy + t.rt * ey / en;
    phi[k] = back_turn(t, px, py);
    w[k] = 1.0 / sigma2_at(t, px, py, C);
  }
  double d[3][3], tg[3][3], J = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    helix_eval(h[k], phi[k], vx, vy, vz, d[k], tg[k]);
    J += w[k] * (d[k][0] * d[k][0] + d[k][1] * d[k][1] + d[k][2] * d[k][2]);
  }
  int status = -1;
  for (int it = 1; it <= kRefineIters; ++it) {
    double sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0, bx = 0, by = 0, bz = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double tt = tg[k][0] * tg[k][0] + tg[k][1] * tg[k][1] + tg[k][2] * tg[k][2];
      const double ux = tg[k][0], uy = tg[k][1], uz = tg[k][2], wk = w[k], wt = wk / tt;
      sxx += wk - wt * ux * ux; sxy -= wt * ux * uy; sxz -= wt * ux * uz;
      syy += wk - wt * uy * uy; syz -= wt * uy * uz; szz += wk - wt * uz * uz;
      const double ud = (ux * d[k][0] + uy * d[k][1] + uz * d[k][2]) * wt;
      bx += wk * d[k][0] - ud * ux; by += wk * d[k][1] - ud * uy; bz += wk * d[k][2] - ud * uz;
    }
    // S^-1 b by the adjugate
    const double a00 = syy * szz - syz * syz, a01 = sxz * syz - sxy * szz, a02 = sxy * syz - sxz * syy;
    const double a11 = sxx * szz - sxz * sxz, a12 = sxy * sxz - sxx * syz, a22 = sxx * syy - sxy * sxy;
    const double det = sxx * a00 + sxy * a01 + sxz * a02;
    const double tr = sxx + syy + szz;
    if (!(det > 1e-12 * tr * tr * tr)) break;                 // parallel tracks: no unique vertex
    const double dvx = (a00 * bx + a01 * by + a02 * bz) / det;
    const double dvy = (a01 * bx + a11 * by + a12 * bz) / det;
    const double dvz = (a02 * bx + a12 * by + a22 * bz) / det;
    double dp[3], dpmax = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double tt = tg[k][0] * tg[k][0] + tg[k][1] * tg[k][1] + tg[k][2] * tg[k][2];
      dp[k] = (tg[k][0] * (dvx - d[k][0]) + tg[k][1] * (dvy - d[k][1]) + tg[k][2] * (dvz - d[k][2])) / tt;
      dpmax = fmax(dpmax, fabs(dp[k]));
    }
    const double dvmax = fmax(fabs(dvx), fmax(fabs(dvy), fabs(dvz)));
    if (dvmax < 1e-10 && dpmax < 1e-12) { status = it; break; }
    // a step below 1e-6 mm is taken as it is: near the minimum the rounding
    // of J exceeds the decrease such a step brings, and Gauss-Newton
    // converges there without a line search
    const bool small = dvmax < 1e-6 && dpmax < 1e-8;
    bool accepted = false;
    double f = 1.0;
    for (int hv = 0; hv <= kRefineHalvings && !accepted; ++hv, f *= 0.5) {
      double nd[3][3], nt[3][3], Jn = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        helix_eval(h[k], phi[k] + f * dp[k], vx + f * dvx, vy + f * dvy, vz + f * dvz, nd[k], nt[k]);
        Jn += w[k] * (nd[k][0] * nd[k][0] + nd[k][1] * nd[k][1] + nd[k][2] * nd[k][2]);
      }
      if (Jn <= J || small) {
        vx += f * dvx; vy += f * dvy; vz += f * dvz; J = Jn;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          phi[k] += f * dp[k];
#pragma unroll
          for (int i = 0; i < 3; ++i) { d[k][i] = nd[k][i]; tg[k][i] = nt[k][i]; }
        }
        accepted = true;
      }
    }
    if (!accepted) break;
  }
  o[0] = vx; o[1] = vy; o[2] = vz; o[3] = J;
  return status;
}

// One lane per listed triple (rows {frame, a, b, c} of track indices), the
// tracks' float64 parameters prepared once per track beforehand.
__global__ void __launch_bounds__(256) k_refine(const VTrack* __restrict__ vt, const int32_t* __restrict__ vok,
                                                int n_tracks, const int32_t* __restrict__ rows, int n,
                                                const int32_t* __restrict__ n_valid, Consts C, double* out,
                                                int32_t* status) {
  int lim = n;
  if (n_valid) lim = min(n, max(*n_valid, 0));
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < lim; i += gridDim.x * blockDim.x) {
    const int a = rows[4 * (size_t)i + 1], b = rows[4 * (size_t)i + 2], e = rows[4 * (size_t)i + 3];
    double o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = __builtin_nan("");
    int st = -2;
    if ((unsigned)a < (unsigned)n_tracks && (unsigned)b < (unsigned)n_tracks && (unsigned)e < (unsigned)n_tracks &&
        vok[a] && vok[b] && vok[e])
      st = refine_vertex(vt[a], vt[b], vt[e], C, o);
    double* dst = out + 8 * (size_t)i;
#pragma unroll
    for (int k = 0; k < 8; ++k) dst[k] = o[k];
    status[i] = st;
  }
}

constexpr int kVtxTracks = 256;   // tracks of one frame staged in LDS for the vertex wave
constexpr int kPairWords = 64;    // pair-prefilter bits per frame: 64 x 64 (512 B of LDS)
constexpr int kPairFilterMin = 512;   // triples of a frame from which the prefilter pays

// Vertex stage of one frame by one wave (Alg. 4): tracks split by charge,
// lanes over the flat index of e+e+e- triples (unordered e+ pair, e-) for
// the energy test and the combination cap; the energy-passing triples are
// compacted so that the vertex estimate runs on full waves; a wave-wide
// minimum of the vertex chi2 (ties to the lowest triple index) gives the
// reported vertex.  id(j) gives the j-th track slot.
// Optional record of the energy-passing triples of a frame (debug view of
// the standalone vertex entry point): rows {frame, track a, track b, track c}
// (a, b the e+ tracks, c the e- track, as given by id) appended to rows[cap]
// with the row count at *n.
struct TripleRec {
  int32_t* rows;
  int32_t* n;
  int cap;
};

template <class Id>
__device__ void vertex_wave(int f, int n, const Id& id, const VTrack* __restrict__ vt,
                            const int32_t* __restrict__ vok, const Consts& C, uint32_t* __restrict__ flags,
                            int32_t* __restrict__ ncombo, float* __restrict__ vtx, TripleRec rec = TripleRec{}) {
  const int lane = threadIdx.x;
  const double elo = kMassMu - (double)C.de_max, ehi = kMassMu + (double)C.de_max;
  if (n > kVtxTracks) {
    // more tracks than the LDS table holds (lifted caps): one lane, serially
    if (lane == 0) {
      long long cnt = 0;
      for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b)
          for (int e = 0; e < n; ++e) {
            const int ta = id(a), tb = id(b), te = id(e);
            if (!vok[ta] || !vok[tb] || !vok[te] || vt[ta].q < 0 || vt[tb].q < 0 || vt[te].q > 0) continue;
            const double s = vt[ta].E + vt[tb].E + vt[te].E;
            const bool ep = s >= elo && s <= ehi;
            cnt += ep;
            if (ep && rec.rows) {
              const int r = atomicAdd(rec.n, 1);
              if (r < rec.cap) *reinterpret_cast<int4*>(rec.rows + 4 * r) = make_int4(f, ta, tb, te);
            }
          }
      *ncombo = (int32_t)min(cnt, (long long)0x7fffffff);
      if (cnt > C.max_combo) { *flags |= MU3E_COMBO_OVF | MU3E_KEEP; return; }
      bool found = false;
      double best[4] = {0, 0, 0, 0};
      for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b)
          for (int e = 0; e < n; ++e) {
            const int ta = id(a), tb = id(b), te = id(e);
            if (!vok[ta] || !vok[tb] || !vok[te] || vt[ta].q < 0 || vt[tb].q < 0 || vt[te].q > 0) continue;
            const double s = vt[ta].E + vt[tb].E + vt[te].E;
            if (!(s >= elo && s <= ehi)) continue;
            double v[4];
            if (vertex_triple(&vt[ta], &vt[tb], &vt[te], C, v) && (!found || v[3] < best[3])) {
              for (int k = 0; k < 4; ++k) best[k] = v[k];
              found = true;
            }
          }
      if (found) {
        *flags |= MU3E_VERTEX | MU3E_KEEP;
        for (int k = 0; k < 4; ++k) vtx[k] = (float)best[k];
      }
    }
    return;
  }
  // ---- split by charge (ballot compaction): the e+ tracks from the front
  // of sid, the e- tracks from its back; their energies alongside in sE
  __shared__ int sid[kVtxTracks];
  __shared__ double sE[kVtxTracks];
  int np = 0, nn = 0;
  for (int base = 0; base < n; base += kWave) {
    const int j = base + lane;
    const int t = j < n ? id(j) : -1;
    const bool ok = t >= 0 && vok[t];
    const bool ps = ok && vt[t].q > 0, ng = ok && vt[t].q < 0;
    const unsigned long long mp = ballot(ps), mn = ballot(ng);
    if (ps) { const int k = np + rank_below(mp); sid[k] = t; sE[k] = vt[t].E; }
    if (ng) { const int k = kVtxTracks - 1 - (nn + rank_below(mn)); sid[k] = t; sE[k] = vt[t].E; }
    np += __popcll(mp);
    nn += __popcll(mn);
  }
  __syncthreads();
  const int npair = np * (np - 1) / 2;
  const int total = npair * nn;   // n <= 256 tracks: below 2^23
  // flat triple index k -> (e+ i, e+ j > i, e- e): k = pair * nn + e, pairs in
  // row-major order (row i holds np - 1 - i pairs and starts at
  // i (2 np - i - 1) / 2), the row found by the quadratic formula and corrected
  auto pair_of = [&](int q, int& i, int& j) {   // e+ pair index q -> (i, j > i)
    const double b = 2.0 * np - 1.0;
    int r = (int)((b - sqrt(fmax(b * b - 8.0 * q, 0.0))) * 0.5);
    r = r < 0 ? 0 : (r > np - 2 ? np - 2 : r);
    while (r > 0 && r * (2 * np - r - 1) / 2 > q) --r;
    while (r + 1 <= np - 2 && (r + 1) * (2 * np - r - 2) / 2 <= q) ++r;
    i = r;
    j = q - r * (2 * np - r - 1) / 2 + r + 1;
  };
  auto decode = [&](int k, int& i, int& j, int& e) {
    const int q = (int)(((double)k + 0.5) / (double)nn);
    e = k - q * nn;
    pair_of(q, i, j);
  };
  // ---- prefilter: bit p of spw for every track pair a triple can use (the
  // e+ pairs in the order of their index q, then the e+e- pairs (i, e) at
  // npair + i nn + e): whether its circles may meet near the target.  A
  // triple whose three pairs do not all pass has no vertex estimate, so it
  // is counted (and listed) but not queued for one; at lambda = 64 about
  // four in five energy-passing triples drop out here.  Frames with more
  // pairs than the table holds queue every energy-passing triple.
  __shared__ unsigned long long spw[kPairWords];
  const int npairs = npair + np * nn;
  const bool pf = total >= kPairFilterMin && npairs <= 64 * kPairWords;
  if (pf) {
    const double lim = (double)C.r_target + (double)C.target_tol;
    for (int base = 0; base < npairs; base += kWave) {
      const int p = base + lane;
      bool ok = false;
      if (p < npairs) {
        int ta, tb;
        if (p < npair) {
          int i, j;
          pair_of(p, i, j);
          ta = sid[i]; tb = sid[j];
        } else {
          const int i = (p - npair) / nn, e = p - npair - i * nn;
          ta = sid[i]; tb = sid[kVtxTracks - 1 - e];
        }
        ok = pair_may_meet(vt[ta], vt[tb], lim * lim);
      }
      const unsigned long long m = ballot(ok);
      if (lane == 0) spw[base / kWave] = m;
    }
    __syncthreads();
  }
  auto pair_bit = [&](int p) -> bool { return (spw[p >> 6] >> (p & 63)) & 1ull; };
  // ---- energy test over every triple (the count is exact even above the
  // cap), and while the count stays within the cap, the passing triples are
  // ballot-compacted into an LDS queue whose full waves get the vertex
  // estimate: per triple its intersection points (one lane each), then the
  // existing (triple, combination) pairs a full wave at a time.  The result
  // is the passing combination with the lowest chi2, ties to the lowest
  // (triple index, combination).
  __shared__ VPoints sP[kWave];
  __shared__ int sT[3 * kWave];
  __shared__ int sq[8 * kWave];
  __shared__ int sk[2 * kWave];   // queue of energy-passing triple indices
  __shared__ int skey[kWave];     // the triple index of each lane's points in sP
  double best = 1e300;
  long long bestk = 0x7fffffffffffffffLL;
  double bv[3] = {0, 0, 0};
  auto estimate = [&](int m) {   // the first m (<= kWave) queued triples
    int ta = 0, tb = 0, te = 0, k = 0;
    int mc = 0;
    if (lane < m) {
      k = sk[lane];
      int i, j, e;
      decode(k, i, j, e);
      ta = sid[i]; tb = sid[j]; te = sid[kVtxTracks - 1 - e];
      VPoints P;
      if (vertex_points(&vt[ta], &vt[tb], &vt[te], C, P)) {
        mc = vertex_combos(P);
        sP[lane] = P;
      }
    }
    sT[3 * lane] = ta; sT[3 * lane + 1] = tb; sT[3 * lane + 2] = te;
    skey[lane] = k;   // for the tie-break key
    const int nc = __popc((unsigned)mc);   // <= 8
    int pos = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
      const unsigned long long mb = ballot((nc >> bit) & 1);
      pos += rank_below(mb) << bit;
      tot += __popcll(mb) << bit;
    }
    for (int c = 0; c < 8; ++c)
      if (mc >> c & 1) sq[pos++] = lane * 8 + c;
    __syncthreads();
    for (int q0 = 0; q0 < tot; q0 += kWave) {
      if (q0 + lane < tot) {
        const int ec = sq[q0 + lane];
        const int l = ec >> 3, c = ec & 7;
        double u[4];
        if (vertex_combo(&vt[sT[3 * l]], &vt[sT[3 * l + 1]], &vt[sT[3 * l + 2]], C, sP[l], c, u)) {
          const long long key = (long long)skey[l] * 8 + c;
          if (u[3] < best || (u[3] == best && key < bestk)) {
            best = u[3]; bestk = key; bv[0] = u[0]; bv[1] = u[1]; bv[2] = u[2];
          }
        }
      }
    }
    __syncthreads();
  };
  int cnt = 0, nq = 0;
  // each lane's triple (ci, cj, ce) of flat index base + lane: decoded once,
  // then advanced by kWave = stq pairs and ste e- tracks per round with
  // integer steps (a row i of e+ pairs holds np - 1 - i of them)
  const int stq = nn > 0 ? kWave / nn : 0, ste = kWave - stq * nn;
  int ci = 0, cj = 0, ce = 0;
  if (lane < total) decode(lane, ci, cj, ce);
  for (int base = 0; base < total; base += kWave) {
    const int k = base + lane;
    const int i = ci, j = cj, e = ce;
    bool ep = false;
    if (k < total) {
      const double s = sE[i] + sE[j] + sE[kVtxTracks - 1 - e];
      ep = s >= elo && s <= ehi;
    }
    if (k + kWave < total) {   // the next index exists: its pair row is reached
      int dq = stq;
      ce += ste;
      if (ce >= nn) { ce -= nn; ++dq; }
      int off = cj - ci - 1 + dq, len = np - 1 - ci;
      while (off >= len) { off -= len; ++ci; --len; }
      cj = ci + 1 + off;
    }
    const unsigned long long bm = ballot(ep);
    if (bm == 0ull) continue;   // wave-uniform
    const int c = __popcll(bm);
    // queued for the estimate: energy-passing, and all three pairs may meet
    const bool eq = ep && (!pf || (pair_bit(i * (2 * np - i - 1) / 2 + j - i - 1) &&
                                   pair_bit(npair + i * nn + e) && pair_bit(npair + j * nn + e)));
    if (rec.rows) {   // debug record (wave-uniform pointer)
      int r0 = 0;
      if (lane == 0) r0 = atomicAdd(rec.n, c);
      r0 = lane_value(r0, 0);
      const int r = r0 + rank_below(bm);
      if (ep && r < rec.cap)
        *reinterpret_cast<int4*>(rec.rows + 4 * r) = make_int4(f, sid[i], sid[j], sid[kVtxTracks - 1 - e]);
    }
    cnt += c;
    if (cnt > C.max_combo) continue;   // over the cap: only counted from here on
    const unsigned long long bq = ballot(eq);
    if (eq) sk[nq + rank_below(bq)] = k;
    nq += __popcll(bq);
    if (nq >= kWave) {
      __syncthreads();
      estimate(kWave);
      const int rem = nq - kWave;
      const int v = lane < rem ? sk[kWave + lane] : 0;
      __syncthreads();
      if (lane < rem) sk[lane] = v;
      __syncthreads();
      nq = rem;
    }
  }
  if (lane == 0) *ncombo = cnt;
  if (cnt > C.max_combo) {
    if (lane == 0) *flags |= MU3E_COMBO_OVF | MU3E_KEEP;
    __syncthreads();
    return;
  }
  if (nq > 0) { __syncthreads(); estimate(nq); }
  // wave-wide minimum of (chi2, key)
  double wb = best;
  long long wk = bestk;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_xor(wb, o, 64);
    const long long ok = __shfl_xor(wk, o, 64);
    if (ob < wb || (ob == wb && ok < wk)) { wb = ob; wk = ok; }
  }
  if (wk != 0x7fffffffffffffffLL && bestk == wk) {
    *flags |= MU3E_VERTEX | MU3E_KEEP;
    vtx[0] = (float)bv[0]; vtx[1] = (float)bv[1]; vtx[2] = (float)bv[2]; vtx[3] = (float)best;
  }
  __syncthreads();
}

// Frames able to form an e+e+e- triple (two e+ and one e- tracks, no
// overflow so far) get a slice of the candidate track table; frames with
// more than max_tracks tracks are flagged (Alg. 3: "marked for storage").
// Two passes without atomics: k_vcount counts per block of frames,
// k_vplace offsets each block by the counts of the blocks before it.  Block
// b of kVBlocks-sized grids owns frames [b * per, (b + 1) * per).
constexpr int kVBlocks = 512;

__device__ inline bool vertex_candidate(int f, const Consts& C, const uint32_t* __restrict__ flags,
                                        const int32_t* __restrict__ counts, const int32_t* __restrict__ ccnt,
                                        int& nt) {
  nt = 0;
  if (flags[f] & (MU3E_HITS_OVF | MU3E_TRIPLET_OVF | MU3E_TRACK_OVF | MU3E_LIST_FULL)) return false;
  nt = counts[3 * f + 1];
  if (nt > C.max_trk) return false;
  const int cc = ccnt[f];
  return (cc & 0xffff) >= 2 && (cc >> 16) >= 1;
}


__global__ void __launch_bounds__(256)
k_vcount(int F, int per, Consts C, uint32_t* __restrict__ flags, const int32_t* __restrict__ counts,
         const int32_t* __restrict__ ccnt, int32_t* __restrict__ blk, int nslot) {
  __shared__ int tmp[512];
  const int f0 = blockIdx.x * per, f1 = min(F, f0 + per);
  int nc = 0, ntot = 0, nbig = 0, unused = 0;
  for (int f = f0 + (int)threadIdx.x; f < f1; f += 256) {
    const uint32_t fl = flags[f];
    if (!(fl & (MU3E_HITS_OVF | MU3E_TRIPLET_OVF | MU3E_LIST_FULL)) && counts[3 * f + 1] > C.max_trk)
      flags[f] = fl | MU3E_TRACK_OVF | MU3E_KEEP;
    int nt;
    if (vertex_candidate(f, C, flags, counts, ccnt, nt)) { ++nc; ntot += nt; nbig += nt > nslot; }
  }
  block_sum2(nc, ntot, tmp);
  block_sum2(nbig, unused, tmp);
  if (threadIdx.x == 0) {
    blk[3 * blockIdx.x] = nc;
    blk[3 * blockIdx.x + 1] = ntot;
    blk[3 * blockIdx.x + 2] = nbig;   // candidate frames with more tracks than slots
  }
}

__global__ void __launch_bounds__(256)
k_vplace(int F, int per, Consts C, const uint32_t* __restrict__ flags, const int32_t* __restrict__ counts,
         const int32_t* __restrict__ ccnt, const int32_t* __restrict__ blk, int32_t* __restrict__ vbase,
         int32_t* __restrict__ vpos, int32_t* __restrict__ cand, int vcap, int32_t* __restrict__ counters) {
  __shared__ int tmp[1024];
  const int B = gridDim.x;
  // offsets of this block: the counts of the blocks before it (and totals)
  int cb = 0, tb = 0, ca = 0, ta = 0, big = 0, unused = 0;
  for (int j = threadIdx.x; j < B; j += 256) {
    const int c = blk[3 * j], t = blk[3 * j + 1];
    ca += c; ta += t; big += blk[3 * j + 2];
    if (j < (int)blockIdx.x) { cb += c; tb += t; }
  }
  block_sum2(cb, tb, tmp);
  block_sum2(ca, ta, tmp);
  block_sum2(big, unused, tmp);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counters[3] = ca;
    counters[4] = ta;
    counters[11] = big;
    if (ta > vcap) atomicOr(&counters[2], ST_TRACK_FULL);
  }
  const int f0 = blockIdx.x * per, f1 = min(F, f0 + per);
  for (int base = f0; base < f1; base += 256) {
    const int f = base + (int)threadIdx.x;
    int nt = 0;
    const bool is_c = f < f1 && vertex_candidate(f, C, flags, counts, ccnt, nt);
    // block exclusive scan of (is_c, nt) over the tile
    tmp[threadIdx.x] = is_c ? 1 : 0;
    tmp[256 + threadIdx.x] = is_c ? nt : 0;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int i = threadIdx.x;
      const int a = i >= o ? tmp[i - o] : 0, b = i >= o ? tmp[256 + i - o] : 0;
      __syncthreads();
      tmp[i] += a;
      tmp[256 + i] += b;
      __syncthreads();
    }
    const int ec = tmp[threadIdx.x] - (is_c ? 1 : 0), et = tmp[256 + threadIdx.x] - (is_c ? nt : 0);
    const int tc = tmp[255], tt = tmp[511];
    if (f < f1) {
      if (is_c) {
        vbase[f] = tb + et;
        vpos[f] = 0;
        cand[cb + ec] = f;
      } else {
        vbase[f] = -1;
      }
    }
    cb += tc;
    tb += tt;
    __syncthreads();
  }
}

// Float64 vertex-stage quantities of the accepted tracks of candidate frames
// with more tracks than slots, placed in the frames' slices of the candidate
// table (vt, vok); one wave per 64-entry slice of the triplet list.  Returns
// at once when there is no such frame.
__global__ void __launch_bounds__(64)
k_vprep(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z, int n_hits,
        const int32_t* __restrict__ lo, Consts C, TripList T, Slices S, const int32_t* __restrict__ res,
        const int32_t* __restrict__ counts, const int32_t* __restrict__ counters, const int32_t* __restrict__ vbase,
        int32_t* __restrict__ vpos, int vcap, VTrack* __restrict__ vt, int32_t* __restrict__ vok, int nslot) {
  if (counters[11] == 0) return;   // every candidate frame's tracks are in its slot row
  const int ns = counters[10];
  for (int v = blockIdx.x; v < ns; v += gridDim.x) {
    const int2 sl = S.all[v];
    if ((int)threadIdx.x >= sl.y) continue;
    const int e = sl.x + (int)threadIdx.x;
    if (res[4 * e] != TR_ACCEPT) continue;
    const int f = T.trips[2 * e];
    const int b = vbase[f];
    if (b < 0 || counts[3 * f + 1] <= nslot) continue;
    const int pos = atomicAdd(&vpos[f], 1);
    if (b + pos >= vcap) continue;   // table full: reported by k_vplace
    const uint32_t pk = (uint32_t)T.trips[2 * e + 1];
    const EntryHits eh = entry_hits(lo, f, pk);
    const int32_t h[4] = {eh.g0, eh.g1, eh.g2, eh.b3 + res[4 * e + 1]};
    vok[b + pos] = vtrack_make(X, Y, Z, n_hits, h, C, vt[b + pos]) ? 1 : 0;
  }
}

struct RangeId {
  int base;
  __device__ int operator()(int j) const { return base + j; }
};

// One wave per candidate frame.  A frame with at most kSmallSlots tracks
// refits them here (lanes over its slot row) into LDS; one with at most
// nslot into its slice of the track table; a larger one uses the table slice
// filled by k_vprep.  Each frame is a long chain of dependent float64 work,
// so two waves per SIMD (at most 256 registers, a few spilled) beat one wave
// with every value in registers.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_vframes_list(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z, int n_hits,
               const int32_t* __restrict__ lo, Consts C, TripList T, const int32_t* __restrict__ res,
               const int32_t* __restrict__ tslot, int nslot, int32_t* __restrict__ counters,
               const int32_t* __restrict__ cand, const int32_t* __restrict__ vbase, const int32_t* __restrict__ vpos,
               int vcap, VTrack* __restrict__ vt, int32_t* __restrict__ vok, uint32_t* __restrict__ flags,
               int32_t* __restrict__ counts, float* __restrict__ vtx) {
  __shared__ VTrack svt[kSmallSlots];
  __shared__ int32_t svok[kSmallSlots];
  const int lane = threadIdx.x;
  const int nc = counters[3];
  // refit of the tracks of frame f's slot row: lane j takes slot j (j < nt)
  auto refit = [&](int f, int j, VTrack& v) -> bool {
    const int e = tslot[f * nslot + j];
    const uint32_t pk = (uint32_t)T.trips[2 * e + 1];
    const EntryHits eh = entry_hits(lo, f, pk);
    const int32_t h[4] = {eh.g0, eh.g1, eh.g2, eh.b3 + res[4 * e + 1]};
    return vtrack_make(X, Y, Z, n_hits, h, C, v);
  };
  // candidate frames: the first by block index, then, when there are more
  // candidates than waves, claimed one at a time (their work varies by
  // orders of magnitude at high rates, so a fixed deal leaves the slowest
  // wave far behind); each wave's last claim is past the end, so every wave
  // leaves the loop
  auto next = [&]() {
    if (nc <= (int)gridDim.x) return nc;
    int v = 0;
    if (lane == 0) v = (int)gridDim.x + atomicAdd(&counters[16], 1);
    return lane_value(v, 0);
  };
  for (int c = blockIdx.x; c < nc; c = next()) {
    const int f = cand[c];
    const int nt = counts[3 * f + 1];
    if (nt <= kSmallSlots) {
      if (lane < nt) {
        VTrack v;
        svok[lane] = refit(f, lane, v) ? 1 : 0;
        svt[lane] = v;
      }
      __syncthreads();
      vertex_wave(f, nt, RangeId{0}, svt, svok, C, &flags[f], &counts[3 * f + 2], vtx + 4 * f);
      continue;
    }
    const int b = vbase[f];
    if (b < 0) continue;
    if (b + nt > vcap) {   // table full (reported in the status word): the frame is kept unprocessed
      if (lane == 0) flags[f] |= MU3E_LIST_FULL | MU3E_KEEP;
      continue;
    }
    if (nt <= nslot) {   // refitted here; otherwise k_vprep filled the slice
      for (int j = lane; j < nt; j += kWave) {
        VTrack v;
        vok[b + j] = refit(f, j, v) ? 1 : 0;
        vt[b + j] = v;
      }
      __threadfence_block();
      __syncthreads();
    }
    vertex_wave(f, nt <= nslot ? nt : vpos[f], RangeId{b}, vt, vok, C, &flags[f], &counts[3 * f + 2], vtx + 4 * f);
  }
}

__global__ void __launch_bounds__(256)
k_vprep_range(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z, int n_hits,
              Consts C, const int32_t* __restrict__ hit, int n, VTrack* __restrict__ vt, int32_t* __restrict__ vok) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    vok[t] = vtrack_make(X, Y, Z, n_hits, hit + 4 * t, C, vt[t]) ? 1 : 0;
}

__global__ void __launch_bounds__(64)
k_vframes_range(int F, int n_tracks, Consts C, const int32_t* __restrict__ off, const VTrack* __restrict__ vt,
                const int32_t* __restrict__ vok, uint32_t* __restrict__ flags, int32_t* __restrict__ combos,
                float* __restrict__ vtx, TripleRec rec) {
  const int lane = threadIdx.x;
  for (int f = blockIdx.x; f < F; f += gridDim.x) {
    if (lane < 4) vtx[4 * f + lane] = __builtin_nanf("");
    const int b = off[f], nt = off[f + 1] - off[f];
    uint32_t fl = 0;
    int32_t nc = 0;
    const bool valid = b >= 0 && nt >= 0 && off[f + 1] <= n_tracks;   // malformed ranges: no triples
    if (valid && nt > C.max_trk) fl = MU3E_TRACK_OVF | MU3E_KEEP;
    __syncthreads();
    if (valid && nt <= C.max_trk && nt >= 3) {
      __shared__ uint32_t sfl;
      __shared__ int32_t snc;
      if (lane == 0) { sfl = 0; snc = 0; }
      __syncthreads();
      vertex_wave(f, nt, RangeId{b}, vt, vok, C, &sfl, &snc, vtx + 4 * f, rec);
      __syncthreads();
      fl = sfl;
      nc = snc;
    }
    if (lane == 0) { flags[f] = fl; combos[f] = nc; }
    __syncthreads();
  }
}

// ================================================================ chunks
// Ingest of a chunk as the readout writes it (Section V-A): hit records of
// three float32 (x, y, z) from the front, sorted by frame and layer; at the
// tail the frame count F (last int32) and, just before it, the 4F + 1 layer
// offsets (hit indices within the chunk).  k_unpack turns it into the SoA
// hits and layer offsets the selection reads, padding frames F .. max_frames
// - 1 as empty, so that a plan bound to max_frames frames runs any chunk.  A
// chunk whose tail is inconsistent (F out of range, offsets overlapping the
// hit records, more hits than max_hits) yields no frames and info = {-1, -1}.
struct ChunkTail {
  int F, n;
  bool ok;
};

__device__ inline ChunkTail chunk_tail(const unsigned char* __restrict__ chunk, long long bytes, int max_frames,
                                       int max_hits) {
  ChunkTail t{0, 0, false};
  if (bytes < 4) return t;
  const int32_t* tail = reinterpret_cast<const int32_t*>(chunk + (bytes & ~3LL) - 4);
  const int F = tail[0];
  if (F < 0 || F > max_frames) return t;
  const long long obytes = 4LL * (4LL * F + 1);
  if (obytes + 4 > (bytes & ~3LL)) return t;
  const int32_t* off = tail - (4 * F + 1);
  const int n = off[4 * F];
  if (n < 0 || n > max_hits || 12LL * n > (bytes & ~3LL) - 4 - obytes || off[0] != 0) return t;
  t.F = F;
  t.n = n;
  t.ok = true;
  return t;
}

__global__ void __launch_bounds__(256)
k_unpack(const unsigned char* __restrict__ chunk, long long bytes, int max_frames, int max_hits, float* __restrict__ X,
         float* __restrict__ Y, float* __restrict__ Z, int32_t* __restrict__ lo, int32_t* __restrict__ info) {
  const ChunkTail t = chunk_tail(chunk, bytes, max_frames, max_hits);
  const int32_t* off = reinterpret_cast<const int32_t*>(chunk + (bytes & ~3LL) - 4) - (4 * t.F + 1);
  const float* rec = reinterpret_cast<const float*>(chunk);
  const int stride = gridDim.x * blockDim.x;
  const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) { info[0] = t.ok ? t.F : -1; info[1] = t.ok ? t.n : -1; }
  const int nl = 4 * max_frames + 1;
  for (int j = i0; j < nl; j += stride) lo[j] = !t.ok ? 0 : (j <= 4 * t.F ? off[j] : t.n);
  if (!t.ok) return;
  for (int i = i0; i < t.n; i += stride) {
    X[i] = rec[3 * i];
    Y[i] = rec[3 * i + 1];
    Z[i] = rec[3 * i + 2];
  }
}

// =========================================================== frame pairs
// Overlapping frame pairs (tracks across a frame boundary, Section VII):
// merged frame g holds, per layer, the hits of frame g and then those of
// frame g + 1, so that the selection run on the merged frames finds tracks
// whose hits fall into two consecutive frames.  Its layer offsets have a
// closed form, lo'[4g + l] = lo[4g + l] + lo[4g + 4 + l] - lo[4]; one wave
// per input frame copies its hits to their two places (the first part of
// merged frame f, the second of merged frame f - 1).  Writes stay inside
// [0, cap) whatever the offsets (a frame whose own offsets are malformed is
// not copied); malformed input offsets give malformed merged offsets, which
// the selection skips.
__global__ void __launch_bounds__(256)
k_pairs(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
        const int32_t* __restrict__ lo, int F, int n_hits, float* __restrict__ Xo, float* __restrict__ Yo,
        float* __restrict__ Zo, int32_t* __restrict__ loo, long long cap) {
  const int lane = (int)threadIdx.x % kWave;
  const int waves = (int)(gridDim.x * blockDim.x) / kWave;
  const int base4 = F > 1 ? lo[4] : 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t <= 4 * (F - 1); t += gridDim.x * blockDim.x)
    loo[t] = lo[t] + lo[t + 4] - base4;
  // one wave per input frame, lanes over its hits (all four layers)
  for (int f = (int)(blockIdx.x * blockDim.x + threadIdx.x) / kWave; f < F; f += waves) {
    const int o = lane < 5 ? lo[4 * f + lane] : 0;
    const int b0 = lane_value(o, 0), b4 = lane_value(o, 4);
    int bl[5], good = b0 >= 0 && b4 <= n_hits;
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      bl[l] = lane_value(o, l);
      if (l > 0) good = good && bl[l] >= bl[l - 1];
    }
    if (!good) continue;
    // where layer l of frame f starts as the first part of merged frame f
    // and after frame f - 1's hits in merged frame f - 1
    long long d0[4], d1[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      d0[l] = f < F - 1 ? (long long)bl[l] + lo[4 * f + 4 + l] - base4 : -1;
      d1[l] = f > 0 ? (long long)lo[4 * f - 4 + l] + bl[l] - base4 + (lo[4 * f - 3 + l] - lo[4 * f - 4 + l]) : -1;
    }
    for (int i = b0 + lane; i < b4; i += kWave) {
      const int l = (i >= bl[1]) + (i >= bl[2]) + (i >= bl[3]);
      const long long k = i - (l == 0 ? bl[0] : l == 1 ? bl[1] : l == 2 ? bl[2] : bl[3]);
      const long long e0 = l == 0 ? d0[0] : l == 1 ? d0[1] : l == 2 ? d0[2] : d0[3];
      const long long e1 = l == 0 ? d1[0] : l == 1 ? d1[1] : l == 2 ? d1[2] : d1[3];
      const float x = X[i], y = Y[i], z = Z[i];
      if (e0 >= 0 && e0 + k < cap) { Xo[e0 + k] = x; Yo[e0 + k] = y; Zo[e0 + k] = z; }
      if (e1 >= 0 && e1 + k < cap) { Xo[e1 + k] = x; Yo[e1 + k] = y; Zo[e1 + k] = z; }
    }
  }
}

// ================================================================== k_fit
__global__ void __launch_bounds__(256)
k_fit(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z, int n_hits,
      const int32_t* __restrict__ trip, int n, Consts C, float* __restrict__ out) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int g0 = trip[3 * t], g1 = trip[3 * t + 1], g2 = trip[3 * t + 2];
    float* o = out + 8 * t;
    const bool inb = (unsigned)g0 < (unsigned)n_hits && (unsigned)g1 < (unsigned)n_hits &&
                     (unsigned)g2 < (unsigned)n_hits;
    Fit<float> f;
    f.ok = false;
    if (inb) f = fit_triplet<float>(X[g0], Y[g0], Z[g0], X[g1], Y[g1], Z[g1], X[g2], Y[g2], Z[g2], C);
    if (!f.ok) {
      for (int k = 0; k < 8; ++k) o[k] = __builtin_nanf("");
      continue;
    }
    o[0] = f.kappa; o[1] = f.s2kappa; o[2] = f.chi2; o[3] = f.rstar; o[4] = f.s2r;
    o[5] = (float)f.c.sgn * f.c.rho; o[6] = f.th1; o[7] = f.th2;
  }
}


// Adjoint of the single triplet fit: for every triplet, grad_chi2[t] times
// the derivative of its chi2 with respect to the coordinates of its three
// hits is added to grad[hit][3] (float32 atomics: the order of the additions
// is not fixed).  Degenerate triplets and out-of-range indices add nothing.
__global__ void __launch_bounds__(256)
k_fit_bwd(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z, int n_hits,
          const int32_t* __restrict__ trip, int n, Consts C, const float* __restrict__ gchi2,
          float* __restrict__ grad) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int g[3] = {trip[3 * t], trip[3 * t + 1], trip[3 * t + 2]};
    if ((unsigned)g[0] >= (unsigned)n_hits || (unsigned)g[1] >= (unsigned)n_hits ||
        (unsigned)g[2] >= (unsigned)n_hits)
      continue;
    double h[9], d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 3; ++k) {
      h[3 * k] = X[g[k]];
      h[3 * k + 1] = Y[g[k]];
      h[3 * k + 2] = Z[g[k]];
    }
    float c;
    if (!fit_chi2_adjoint<float>(h, C, gchi2[t], c, d)) continue;
    for (int k = 0; k < 9; ++k) atomicAdd(&grad[3 * g[k / 3] + k % 3], (float)d[k]);
  }
}

// ============================================================== alignment
// Summed triplet-fit chi2 under per-sensor alignment (tx, ty, tz, alpha):
// a hit h on sensor s is moved to R_z(alpha_s) h + t_s (in float64) and the
// triplet is fitted in float32 as in the track stage.
constexpr int kAlignBlocks = 1024;
constexpr int kAlignMaxSensors = 2048;   // float64 LDS accumulators per block

__global__ void __launch_bounds__(256)
k_align_fwd(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
            const uint16_t* __restrict__ S, int n_hits, const int32_t* __restrict__ trip, int n,
            const float* __restrict__ theta, int n_sensors, Consts C, float* __restrict__ chi2) {
  extern __shared__ double strig[];   // cos, sin of each sensor's angle, once per block
  for (int j = threadIdx.x; j < n_sensors; j += blockDim.x) align_trig(theta, j, strig);
  __syncthreads();
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    chi2[t] = align_chi2_one(X, Y, Z, S, n_hits, n_sensors, theta, strig, trip + 3 * t, C);
}

// cos, sin of each sensor's angle for the backward pass (into the workspace).
__global__ void __launch_bounds__(256) k_align_trig(const float* __restrict__ theta, int n_sensors,
                                                    double* __restrict__ trig) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n_sensors; j += gridDim.x * blockDim.x)
    align_trig(theta, j, trig);
}

// Per block: sum over its triplets of grad_chi2[t] d chi2_t / d theta into
// float64 LDS accumulators, then one partial row per block.
__global__ void __launch_bounds__(256)
k_align_bwd(const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
            const uint16_t* __restrict__ S, int n_hits, const int32_t* __restrict__ trip, int n,
            const float* __restrict__ theta, const double* __restrict__ trig, int n_sensors, Consts C,
            const float* __restrict__ gchi2, double* __restrict__ partial) {
  extern __shared__ double acc[];   // 4 * n_sensors float64 accumulators
  const int np = 4 * n_sensors;
  for (int j = threadIdx.x; j < np; j += blockDim.x) acc[j] = 0.0;
  __syncthreads();
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    double gs[12];
    int s[3];
    if (!align_grad_one(X, Y, Z, S, n_hits, n_sensors, theta, trig, trip + 3 * t, C, gchi2[t], s, gs)) continue;
    for (int k = 0; k < 3; ++k) {
      double* a = acc + 4 * s[k];
      atomicAdd(a + 0, gs[4 * k]);
      atomicAdd(a + 1, gs[4 * k + 1]);
      atomicAdd(a + 2, gs[4 * k + 2]);
      atomicAdd(a + 3, gs[4 * k + 3]);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < np; j += blockDim.x) partial[(size_t)blockIdx.x * np + j] = acc[j];
}

// Column sums of the per-block rows of partial ([blocks][np] float64), in
// two kernels: block (x, g) of k_align_reduce takes 64 columns and the rows
// of group g (blocks / kAlignGroups of them), each of its four waves every
// fourth row with eight independent sums per lane (so that eight loads are
// in flight), and writes its group sum to part2[g]; k_align_reduce2 adds the
// kAlignGroups group sums of each column in order.  Every sum is taken in a
// fixed order, so the result is deterministic.  (A single launch in which
// the last block of each column group adds the group sums needs
// device-scope fences, which write back the L2 of every XCD: it ran twice as
// long as both kernels together.)
constexpr int kAlignGroups = 16;

__global__ void __launch_bounds__(256)
k_align_reduce(const double* __restrict__ partial, int blocks, int np, double* __restrict__ part2) {
  __shared__ double part[4][kWave];
  const int l = (int)threadIdx.x % kWave, w = (int)threadIdx.x / kWave;
  const int j = (int)blockIdx.x * kWave + l;
  const int rows = (blocks + kAlignGroups - 1) / kAlignGroups;
  const int r0 = (int)blockIdx.y * rows, r1 = min(blocks, r0 + rows);
  double s = 0.0;
  if (j < np) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int b = r0 + w;
    for (; b + 28 < r1; b += 32) {   // rows b, b + 4, ..., b + 28
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] += partial[(size_t)(b + 4 * k) * np + j];
    }
    for (; b < r1; b += 4) a[0] += partial[(size_t)b * np + j];
    s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  part[w][l] = s;
  __syncthreads();
  if (w == 0 && j < np) part2[(size_t)blockIdx.y * np + j] = (part[0][l] + part[1][l]) + (part[2][l] + part[3][l]);
}

__global__ void __launch_bounds__(256)
k_align_reduce2(const double* __restrict__ part2, int np, float* __restrict__ grad) {
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= np) return;
  double t = 0.0;
  for (int g = 0; g < kAlignGroups; ++g) t += part2[(size_t)g * np + j];
  grad[j] = (float)t;
}

// Start of a run: counters cleared except counters[7] = handed0 (the
// triplet entries of the chunks the cuts' waves start with), and the claim
// counters and tallies cleared (one block per 4 KiB line group).
__global__ void __launch_bounds__(256) k_init(int32_t* __restrict__ counters, int handed0,
                                              int32_t* __restrict__ claims) {
  const int i = threadIdx.x;
  if (blockIdx.x == 0 && i < kCounters) counters[i] = i == 7 ? handed0 : 0;
  for (int j = i; j < kClaimStride; j += 256) claims[blockIdx.x * kClaimStride + j] = 0;
}

// =============================================================== host side
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t counters, claims, chunks, trips, res, sfit, sall, sblk, redo, vt, vok, ccnt, vbase, vpos, cand, vblk, tslot,
      defer, total;
  int nslot;
};

// Track slots per frame: the track capacity per frame the caller provides,
// rounded up to a power of two, within [kSmallSlots, kMaxSlots].
inline int track_slots(int64_t F, int64_t kc) {
  const int64_t per = F > 0 ? (kc + F - 1) / F : 0;
  int n = kSmallSlots;
  while (n < per && n < kMaxSlots) n *= 2;
  return n;
}

// Entries of each slice table: at most ceil(count / 64) slices per chunk.
inline int64_t slice_capacity(int64_t tc) { return tc / kWave + tc / kMinChunk + 2; }

Layout layout(int64_t F, int64_t tc, int64_t kc) {
  Layout L;
  size_t o = 0;
  L.counters = o; o += align256(kCounters * sizeof(int32_t));
  L.claims = o; o += align256((size_t)kClaimRanges * kClaimStride * sizeof(int32_t));
  L.chunks = o; o += align256((size_t)(tc / kMinChunk + 1) * 4 * sizeof(int32_t));
  L.trips = o; o += align256((size_t)tc * 2 * sizeof(int32_t));
  L.res = o; o += align256((size_t)tc * 4 * sizeof(int32_t));
  L.sfit = o; o += align256((size_t)slice_capacity(tc) * sizeof(int2));
  L.sall = o; o += align256((size_t)slice_capacity(tc) * sizeof(int2));
  L.sblk = o; o += align256((size_t)2 * ((tc / kMinChunk + 1 + 255) / 256) * sizeof(int32_t));
  L.redo = o; o += align256((size_t)(kc / 8 + 1024) * sizeof(int32_t));
  L.vt = o; o += align256((size_t)kc * sizeof(VTrack));
  L.vok = o; o += align256((size_t)kc * sizeof(int32_t));
  L.ccnt = o; o += align256((size_t)F * sizeof(int32_t));
  L.vbase = o; o += align256((size_t)F * sizeof(int32_t));
  L.vpos = o; o += align256((size_t)F * sizeof(int32_t));
  L.cand = o; o += align256((size_t)F * sizeof(int32_t));
  L.vblk = o; o += align256((size_t)3 * kVBlocks * sizeof(int32_t));
  L.nslot = track_slots(F, kc);
  L.tslot = o; o += align256((size_t)F * L.nslot * sizeof(int32_t));
  L.defer = o; o += align256((size_t)F * sizeof(int32_t));
  L.total = o;
  return L;
}

bool make_consts(const mu3e_params_t* p, Consts& C) {
  for (int i = 0; i < 4; ++i) { C.R[i] = p->r_layer[i]; C.zh[i] = p->z_half[i]; }
  if (!(C.R[0] > 0 && C.R[1] > C.R[0] && C.R[2] > C.R[1] && C.R[3] > C.R[2])) return false;
  C.b = p->b_tesla; C.xx0 = p->x_over_x0; C.sig_pix = p->sigma_pixel;
  if (!(C.b > 0 && C.xx0 > 0 && C.sig_pix > 0)) return false;
  C.dl_lo = p->dlambda.lo; C.dl_hi = p->dlambda.hi;
  C.c01_lo = p->cosphi01.lo; C.c01_hi = p->cosphi01.hi;
  C.c12_lo = p->cosphi12.lo; C.c12_hi = p->cosphi12.hi;
  C.rtc_lo = p->rtc_abs.lo; C.rtc_hi = p->rtc_abs.hi;
  if (!(C.dl_lo <= C.dl_hi && C.c01_lo <= C.c01_hi && C.c12_lo <= C.c12_hi && C.rtc_lo >= 0 &&
        C.rtc_lo <= C.rtc_hi))
    return false;
  C.chi2_trk = p->chi2_track_max;
  C.max_trip = p->max_triplets; C.max_trk = p->max_tracks; C.max_combo = p->max_combos;
  C.max_lh = p->max_layer_hits;
  if (C.max_trip < 0 || C.max_trk < 0 || C.max_combo < 0 || C.max_lh < 0) return false;
  C.de_max = p->de_max; C.r_target = p->r_target; C.target_tol = p->target_tol;
  C.chi2_v = p->chi2_vertex_max; C.d_target = p->d_target_max; C.p_sum = p->p_sum_max;
  C.inv01 = 1.0f / (C.R[1] - C.R[0]);
  C.inv12 = 1.0f / (C.R[2] - C.R[1]);
  C.d01 = C.R[1] - C.R[0];
  C.dl_abs = fabsf(C.dl_lo) + fabsf(C.dl_hi);
  C.invRR01 = 1.0f / (C.R[0] * C.R[1]);
  C.invRR12 = 1.0f / (C.R[1] * C.R[2]);
  C.rtc_lo2 = C.rtc_lo * C.rtc_lo;
  C.rtc_hi2 = C.rtc_hi * C.rtc_hi;
  return true;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
  return cus;
}

// Pointers into a caller workspace.
struct WsView {
  int32_t *counters, *claims, *chunks, *trips, *res, *redo, *ccnt, *vbase, *vpos, *cand, *vok, *vblk, *sblk, *tslot,
      *defer;
  Slices S;
  VTrack* vt;
  int redo_cap, nslot;
};

WsView ws_view(void* workspace, const Layout& L, int track_capacity) {
  char* ws = static_cast<char*>(workspace);
  WsView W;
  W.counters = reinterpret_cast<int32_t*>(ws + L.counters);
  W.claims = reinterpret_cast<int32_t*>(ws + L.claims);
  W.chunks = reinterpret_cast<int32_t*>(ws + L.chunks);
  W.trips = reinterpret_cast<int32_t*>(ws + L.trips);
  W.res = reinterpret_cast<int32_t*>(ws + L.res);
  W.S.fit = reinterpret_cast<int2*>(ws + L.sfit);
  W.S.all = reinterpret_cast<int2*>(ws + L.sall);
  W.sblk = reinterpret_cast<int32_t*>(ws + L.sblk);
  W.redo = reinterpret_cast<int32_t*>(ws + L.redo);
  W.vt = reinterpret_cast<VTrack*>(ws + L.vt);
  W.vok = reinterpret_cast<int32_t*>(ws + L.vok);
  W.ccnt = reinterpret_cast<int32_t*>(ws + L.ccnt);
  W.vbase = reinterpret_cast<int32_t*>(ws + L.vbase);
  W.vpos = reinterpret_cast<int32_t*>(ws + L.vpos);
  W.cand = reinterpret_cast<int32_t*>(ws + L.cand);
  W.vblk = reinterpret_cast<int32_t*>(ws + L.vblk);
  W.tslot = reinterpret_cast<int32_t*>(ws + L.tslot);
  W.nslot = L.nslot;
  W.defer = reinterpret_cast<int32_t*>(ws + L.defer);
  W.redo_cap = track_capacity / 8 + 1024;
  return W;
}

TrackOut track_out(const WsView& W, uint32_t* flags, int32_t* counts) {
  TrackOut O;
  O.flags = flags;
  O.res = W.res;
  O.redo = W.redo;
  O.redo_cap = W.redo_cap;
  O.counts = counts;
  O.ccnt = W.ccnt;
  O.tslot = W.tslot;
  O.nslot = W.nslot;
  return O;
}

// The triplet list of a launch with `waves` appending waves: chunks of about
// capacity / (2 waves) entries (so that half the list is left to spare for
// partly filled chunks), clamped to [kMinChunk, kMaxChunk].
TripList trip_list(const WsView& W, int capacity, int waves) {
  TripList T;
  T.trips = W.trips;
  T.chunks = W.chunks;
  T.capacity = capacity;
  int64_t c = waves > 0 ? (int64_t)capacity / (2 * (int64_t)waves) : kMaxChunk;
  if (c < kMinChunk) c = kMinChunk;
  if (c > kMaxChunk) c = kMaxChunk;
  T.chunk = (int)c;
  T.pre = waves < capacity / T.chunk ? waves : capacity / T.chunk;
  return T;
}

// Deferred frames (a layer above the LDS tile) after the cuts kernel of
// either form; a grid of 4 waves per CU claims them one at a time.
void launch_tiles(const mu3e_hits_t& h, const Consts& C, int cus, int tile, const WsView& W, const TripList& T,
                  uint32_t* flags, int32_t* counts, hipStream_t stream) {
  if (tile == 64)
    hipLaunchKernelGGL(k_tiles<64>, dim3(cus * 4), dim3(kWave), 0, stream, h.x, h.y, h.z, h.layer_offsets, C, flags,
                       counts, T, W.counters, W.claims, W.defer);
  else
    hipLaunchKernelGGL(k_tiles<128>, dim3(cus * 4), dim3(kWave), 0, stream, h.x, h.y, h.z, h.layer_offsets, C, flags,
                       counts, T, W.counters, W.claims, W.defer);
}

// Track stage after the cuts of either form: slice tables, float32 fits of
// the entries not fitted yet, float64 re-evaluation.  after_fits (nullable)
// is recorded after k_tracks.
void launch_tracks(const mu3e_hits_t& h, const Consts& C, int cus, const WsView& W, const TripList& T,
                   uint32_t* flags, int32_t* counts, hipStream_t stream, hipEvent_t after_fits) {
  const TrackOut O = track_out(W, flags, counts);
  const int nbk = (int)(((int64_t)T.capacity / T.chunk + 1 + 255) / 256);
  hipLaunchKernelGGL(k_scount, dim3(nbk), dim3(256), 0, stream, T, W.sblk, W.counters, W.claims);
  hipLaunchKernelGGL(k_splace, dim3(nbk), dim3(256), 0, stream, T, W.S, W.sblk, W.counters);
  // many more waves than fit at once: the slices outnumber them only a few
  // times, and the hardware refills finished waves, which balances better
  // than a ragged last round of a resident grid
  hipLaunchKernelGGL(k_tracks, dim3(cus * 128), dim3(kWave), 0, stream, h.x, h.y, h.z, h.layer_offsets, C, flags, T,
                     W.S, O, W.counters);
  if (after_fits) (void)hipEventRecord(after_fits, stream);
  hipLaunchKernelGGL(k_tracks_redo, dim3(cus), dim3(kWave), 0, stream, h.x, h.y, h.z, h.layer_offsets, C, T, O,
                     W.counters);
}

// Vertex stage (Alg. 4) after the track stage of either form; vcap is the
// capacity of the candidate track table.
void launch_vertex(const mu3e_hits_t& h, const Consts& C, int F, int cus, const WsView& W, const TripList& T,
                   uint32_t* flags, int32_t* counts, float* vtx, int vcap, hipStream_t stream, hipEvent_t* ev) {
  int nb = (F + 255) / 256;
  if (nb > kVBlocks) nb = kVBlocks;
  const int per = ((F + nb - 1) / nb + 255) / 256 * 256;
  nb = (F + per - 1) / per;
  hipLaunchKernelGGL(k_vcount, dim3(nb), dim3(256), 0, stream, F, per, C, flags, counts, W.ccnt, W.vblk, W.nslot);
  hipLaunchKernelGGL(k_vplace, dim3(nb), dim3(256), 0, stream, F, per, C, flags, counts, W.ccnt, W.vblk, W.vbase,
                     W.vpos, W.cand, vcap, W.counters);
  hipLaunchKernelGGL(k_vprep, dim3(cus * 16), dim3(kWave), 0, stream, h.x, h.y, h.z, h.n_hits, h.layer_offsets, C, T,
                     W.S, W.res, counts, W.counters, W.vbase, W.vpos, vcap, W.vt, W.vok, W.nslot);
  if (ev) (void)hipEventRecord(ev[3], stream);
  // two waves per SIMD are resident (float64-heavy, many registers): no
  // more blocks than that, so that every candidate frame starts at once
  hipLaunchKernelGGL(k_vframes_list, dim3(cus * 8), dim3(kWave), 0, stream, h.x, h.y, h.z, h.n_hits, h.layer_offsets,
                     C, T, W.res, W.tslot, W.nslot, W.counters, W.cand, W.vbase, W.vpos, vcap, W.vt, W.vok, flags,
                     counts, vtx);
  if (ev) (void)hipEventRecord(ev[4], stream);
}

bool hits_ok(const mu3e_hits_t* h) {
  return h && h->n_frames >= 0 && h->n_hits >= 0 &&
         (h->n_frames == 0 || (h->layer_offsets && (h->n_hits == 0 || (h->x && h->y && h->z))));
}

}  // namespace

extern "C" {

const char* mu3e_status_string(int s) {
  switch (s) {
    case MU3E_OK: return "ok";
    case MU3E_ERR_INVALID_ARG: return "invalid argument";
    case MU3E_ERR_HIP: return "HIP runtime error";
    case MU3E_ERR_CAPACITY: return "workspace too small";
    case MU3E_ERR_UNSUPPORTED: return "unsupported parameter";
  }
  return "unknown status";
}

size_t mu3e_select_workspace_size(int32_t n_frames, int32_t triplet_capacity, int32_t track_capacity) {
  if (n_frames < 0 || triplet_capacity < 0 || triplet_capacity > kMaxTripletCapacity || track_capacity < 0)
    return 0;
  return layout(n_frames, triplet_capacity, track_capacity).total;
}

}  // extern "C"

namespace {

// The plain-form sequence of mu3e_select_frames on a given workspace.
mu3e_status select_impl(const mu3e_hits_t* hits, const mu3e_params_t* params, uint32_t* frame_flags,
                        int32_t* frame_counts, float* frame_vertex, void* workspace, size_t workspace_bytes,
                        int32_t triplet_capacity, int32_t track_capacity, mu3e_debug_t* dbg, hipStream_t stream,
                        hipEvent_t* ev) {
  if (!hits_ok(hits) || !params || triplet_capacity < 0 || triplet_capacity > kMaxTripletCapacity ||
      track_capacity < 0)
    return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (C.max_lh > kMaxTiledLayerHits) return MU3E_ERR_UNSUPPORTED;
  const int F = hits->n_frames;
  const Layout L = layout(F, triplet_capacity, track_capacity);
  if (!workspace || workspace_bytes < L.total) return MU3E_ERR_CAPACITY;
  if (F > 0 && (!frame_flags || !frame_counts || !frame_vertex)) return MU3E_ERR_INVALID_ARG;
  const WsView W = ws_view(workspace, L, track_capacity);
  const int cus = device_cus();
  // waves of the cuts kernel: 20 per CU (all resident), at least enough for
  // 2048 frames each
  int g1 = cus * 20;
  if (g1 < (F + 2047) / 2048) g1 = (F + 2047) / 2048;
  if (g1 > F) g1 = F > 0 ? F : 1;
  const TripList T = trip_list(W, triplet_capacity, g1);
  if (dbg) {
    dbg->counters = W.counters; dbg->triplets = W.trips; dbg->tracks = W.res;
    dbg->triplet_capacity = triplet_capacity; dbg->track_capacity = track_capacity;
    dbg->chunks = W.chunks; dbg->max_chunks = triplet_capacity / kMinChunk + 1; dbg->chunk_size = T.chunk;
  }
  if (ev && hipEventRecord(ev[0], stream) != hipSuccess) return MU3E_ERR_HIP;
  hipLaunchKernelGGL(k_init, dim3(kClaimRanges), dim3(256), 0, stream, W.counters, T.pre * T.chunk, W.claims);
  if (F == 0) {
    for (int k = 1; ev && k < 5; ++k) (void)hipEventRecord(ev[k], stream);
    return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
  }
  hipLaunchKernelGGL(k_cuts<kPlainTile>, dim3(g1), dim3(kWave), 0, stream, hits->x, hits->y, hits->z,
                     hits->layer_offsets, F, hits->n_hits, C, frame_flags, frame_counts, frame_vertex, W.ccnt, T,
                     W.counters, W.claims, W.defer);
  launch_tiles(*hits, C, cus, kPlainTile, W, T, frame_flags, frame_counts, stream);
  if (ev) (void)hipEventRecord(ev[1], stream);
  launch_tracks(*hits, C, cus, W, T, frame_flags, frame_counts, stream, nullptr);
  if (ev) (void)hipEventRecord(ev[2], stream);
  launch_vertex(*hits, C, F, cus, W, T, frame_flags, frame_counts, frame_vertex, track_capacity, stream, ev);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

// Device address of `scratch` on each device, resolved on the first call of
// mu3e_select_frames_static on that device (with the device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

mu3e_status scratch_of_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MU3E_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return MU3E_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MU3E_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MU3E_OK;
}

}  // namespace

extern "C" {

mu3e_status mu3e_select_frames_timed(const mu3e_hits_t* hits, const mu3e_params_t* params, uint32_t* frame_flags,
                                     int32_t* frame_counts, float* frame_vertex, void* workspace,
                                     size_t workspace_bytes, int32_t triplet_capacity, int32_t track_capacity,
                                     mu3e_debug_t* dbg, hipStream_t stream, hipEvent_t* ev) {
  return select_impl(hits, params, frame_flags, frame_counts, frame_vertex, workspace, workspace_bytes,
                     triplet_capacity, track_capacity, dbg, stream, ev);
}

mu3e_status mu3e_select_frames(const mu3e_hits_t* hits, const mu3e_params_t* params, uint32_t* frame_flags,
                               int32_t* frame_counts, float* frame_vertex, void* workspace,
                               size_t workspace_bytes, int32_t triplet_capacity, int32_t track_capacity,
                               mu3e_debug_t* dbg, hipStream_t stream) {
  return select_impl(hits, params, frame_flags, frame_counts, frame_vertex, workspace, workspace_bytes,
                     triplet_capacity, track_capacity, dbg, stream, nullptr);
}

mu3e_status mu3e_select_frames_static(const mu3e_hits_t* hits, const mu3e_params_t* params, uint32_t* frame_flags,
                                      int32_t* frame_counts, float* frame_vertex, int32_t triplet_capacity,
                                      int32_t track_capacity, mu3e_debug_t* dbg, hipStream_t stream) {
  // sizes first (no device call): a request beyond the static array is refused
  if (!hits || hits->n_frames < 0 || triplet_capacity < 0 || triplet_capacity > kMaxTripletCapacity ||
      track_capacity < 0)
    return MU3E_ERR_INVALID_ARG;
  if (layout(hits->n_frames, triplet_capacity, track_capacity).total > sizeof(scratch)) return MU3E_ERR_CAPACITY;
  void* ws = nullptr;
  const mu3e_status st = scratch_of_current_device(&ws);
  if (st != MU3E_OK) return st;
  return select_impl(hits, params, frame_flags, frame_counts, frame_vertex, ws, sizeof(scratch), triplet_capacity,
                     track_capacity, dbg, stream, nullptr);
}

mu3e_status mu3e_chunk_unpack(const void* chunk, int64_t chunk_bytes, int32_t max_frames, int32_t max_hits, float* x,
                              float* y, float* z, int32_t* layer_offsets, int32_t* info, hipStream_t stream) {
  if (!chunk || chunk_bytes < 4 || max_frames < 0 || max_hits < 0 || !layer_offsets || !info ||
      (max_hits > 0 && (!x || !y || !z)) || (reinterpret_cast<uintptr_t>(chunk) & 3))
    return MU3E_ERR_INVALID_ARG;
  const int cus = device_cus();
  const int64_t work = (int64_t)max_hits > 4 * (int64_t)max_frames + 1 ? max_hits : 4 * (int64_t)max_frames + 1;
  const int blocks = (int)((work + 255) / 256 < cus * 8 ? (work + 255) / 256 : cus * 8);
  hipLaunchKernelGGL(k_unpack, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream,
                     static_cast<const unsigned char*>(chunk), (long long)chunk_bytes, max_frames, max_hits, x, y, z,
                     layer_offsets, info);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_pair_frames(const mu3e_hits_t* hits, float* x, float* y, float* z, int32_t* layer_offsets,
                             int64_t capacity, hipStream_t stream) {
  if (!hits_ok(hits) || hits->n_frames < 2 || !layer_offsets || capacity < 0) return MU3E_ERR_INVALID_ARG;
  if (capacity < 2 * (int64_t)hits->n_hits) return MU3E_ERR_CAPACITY;
  if (capacity > 0 && (!x || !y || !z)) return MU3E_ERR_INVALID_ARG;
  const int cus = device_cus();
  const int64_t waves = hits->n_frames;
  const int blocks = (int)((waves + 3) / 4 < cus * 16 ? (waves + 3) / 4 : cus * 16);
  hipLaunchKernelGGL(k_pairs, dim3(blocks), dim3(256), 0, stream, hits->x, hits->y, hits->z, hits->layer_offsets,
                     hits->n_frames, hits->n_hits, x, y, z, layer_offsets, (long long)capacity);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_fit_triplets(const mu3e_hits_t* hits, const int32_t* trip, int32_t n, const mu3e_params_t* params,
                              float* out, hipStream_t stream) {
  if (!hits || hits->n_hits < 0 || n < 0 || !params || (n > 0 && (!trip || !out || !hits->x || !hits->y || !hits->z)))
    return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (n == 0) return MU3E_OK;
  const int cus = device_cus();
  const int blocks = (n + 255) / 256 < cus * 8 ? (n + 255) / 256 : cus * 8;
  hipLaunchKernelGGL(k_fit, dim3(blocks), dim3(256), 0, stream, hits->x, hits->y, hits->z, hits->n_hits, trip, n, C,
                     out);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

size_t mu3e_vertex_workspace_size(int32_t n_tracks) {
  if (n_tracks < 0) return 0;
  return align256((size_t)n_tracks * sizeof(VTrack)) + align256((size_t)n_tracks * sizeof(int32_t));
}

mu3e_status mu3e_vertex_debug(const mu3e_hits_t* hits, const mu3e_tracks_t* tracks, const mu3e_params_t* params,
                              uint32_t* frame_flags, int32_t* frame_combos, float* frame_vertex, void* workspace,
                              size_t workspace_bytes, int32_t* triples, int32_t triple_capacity, int32_t* n_triples,
                              hipStream_t stream) {
  if (!hits || hits->n_hits < 0 || !tracks || !params || tracks->n_frames < 0 || tracks->n_tracks < 0 ||
      triple_capacity < 0 || (triples && !n_triples))
    return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  const int F = tracks->n_frames, n = tracks->n_tracks;
  if (F == 0) return MU3E_OK;
  if (!tracks->frame_offsets || !frame_flags || !frame_combos || !frame_vertex ||
      (n > 0 && (!tracks->hit || !hits->x || !hits->y || !hits->z)))
    return MU3E_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < mu3e_vertex_workspace_size(n)) return MU3E_ERR_CAPACITY;
  VTrack* vt = static_cast<VTrack*>(workspace);
  int32_t* vok = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + align256((size_t)n * sizeof(VTrack)));
  const int cus = device_cus();
  if (n > 0) {
    const int b = (n + 255) / 256 < cus * 8 ? (n + 255) / 256 : cus * 8;
    hipLaunchKernelGGL(k_vprep_range, dim3(b), dim3(256), 0, stream, hits->x, hits->y, hits->z, hits->n_hits, C,
                       tracks->hit, n, vt, vok);
  }
  const int g = F < cus * 16 ? F : cus * 16;
  hipLaunchKernelGGL(k_vframes_range, dim3(g), dim3(kWave), 0, stream, F, n, C, tracks->frame_offsets, vt, vok,
                     frame_flags, frame_combos, frame_vertex, TripleRec{triples, n_triples, triple_capacity});
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_vertex_refine(const mu3e_hits_t* hits, const mu3e_tracks_t* tracks, const int32_t* triples,
                               int32_t n, const int32_t* n_valid, const mu3e_params_t* params, double* out,
                               int32_t* status, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!hits || hits->n_hits < 0 || !tracks || tracks->n_tracks < 0 || n < 0 || !params) return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (n == 0) return MU3E_OK;
  const int nt = tracks->n_tracks;
  if (!triples || !out || !status || (nt > 0 && (!tracks->hit || !hits->x || !hits->y || !hits->z)))
    return MU3E_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < mu3e_vertex_workspace_size(nt)) return MU3E_ERR_CAPACITY;
  VTrack* vt = static_cast<VTrack*>(workspace);
  int32_t* vok = reinterpret_cast<int32_t*>(static_cast<char*>(workspace) + align256((size_t)nt * sizeof(VTrack)));
  const int cus = device_cus();
  if (nt > 0) {
    const int b = (nt + 255) / 256 < cus * 8 ? (nt + 255) / 256 : cus * 8;
    hipLaunchKernelGGL(k_vprep_range, dim3(b), dim3(256), 0, stream, hits->x, hits->y, hits->z, hits->n_hits, C,
                       tracks->hit, nt, vt, vok);
  }
  const int blocks = (n + 255) / 256 < cus * 8 ? (n + 255) / 256 : cus * 8;
  hipLaunchKernelGGL(k_refine, dim3(blocks), dim3(256), 0, stream, vt, vok, nt, triples, n, n_valid, C, out, status);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_vertex(const mu3e_hits_t* hits, const mu3e_tracks_t* tracks, const mu3e_params_t* params,
                        uint32_t* frame_flags, int32_t* frame_combos, float* frame_vertex, void* workspace,
                        size_t workspace_bytes, hipStream_t stream) {
  return mu3e_vertex_debug(hits, tracks, params, frame_flags, frame_combos, frame_vertex, workspace, workspace_bytes,
                           nullptr, 0, nullptr, stream);
}

mu3e_status mu3e_fit_triplets_backward(const mu3e_hits_t* hits, const int32_t* trip, int32_t n,
                                       const mu3e_params_t* params, const float* grad_chi2, float* grad_xyz,
                                       hipStream_t stream) {
  if (!hits || hits->n_hits < 0 || n < 0 || !params ||
      (n > 0 && (!trip || !grad_chi2 || !grad_xyz || !hits->x || !hits->y || !hits->z)))
    return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (n == 0) return MU3E_OK;
  const int cus = device_cus();
  const int blocks = (n + 255) / 256 < cus * 8 ? (n + 255) / 256 : cus * 8;
  hipLaunchKernelGGL(k_fit_bwd, dim3(blocks), dim3(256), 0, stream, hits->x, hits->y, hits->z, hits->n_hits, trip,
                     n, C, grad_chi2, grad_xyz);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

// Workspace of mu3e_align_backward: the per-block rows, the group sums and
// the sensors' cos, sin table.
struct AlignLayout {
  size_t partial, part2, trig, total;
};

static AlignLayout align_layout(int n_sensors) {
  const size_t np = 4 * (size_t)n_sensors;
  AlignLayout L;
  L.partial = 0;
  L.part2 = align256((size_t)kAlignBlocks * np * sizeof(double));
  L.trig = L.part2 + align256((size_t)kAlignGroups * np * sizeof(double));
  L.total = L.trig + align256(2 * (size_t)n_sensors * sizeof(double));
  return L;
}

size_t mu3e_align_workspace_size(int32_t n_sensors) {
  if (n_sensors <= 0 || n_sensors > kAlignMaxSensors) return 0;
  return align_layout(n_sensors).total;
}

static bool align_args_ok(const mu3e_hits_t* hits, const int32_t* trip, int32_t n, const float* theta,
                          int32_t n_sensors) {
  return hits && hits->n_hits >= 0 && n >= 0 && n_sensors > 0 &&
         (n == 0 || (trip && theta && hits->x && hits->y && hits->z && hits->sensor));
}

mu3e_status mu3e_align_chi2(const mu3e_hits_t* hits, const int32_t* trip, int32_t n, const float* theta,
                            int32_t n_sensors, const mu3e_params_t* params, float* chi2, hipStream_t stream) {
  if (!align_args_ok(hits, trip, n, theta, n_sensors) || !params || (n > 0 && !chi2)) return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (n_sensors > kAlignMaxSensors) return MU3E_ERR_UNSUPPORTED;
  if (n == 0) return MU3E_OK;
  const int cus = device_cus();
  // four blocks per compute unit: each block computes the sensor table once
  // and then takes several triplets per lane
  const int b = (n + 255) / 256 < cus * 4 ? (n + 255) / 256 : cus * 4;
  hipLaunchKernelGGL(k_align_fwd, dim3(b), dim3(256), 2 * (size_t)n_sensors * sizeof(double), stream, hits->x,
                     hits->y, hits->z, hits->sensor, hits->n_hits, trip, n, theta, n_sensors, C, chi2);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_align_backward(const mu3e_hits_t* hits, const int32_t* trip, int32_t n, const float* theta,
                                int32_t n_sensors, const mu3e_params_t* params, const float* grad_chi2,
                                float* grad_theta, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!align_args_ok(hits, trip, n, theta, n_sensors) || !params || !grad_theta || (n > 0 && !grad_chi2))
    return MU3E_ERR_INVALID_ARG;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (n_sensors > kAlignMaxSensors) return MU3E_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < mu3e_align_workspace_size(n_sensors)) return MU3E_ERR_CAPACITY;
  const AlignLayout AL = align_layout(n_sensors);
  char* ws = static_cast<char*>(workspace);
  double* partial = reinterpret_cast<double*>(ws + AL.partial);
  double* part2 = reinterpret_cast<double*>(ws + AL.part2);
  double* trig = reinterpret_cast<double*>(ws + AL.trig);
  const int np = 4 * n_sensors;
  const int ncb = (np + kWave - 1) / kWave;
  // the sensors' cos, sin table once into the workspace (in each block's LDS
  // beside the accumulators it lowers the occupancy and ran slower); none
  // without triplets: theta may then be NULL, and the gradient is zero
  if (n > 0)
    hipLaunchKernelGGL(k_align_trig, dim3((n_sensors + 255) / 256), dim3(256), 0, stream, theta, n_sensors, trig);
  hipLaunchKernelGGL(k_align_bwd, dim3(kAlignBlocks), dim3(256), (size_t)np * sizeof(double), stream, hits->x, hits->y,
                     hits->z, hits->sensor, hits->n_hits, trip, n, theta, trig, n_sensors, C, grad_chi2, partial);
  hipLaunchKernelGGL(k_align_reduce, dim3(ncb, kAlignGroups), dim3(256), 0, stream, partial, kAlignBlocks, np, part2);
  hipLaunchKernelGGL(k_align_reduce2, dim3((np + 255) / 256), dim3(256), 0, stream, part2, np, grad_theta);
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

// The persistent kernel of a plan: fused fits or not, LDS tiles of 64 or 128
// hits per layer.
using BatchedFn = void (*)(const float*, const float*, const float*, const int32_t*, int, int, int, Consts,
                           uint32_t*, int32_t*, float*, int32_t*, TripList, TrackOut, int32_t*, int32_t*, int,
                           int32_t*);
static BatchedFn batched_kernel(bool fuse, int tile) {
  if (tile == 64) return fuse ? k_batched<true, 64> : k_batched<false, 64>;
  return fuse ? k_batched<true, 128> : k_batched<false, 128>;
}

constexpr int kMaxParts = 4;   // sub-batches of a plan

// One sub-batch of a plan: a contiguous range of the batch's frames with its
// own part of the workspace, and two graphs, the cuts (counters cleared,
// persistent kernel) and the rest (fits, float64 re-evaluation, vertex
// stage), so that the rest of one sub-batch can overlap the cuts of the next.
struct PlanPart {
  mu3e_hits_t hits;   // layer_offsets advanced to the first frame, n_frames of the part
  WsView W;
  TripList T;
  uint32_t* flags;
  int32_t* counts;
  float* vertex;
  int first, F, Fs, P, kcap;
  mu3e_debug_t dbg;
  hipGraph_t graph[2];
  hipGraphExec_t exec[2];
};

struct mu3e_plan {
  mu3e_tuning_t tuning;
  Consts C;
  int cus, nparts;
  PlanPart part[kMaxParts];
  hipStream_t side[kMaxParts];   // streams of parts 1 .. nparts-1
  hipEvent_t cuts_done[kMaxParts], part_done[kMaxParts];
};

// Frames, capacities and workspace offset of part j of a plan over F frames
// (sizes split evenly; each part's workspace laid out as for
// mu3e_select_workspace_size).
struct PartSplit {
  int first, F, tcap, kcap;
  size_t offset, bytes;
};

static PartSplit part_split(int F, int tcap, int kcap, int n, int j) {
  PartSplit q;
  size_t off = 0;
  for (int k = 0; k <= j; ++k) {
    q.first = (int)((int64_t)F * k / n);
    q.F = (int)((int64_t)F * (k + 1) / n) - q.first;
    q.tcap = (int)((int64_t)tcap * (k + 1) / n - (int64_t)tcap * k / n);
    q.kcap = (int)((int64_t)kcap * (k + 1) / n - (int64_t)kcap * k / n);
    q.offset = off;
    q.bytes = align256(layout(q.F, q.tcap, q.kcap).total);
    off += q.bytes;
  }
  return q;
}

static size_t plan_bytes(int F, int tcap, int kcap, int n) {
  const PartSplit q = part_split(F, tcap, kcap, n, n - 1);
  return n == 1 ? layout(F, tcap, kcap).total : q.offset + q.bytes;
}

// The batched sequence of one part: stage 0 clears the counters and runs
// the persistent cuts (and fits); stage 1 the fits left to k_tracks, the
// float64 re-evaluation and the vertex stage.  ev (nullable, 4 events):
// before and after the persistent kernel, after k_tracks, at the end.
static void part_launch(const mu3e_plan& pl, const PlanPart& q, int stage, hipStream_t s, hipEvent_t* ev) {
  const mu3e_hits_t& h = q.hits;
  if (stage == 0) {
    hipLaunchKernelGGL(k_init, dim3(kClaimRanges), dim3(256), 0, s, q.W.counters, q.T.pre * q.T.chunk, q.W.claims);
    if (q.F == 0) return;
    if (ev) (void)hipEventRecord(ev[0], s);
    const TrackOut O = track_out(q.W, q.flags, q.counts);
    hipLaunchKernelGGL(batched_kernel(pl.tuning.fuse_fits != 0, pl.tuning.tile_hits), dim3(q.P), dim3(kWave), 0, s,
                       h.x, h.y, h.z, h.layer_offsets, q.F, q.Fs, h.n_hits, pl.C, q.flags, q.counts, q.vertex,
                       q.W.ccnt, q.T, O, q.W.counters, q.W.claims, pl.tuning.frames_per_claim, q.W.defer);
    launch_tiles(h, pl.C, pl.cus, pl.tuning.tile_hits, q.W, q.T, q.flags, q.counts, s);
    if (ev) (void)hipEventRecord(ev[1], s);
    return;
  }
  if (q.F == 0) return;
  // fits left by the persistent kernel (all of them without fusion)
  launch_tracks(h, pl.C, pl.cus, q.W, q.T, q.flags, q.counts, s, ev ? ev[2] : nullptr);
  launch_vertex(h, pl.C, q.F, pl.cus, q.W, q.T, q.flags, q.counts, q.vertex, q.kcap, s, nullptr);
  if (ev) (void)hipEventRecord(ev[3], s);
}

static void plan_free(mu3e_plan* pl) {
  for (int j = 0; j < kMaxParts; ++j) {
    for (int g = 0; g < 2; ++g) {
      if (pl->part[j].exec[g]) (void)hipGraphExecDestroy(pl->part[j].exec[g]);
      if (pl->part[j].graph[g]) (void)hipGraphDestroy(pl->part[j].graph[g]);
    }
    if (pl->side[j]) (void)hipStreamDestroy(pl->side[j]);
    if (pl->cuts_done[j]) (void)hipEventDestroy(pl->cuts_done[j]);
    if (pl->part_done[j]) (void)hipEventDestroy(pl->part_done[j]);
  }
  delete pl;
}

size_t mu3e_plan_workspace_size(int32_t n_frames, int32_t triplet_capacity, int32_t track_capacity,
                                int32_t sub_batches) {
  if (n_frames < 0 || triplet_capacity < 0 || triplet_capacity > kMaxTripletCapacity || track_capacity < 0 ||
      sub_batches < 0 || sub_batches > kMaxParts)
    return 0;
  return plan_bytes(n_frames, triplet_capacity, track_capacity, sub_batches > 0 ? sub_batches : 1);
}

mu3e_status mu3e_plan_create(mu3e_plan_t** out, const mu3e_hits_t* hits, const mu3e_params_t* params,
                             uint32_t* frame_flags, int32_t* frame_counts, float* frame_vertex, void* workspace,
                             size_t workspace_bytes, int32_t triplet_capacity, int32_t track_capacity,
                             const mu3e_tuning_t* tuning) {
  if (!out || !hits_ok(hits) || !params || triplet_capacity < 0 || triplet_capacity > kMaxTripletCapacity ||
      track_capacity < 0)
    return MU3E_ERR_INVALID_ARG;
  *out = nullptr;
  Consts C;
  if (!make_consts(params, C)) return MU3E_ERR_INVALID_ARG;
  if (C.max_lh > kMaxTiledLayerHits) return MU3E_ERR_UNSUPPORTED;
  mu3e_tuning_t t;
  t.waves_per_cu = tuning && tuning->waves_per_cu > 0 ? tuning->waves_per_cu : 16;
  t.frames_per_claim = tuning && tuning->frames_per_claim > 0 ? tuning->frames_per_claim : 4;
  t.fuse_fits = tuning ? (tuning->fuse_fits != 0) : 0;
  t.steal_percent = tuning ? tuning->steal_percent : 0;
  t.tile_hits = tuning && tuning->tile_hits > 0 ? tuning->tile_hits : kPlainTile;
  t.sub_batches = tuning && tuning->sub_batches > 0 ? tuning->sub_batches : 1;
  if (t.steal_percent < 0 || t.steal_percent > 100 || (t.tile_hits != 64 && t.tile_hits != 128) ||
      t.sub_batches > kMaxParts)
    return MU3E_ERR_INVALID_ARG;
  const int F = hits->n_frames;
  if (t.sub_batches > F) t.sub_batches = F > 0 ? F : 1;
  const int n = t.sub_batches;
  if (!workspace || workspace_bytes < plan_bytes(F, triplet_capacity, track_capacity, n)) return MU3E_ERR_CAPACITY;
  if (F > 0 && (!frame_flags || !frame_counts || !frame_vertex)) return MU3E_ERR_INVALID_ARG;
  const int cus = device_cus();
  // persistent: never more waves than can be resident at once
  int resident = 0;
  const hipError_t oe =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, batched_kernel(t.fuse_fits != 0, t.tile_hits), kWave, 0);
  if (oe != hipSuccess) return MU3E_ERR_HIP;
  if (resident > 0 && t.waves_per_cu > resident) t.waves_per_cu = resident;
  mu3e_plan* pl = new (std::nothrow) mu3e_plan();
  if (!pl) return MU3E_ERR_CAPACITY;
  pl->tuning = t;
  pl->C = C;
  pl->cus = cus;
  pl->nparts = n;
  bool ok = true;
  for (int j = 0; j < n && ok; ++j) {
    const PartSplit sp = part_split(F, triplet_capacity, track_capacity, n, j);
    PlanPart& q = pl->part[j];
    q.hits = *hits;
    q.hits.n_frames = sp.F;
    if (F > 0) q.hits.layer_offsets = hits->layer_offsets + 4 * (size_t)sp.first;
    const Layout L = layout(sp.F, sp.tcap, sp.kcap);
    q.W = ws_view(static_cast<char*>(workspace) + sp.offset, L, sp.kcap);
    q.flags = frame_flags ? frame_flags + sp.first : nullptr;
    q.counts = frame_counts ? frame_counts + 3 * (size_t)sp.first : nullptr;
    q.vertex = frame_vertex ? frame_vertex + 4 * (size_t)sp.first : nullptr;
    q.first = sp.first;
    q.F = sp.F;
    q.kcap = sp.kcap;
    q.P = cus * t.waves_per_cu;
    if (q.P > q.F) q.P = q.F > 0 ? q.F : 1;
    q.T = trip_list(q.W, sp.tcap, q.P);
    q.Fs = q.F - (int)((int64_t)q.F * t.steal_percent / 100);
    q.dbg.counters = q.W.counters; q.dbg.triplets = q.W.trips; q.dbg.tracks = q.W.res;
    q.dbg.triplet_capacity = sp.tcap; q.dbg.track_capacity = sp.kcap;
    q.dbg.chunks = q.W.chunks; q.dbg.max_chunks = sp.tcap / kMinChunk + 1; q.dbg.chunk_size = q.T.chunk;
    if (j > 0) ok = hipStreamCreateWithFlags(&pl->side[j], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&pl->cuts_done[j], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&pl->part_done[j], hipEventDisableTiming) == hipSuccess;
    for (int g = 0; g < 2 && ok; ++g) {
      if (g == 1 && q.F == 0) break;   // nothing after the counters are cleared
      hipStream_t cs;
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { ok = false; break; }
      ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        part_launch(*pl, q, g, cs, nullptr);
        ok = hipStreamEndCapture(cs, &q.graph[g]) == hipSuccess;
      }
      ok = ok && hipGraphInstantiate(&q.exec[g], q.graph[g], nullptr, nullptr, 0) == hipSuccess;
      (void)hipStreamDestroy(cs);
    }
  }
  if (!ok) { plan_free(pl); return MU3E_ERR_HIP; }
  *out = pl;
  return MU3E_OK;
}

// Part 0 runs on the caller's stream, part j > 0 on the plan's stream j;
// the cuts of part j start when those of part j - 1 are done (they need the
// whole GPU), the rest of each part follows its cuts on its stream and
// overlaps the next part's cuts; the caller's stream waits for every part.
mu3e_status mu3e_plan_run(mu3e_plan_t* plan, hipStream_t stream) {
  if (!plan) return MU3E_ERR_INVALID_ARG;
  bool ok = true;
  for (int j = 0; j < plan->nparts && ok; ++j) {
    PlanPart& q = plan->part[j];
    hipStream_t s = j == 0 ? stream : plan->side[j];
    if (j > 0) ok = hipStreamWaitEvent(s, plan->cuts_done[j - 1], 0) == hipSuccess;
    ok = ok && hipGraphLaunch(q.exec[0], s) == hipSuccess;
    if (plan->nparts > 1) ok = ok && hipEventRecord(plan->cuts_done[j], s) == hipSuccess;
    if (q.exec[1]) ok = ok && hipGraphLaunch(q.exec[1], s) == hipSuccess;
    if (j > 0) ok = ok && hipEventRecord(plan->part_done[j], s) == hipSuccess;
  }
  for (int j = 1; j < plan->nparts && ok; ++j) ok = hipStreamWaitEvent(stream, plan->part_done[j], 0) == hipSuccess;
  return ok ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_plan_run_timed(mu3e_plan_t* plan, hipStream_t stream, hipEvent_t* events) {
  if (!plan || !events) return MU3E_ERR_INVALID_ARG;
  for (int k = 0; k < 4 * plan->nparts; ++k)
    if (!events[k]) return MU3E_ERR_INVALID_ARG;
  for (int j = 0; j < plan->nparts; ++j) {
    part_launch(*plan, plan->part[j], 0, stream, events + 4 * j);
    part_launch(*plan, plan->part[j], 1, stream, events + 4 * j);
  }
  return hipGetLastError() == hipSuccess ? MU3E_OK : MU3E_ERR_HIP;
}

mu3e_status mu3e_plan_info(const mu3e_plan_t* plan, mu3e_debug_t* dbg, mu3e_tuning_t* tuning) {
  if (!plan) return MU3E_ERR_INVALID_ARG;
  if (dbg) *dbg = plan->part[0].dbg;
  if (tuning) *tuning = plan->tuning;
  return MU3E_OK;
}

mu3e_status mu3e_plan_part_info(const mu3e_plan_t* plan, int32_t part, mu3e_debug_t* dbg, int32_t* first_frame,
                                int32_t* n_frames) {
  if (!plan || part < 0 || part >= plan->nparts) return MU3E_ERR_INVALID_ARG;
  if (dbg) *dbg = plan->part[part].dbg;
  if (first_frame) *first_frame = plan->part[part].first;
  if (n_frames) *n_frames = plan->part[part].F;
  return MU3E_OK;
}

void mu3e_plan_destroy(mu3e_plan_t* plan) {
  if (!plan) return;
  plan_free(plan);
}

}  // extern "C"
