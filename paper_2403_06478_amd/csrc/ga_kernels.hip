// ga_kernels.hip -- MI355X (gfx950) guided extension aligner: device code and
// the C ABI declared in include/ga.h.
//
// Method: AGAThA (PPoPP'24, arXiv 2403.06478), Section 2.1 -- banded
// two-piece affine-gap score table (Eq. 1-3) with per-anti-diagonal maximum
// tracking and the z-drop termination test (Eq. 4-7).
//
// Kernel shape (differs from the paper's chunked row sweep, Sections 4.1-4.2):
// one wave64 per pair (up to 2048 band diagonals; wider bands take 2-4 waves
// of one workgroup) sweeps the band anti-diagonal by anti-diagonal. Lane l
// owns K consecutive diagonals d = i - j of the band (slots), kept entirely in
// VGPRs. Cells of anti-diagonal r lie on diagonals d == r (mod 2), so a step
// updates one parity class of slots from the other class, which holds
// anti-diagonal r-1; the slot's own previous value is anti-diagonal r-2 (the
// diagonal predecessor). Within a lane the up/left neighbours are the adjacent
// slots; at lane edges they arrive by DPP wave_shr:1 / wave_shl:1. Every step
// completes a whole anti-diagonal, so the local maximum of Eq. 6 is one wave
// reduction and the z-drop test of Eq. 5 runs in order with no run-ahead: the
// rolling window of partial maxima (Section 4.1) and the slice boundary
// (Section 4.2) are not needed. With several waves per pair, neighbouring
// waves share two ghost diagonals per edge and swap their edge slots and
// their maxima through LDS once per two anti-diagonals, around one
// workgroup barrier.
//
// Boundary cells (row -1 and column -1) are produced by the same recurrence:
// the slots outside the rectangle start at -inf and the origin at 0, so the
// first cells reached on each diagonal are exactly the boundary gap scores.
// The band edges are walls of -inf: the left wall is the DPP fill value of
// lane 0, the right wall is a slot forced to -inf after each update.
//
// Bases stay 2-bit packed in HBM (plus the N bitmap). Each wave stages the
// bases its band covers in two LDS rings (target and query), one byte per
// base (0..3, N = 4), refilled by its lanes 64 words (256 bases) at a time
// whenever the next block's windows reach past what a ring holds. Per 8-step
// block each lane reads its byte windows from the rings (a block ahead) and
// each slot builds the substitution scores of its next 4 cells with one
// v_perm_b32 table lookup (4 signed bytes); each cell adds its byte through
// an SDWA operand.
//
// The one-wave 24-slot class runs the start and end triangles of its band,
// where an anti-diagonal's finite cells span at most 1024 diagonals, with
// 16 slots per lane on a window placed over them, and moves the state
// between the two slot layouts through LDS (align_pair_split).

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <type_traits>

#include "ga.h"

namespace {

constexpr int NEG = -(1 << 30);                  // -inf sentinel; range guard keeps it apart
constexpr int NEG_MAX = -(1 << 30) - (1 << 29);  // below every reachable value
// Every finite score in the frame lies above LIVE_MIN (the range guard keeps
// them within +-2^29); -inf values, even after their drift, lie below it.
constexpr int LIVE_MIN = -(1 << 29) - (1 << 27);
constexpr int WAVE = 64;

// Slot classes: K slots per lane and NW waves per pair hold the band's
// D <= class_cap diagonals (64*K on one wave, less 4 per extra wave for the
// shared ghost diagonals); a pair goes to the first class that holds it.
constexpr int NCLASS = 15;
// (K, NW, window) = (4,1,fixed) (8,1,fixed) (16,1,fixed) (24,1,fixed)
// (32,1,fixed) (8,1,sliding) (16,1,sliding) (24,2,fixed) (32,2,fixed)
// (32,3,fixed) (32,4,fixed) (4,1,sliding) (8,2,fixed) (4,2,fixed)
// (4,4,fixed). The last three spread a band a one-wave class holds over
// more waves: slower per pair at full occupancy (a barrier every two
// anti-diagonals), but each wave's step is shorter, so a batch too small
// to fill the GPU, whose time is its longest sweep, ends sooner.
__host__ __device__ constexpr int class_k(int c) {
    return (c == 0 || c == 11 || c == 13 || c == 14) ? 4
           : (c == 1 || c == 5 || c == 12)         ? 8
           : (c == 2 || c == 6)                     ? 16
           : (c == 3 || c == 7)                     ? 24
                                                    : 32;
}
__host__ __device__ constexpr int class_nw(int c) {
    return c < 7 || c == 11 ? 1 : c < 9 || c == 12 || c == 13 ? 2 : c == 9 ? 3 : 4;
}
__host__ __device__ constexpr bool class_slides(int c) { return c == 5 || c == 6 || c == 11; }
// Neighbouring waves of one pair overlap by 2*HALO diagonals: each holds
// copies ("ghosts") of the HALO diagonals next to its edge, refreshed from
// their owner every HALO anti-diagonals, so the waves exchange state and
// meet at a barrier only every HALO anti-diagonals.
constexpr int HALO = 2;
__host__ __device__ constexpr int wave_stride(int K) { return WAVE * K - 2 * HALO; }
__host__ __device__ constexpr int class_cap(int c) {
    return WAVE * class_k(c) + (class_nw(c) - 1) * wave_stride(class_k(c));
}
constexpr int MAX_DIAGONALS = WAVE * 32 + 3 * wave_stride(32);

constexpr uint32_t ALL_CLASSES = (1u << NCLASS) - 1;

// Slots per lane of the start and end triangles of the one-wave 24- and
// 16-slot classes (0: the whole sweep with one layout); see
// align_pair_split.
constexpr int TRI_K24 = 16;
constexpr int TRI_K16 = 8;

// The class a pair runs in, and whether its one wave slides along the band
// (*slide = -1 down, +1 up, 0 fixed). A band of D diagonals fits class c when
// D <= class_cap(c). When one sequence is short, an anti-diagonal's cells from the
// boundary cell to the cell just past the short sequence's end span at most
// 2*min(n,m) + 3 diagonals; a single wave whose window follows them (moved
// one lane at a time, hence the K of slack) runs such a pair even when the
// whole band would not fit. `mask` restricts the classes considered; a class
// is then taken only in the shape the cheapest-first rule gives it: a
// sliding class only for a band wider than its window, a class of NW waves
// only for a band that reaches its last wave.
// The classes in the order they are tried: cheapest first, four bits per
// class from the lowest nibble. The default is by slots per lane (4,
// sliding 4, 8, sliding 8, 16, sliding 16, 24, 32), then the multi-wave
// classes; an autotuned context replaces it with its measured order.
constexpr uint64_t DEFAULT_ORDER = 0x0ull | (11ull << 4) | (1ull << 8) | (5ull << 12) | (2ull << 16) |
                                   (6ull << 20) | (3ull << 24) | (4ull << 28) | (7ull << 32) |
                                   (8ull << 36) | (9ull << 40) | (10ull << 44) | (13ull << 48) |
                                   (12ull << 52) | (14ull << 56);

__host__ __device__ inline int class_for(int64_t n, int64_t m, int64_t w, int *slide,
                                         uint32_t mask = ALL_CLASSES, uint64_t order = DEFAULT_ORDER) {
    int64_t a0, a1;
    if (w >= 0) {
        a0 = -w > -m ? -w : -m;
        a1 = w < n ? w : n;
    } else {
        a0 = -m;
        a1 = n;
    }
    const int64_t D = a1 - a0 + 1;
    const int64_t span = 2 * (n < m ? n : m) + 11;
    *slide = 0;
    for (int k = 0; k < NCLASS; ++k) {
        const int c = (int)((order >> (4 * k)) & 0xFull);
        if (!((mask >> c) & 1u)) continue;
        if (!class_slides(c)) {
            const int K = class_k(c), NW = class_nw(c);
            const int64_t below = NW > 1 ? WAVE * K + (NW - 2) * wave_stride(K) : 0;  // NW-1 waves' reach
            if (D <= class_cap(c) && D > below) return c;
        } else if (D > class_cap(c) && span + class_k(c) <= class_cap(c)) {
            *slide = n <= m ? -1 : 1;
            return c;
        }
    }
    return -1;
}

// The classes the pairs of a batch (lengths up to max_len, band w) can take
// under `mask` and `order`, as a bit mask. A pair's band spans at most
// Dmax = 2 min(w, max_len) + 1 diagonals. A sliding class only takes bands
// wider than its window, so it is out when Dmax fits the window. A fixed or
// multi-wave class takes the band widths D it holds (up to its capacity,
// above its one-wave-fewer reach) that no class before it in the order
// holds; the holder of D is piecewise constant in D with breaks only where
// a class's range starts or ends, so trying D = 1 and every range end + 1
// up to Dmax finds every class some width picks (a sliding class taking a
// width first can only make this an over-estimate). Host function: the
// persistent schedule skips the launches no pair can reach.
inline uint32_t reachable_classes(int64_t max_len, int64_t w, uint32_t mask, uint64_t order) {
    const int64_t half = w >= 0 && w < max_len ? w : max_len;
    const int64_t Dmax = 2 * half + 1;
    uint32_t out = 0;
    int64_t probe[2 * NCLASS + 1];
    int np = 0;
    probe[np++] = 1;
    for (int c = 0; c < NCLASS; ++c) {
        if (!((mask >> c) & 1u)) continue;
        if (class_slides(c)) {
            if (Dmax > class_cap(c)) out |= 1u << c;
            continue;
        }
        const int K = class_k(c), NW = class_nw(c);
        const int64_t below = NW > 1 ? WAVE * K + (NW - 2) * wave_stride(K) : 0;
        if (below + 1 <= Dmax) probe[np++] = below + 1;
        if (class_cap(c) + 1 <= Dmax) probe[np++] = class_cap(c) + 1;
    }
    for (int t = 0; t < np; ++t) {
        const int64_t D = probe[t];
        for (int k = 0; k < NCLASS; ++k) {
            const int c = (int)((order >> (4 * k)) & 0xFull);
            if (!((mask >> c) & 1u) || class_slides(c)) continue;
            const int K = class_k(c), NW = class_nw(c);
            const int64_t below = NW > 1 ? WAVE * K + (NW - 2) * wave_stride(K) : 0;
            if (D <= class_cap(c) && D > below) {
                out |= 1u << c;
                break;
            }
        }
    }
    return out;
}

// Work groups of one call: the kernel classes (persistent schedule) or the
// power-of-two length buckets (bucketed schedule). Device counters per call:
// [0..32) group list sizes, [32..64) group heads, [64..96) group list starts
// in the one pair list. They sit right before the planning histogram.
constexpr int NGROUP = 32;
constexpr int CNT_COUNT = 0;
constexpr int CNT_HEAD = NGROUP;
constexpr int CNT_START = 2 * NGROUP;
constexpr int CNT_WORDS = 3 * NGROUP;

// The fixed class a power-of-two length bucket b (max(n, m) < 2^b) runs in
// under the bucketed schedule: the first fixed class holding the band of two
// sequences of length 2^b - 1 (-1 if none).
__host__ __device__ inline int bucket_class(int b, int64_t w, uint32_t mask = ALL_CLASSES) {
    const int64_t L = ((int64_t)1 << b) - 1;
    const int64_t half = w >= 0 && w < L ? w : L;
    const int64_t D = 2 * half + 1;
    for (int c = 0; c < NCLASS; ++c)
        if (((mask >> c) & 1u) && !class_slides(c) && D <= class_cap(c)) return c;
    return -1;
}

// Scores are held in a frame that drifts by the piece-1 extension e per
// anti-diagonal: a value V of a cell on anti-diagonal r is stored as
// V + e*r. Then extending a piece-1 gap by one cell costs nothing, and the
// other terms become constants:
//   E1 = max(A_up, E_up)            F1 = max(A_left, F_left)
//   E2 = max(A_up - c2, X_up)       F2 = max(A_left - c2, Y_left)
//   H  = max(A_diag + s', E1, E2, F1, F2)
// with A = H - q, X = E2 - d2, Y = F2 - d2, c2 = (q2+e2) - (q+e), d2 = e2 - e,
// and s' = S + q + 2e (the substitution score with the frame's two-step
// drift folded in; it is what the byte table holds).
struct DpArgs {
    const uint32_t *tw;  // target 2-bit stream; base k of pair p: word t_off[p] + k/16
    const uint32_t *qw;  // query 2-bit stream
    const uint32_t *tn;  // N bitmaps (one bit per base position of the stream), or null
    const uint32_t *qn;
    const int64_t *t_off;
    const int64_t *q_off;
    const int32_t *t_len;
    const int32_t *q_len;
    const int32_t *list;  // the pair list of all groups
    int32_t *counters;
    ga_result_t *out;
    int32_t group;        // this launch's work group
    int32_t w, Z;
    int32_t q1, c2, d2, e1, e2;
    int32_t oe1, oe2;
    // frame value of the boundary cells (-1, r+1), (r+1, -1) of
    // anti-diagonal r (H = -gamma(r+2)): max(ring_a0, ring_b0 + r * ring_d)
    int32_t ring_a0, ring_b0, ring_d;
    uint32_t lut_lo, lut_hi;  // s' per class byte (signed bytes)
};

__device__ __forceinline__ int dpp_from_lower_lane(int fill, int v) {
    // lane l receives lane l-1's v; lane 0 receives `fill` (wave_shr:1)
    return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ int dpp_from_upper_lane(int fill, int v) {
    // lane l receives lane l+1's v; lane 63 receives `fill` (wave_shl:1)
    return __builtin_amdgcn_update_dpp(fill, v, 0x130, 0xf, 0xf, false);
}

// Max over the 64 lanes, returned as a wave-uniform value. The shifted
// operand's fill is INT_MIN, the identity of max, so every step folds into
// one v_max_i32_dpp (rows outside a row_bcast mask keep their value).
__device__ __forceinline__ int wave_max(int v) {
    constexpr int ID = -2147483647 - 1;
    v = max(v, __builtin_amdgcn_update_dpp(ID, v, 0xB1, 0xf, 0xf, false));   // quad_perm 1,0,3,2
    v = max(v, __builtin_amdgcn_update_dpp(ID, v, 0x4E, 0xf, 0xf, false));   // quad_perm 2,3,0,1
    v = max(v, __builtin_amdgcn_update_dpp(ID, v, 0x141, 0xf, 0xf, false));  // row_half_mirror
    v = max(v, __builtin_amdgcn_update_dpp(ID, v, 0x140, 0xf, 0xf, false));  // row_mirror
    v = max(v, __builtin_amdgcn_update_dpp(ID, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(ID, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// (bit `lane` of the wave-uniform mask) ? if1 : if0, one VALU instruction.
__device__ __forceinline__ int select_by_lanes(uint64_t mask, int if1, int if0) {
    int r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if0), "v"(if1), "s"(mask));
    return r;
}

__device__ __forceinline__ uint64_t lanes_from(int x) {  // lanes >= x
    return x <= 0 ? ~0ull : (x >= 64 ? 0ull : (~0ull << x));
}

__device__ __forceinline__ uint64_t lanes_upto(int x) {  // lanes <= x
    return x < 0 ? 0ull : (x >= 63 ? ~0ull : (~0ull >> (63 - x)));
}

__device__ __forceinline__ uint32_t window4(const uint32_t *W, int o) {
    // bytes o..o+3 of the little-endian byte array held in W (o compile-time)
    return (o & 3) ? __builtin_amdgcn_alignbyte(W[(o >> 2) + 1], W[o >> 2], (uint32_t)(o & 3))
                   : W[o >> 2];
}

template <int K>
struct PairState {
    // Register vectors, so a slot at a wave-uniform position (the band wall,
    // a cell leaving the rectangle) can be indexed without leaving registers
    // (s_set_gpr_idx from 16 slots up, a select per slot below that).
    typedef int VecK __attribute__((ext_vector_type(K)));
    VecK A, E, X, F, Y;
    uint32_t S4[K];  // s' of the slot's next 4 cells, one signed byte each
    // the lane-edge neighbours: A, E, X of the lower lane's slot K-1 and
    // A, F, Y of the upper lane's slot 0, received by DPP each step into
    // the same registers. Lane 0 of the first three and lane 63 of the
    // others have no neighbour and keep -inf from the pair's start: a DPP
    // move leaves such a lane's old value, so no fill precedes it.
    int eA, eE, eX, fA, fF, fY;
};

// One slot update (class C slot S, block cell KC). Inputs come from the
// other class (anti-diagonal r-1) and the slot's own A (anti-diagonal r-2).
template <int K, int S, int KC>
__device__ __forceinline__ void update_slot(PairState<K> &st, const DpArgs &P, const int (&B)[K],
                                            int ae, int be, int ee, int xe, int af, int bf, int ff,
                                            int yf) {
    const int au = (S == 0) ? ae : st.A[S == 0 ? 0 : S - 1];
    const int bu = (S == 0) ? be : B[S == 0 ? 0 : S - 1];
    const int eu = (S == 0) ? ee : st.E[S == 0 ? 0 : S - 1];
    const int xu = (S == 0) ? xe : st.X[S == 0 ? 0 : S - 1];
    const int al = (S == K - 1) ? af : st.A[S == K - 1 ? 0 : S + 1];
    const int bl = (S == K - 1) ? bf : B[S == K - 1 ? 0 : S + 1];
    const int fl = (S == K - 1) ? ff : st.F[S == K - 1 ? 0 : S + 1];
    const int yl = (S == K - 1) ? yf : st.Y[S == K - 1 ? 0 : S + 1];
    const int e1 = max(au, eu);
    const int e2 = max(bu, xu);
    const int f1 = max(al, fl);
    const int f2 = max(bl, yl);
    const int hd = st.A[S] + __builtin_amdgcn_sbfe((int)st.S4[S], 8 * KC, 8);
    const int h = max(max(max(max(hd, e1), e2), f1), f2);  // two v_max3
    st.A[S] = h - P.q1;
    st.E[S] = e1;
    st.X[S] = e2 - P.d2;
    st.F[S] = f1;
    st.Y[S] = f2 - P.d2;
}

// Slots S, S+2, ... of one parity class (static unroll).
template <int K, int KC, int S>
__device__ __forceinline__ void update_class(PairState<K> &st, const DpArgs &P, const int (&B)[K],
                                             int ae, int be, int ee, int xe, int af, int bf, int ff,
                                             int yf) {
    if constexpr (S < K) {
        update_slot<K, S, KC>(st, P, B, ae, be, ee, xe, af, bf, ff, yf);
        update_class<K, KC, S + 2>(st, P, B, ae, be, ee, xe, af, bf, ff, yf);
    }
}

// Update the slots of parity class C with cell index KC (0..3) of the block.
// Beyond the wave's outer lanes (lane 0's lower neighbour for class 0,
// lane 63's upper one for class 1) the values are -inf: the band edge, or
// in a multi-wave pair the next wave's edge, which the ghost diagonals
// stand in for.
template <int K, int C, int KC, bool EDGE_REGS = true>
__device__ __forceinline__ void dp_step(PairState<K> &st, const DpArgs &P) {
    int ae = 0, ee = 0, xe = 0;  // class 0: slot -1 = lower lane's slot K-1 (up)
    int af = 0, ff = 0, yf = 0;  // class 1: slot K = upper lane's slot 0 (left)
    if constexpr (!EDGE_REGS) {
        // (one wave of 32 slots: no registers to spare for the six edge
        // registers; a -inf fill per move instead)
        if (C == 0) {
            ae = dpp_from_lower_lane(NEG, st.A[K - 1]);
            ee = dpp_from_lower_lane(NEG, st.E[K - 1]);
            xe = dpp_from_lower_lane(NEG, st.X[K - 1]);
        } else {
            af = dpp_from_upper_lane(NEG, st.A[0]);
            ff = dpp_from_upper_lane(NEG, st.F[0]);
            yf = dpp_from_upper_lane(NEG, st.Y[0]);
        }
    } else if (C == 0) {
        ae = st.eA = dpp_from_lower_lane(st.eA, st.A[K - 1]);
        ee = st.eE = dpp_from_lower_lane(st.eE, st.E[K - 1]);
        xe = st.eX = dpp_from_lower_lane(st.eX, st.X[K - 1]);
    } else {
        af = st.fA = dpp_from_upper_lane(st.fA, st.A[0]);
        ff = st.fF = dpp_from_upper_lane(st.fF, st.F[0]);
        yf = st.fY = dpp_from_upper_lane(st.fY, st.Y[0]);
    }
    // piece-2 openings of the other class, shared by both neighbours
    int B[K];
#pragma unroll
    for (int s = 0; s < K; ++s) B[s] = ((s & 1) != C) ? st.A[s] - P.c2 : 0;
    const int be = ae - P.c2, bf = af - P.c2;
    update_class<K, KC, C>(st, P, B, ae, be, ee, xe, af, bf, ff, yf);
}

// Force slot `sl` of the one lane in `hit` to -inf in the arrays a clamp
// kills: A always, E and X (the values read from above) or F and Y (read
// from the left). The slot always belongs to class C, the class just
// updated (its diagonal has the parity of the anti-diagonal), so with few
// slots the write is a select over the class's K/2 slots per array; from
// 16 slots up an indexed register write (s_set_gpr_idx) is cheaper.
template <int K, int C, bool EX>
__device__ __forceinline__ void kill_slot(PairState<K> &st, bool hit, int sl) {
    if constexpr (K <= 8) {
        const int t = sl >> 1;  // sl = C + 2t
#pragma unroll
        for (int u = 0; u < K / 2; ++u) {
            if (hit && u == t) {
                st.A[C + 2 * u] = NEG;
                if (EX) {
                    st.E[C + 2 * u] = NEG;
                    st.X[C + 2 * u] = NEG;
                } else {
                    st.F[C + 2 * u] = NEG;
                    st.Y[C + 2 * u] = NEG;
                }
            }
        }
    } else if (hit) {  // one lane: indexed register writes under its exec mask
        st.A[sl] = NEG;
        if (EX) {
            st.E[sl] = NEG;
            st.X[sl] = NEG;
        } else {
            st.F[sl] = NEG;
            st.Y[sl] = NEG;
        }
    }
}

// The band's right wall is the first diagonal past the band: slot
// `wall_pos` of the lane flagged in `wall_lanes` (a slot of class C). After
// each update of its class it is forced back to -inf there; its A, E and X
// are all it feeds forward, so the dead slots beyond it never leave -inf
// either and nothing crosses the band edge.
template <int K, int C>
__device__ __forceinline__ void clamp_wall(PairState<K> &st, uint64_t wall_lanes, int wall_pos) {
    const bool wl = __builtin_amdgcn_inverse_ballot_w64(wall_lanes);
    kill_slot<K, C, true>(st, wl, __builtin_amdgcn_readfirstlane(wall_pos));
}

// A cell that has just left the rectangle (the slot at array position p of
// class C, just updated): it feeds only cells outside the rectangle, so it
// is forced to -inf with the values its successors read -- A, E, X when it
// is past the target end (i = n: read from above), A, F, Y when it is past
// the query end (j = m: read from the left). Its successors then stay -inf,
// and the lane maxima need no mask for them.
template <int K, int C, bool PAST_T>
__device__ __forceinline__ void clamp_cell(PairState<K> &st, int p) {
    const int pl = __builtin_amdgcn_readfirstlane(p);
    if constexpr (K == 4 || K == 8) {
        // 0 <= p < 64K: shift and mask (with K >= 16 the slot index feeds
        // an indexed register write, which the signed form keeps in
        // registers)
        const unsigned pu = (unsigned)pl;
        const bool hit = __builtin_amdgcn_inverse_ballot_w64(1ull << (pu / K));
        kill_slot<K, C, PAST_T>(st, hit, (int)(pu % K));
    } else {
        const bool hit = __builtin_amdgcn_inverse_ballot_w64(1ull << (pl / K));
        kill_slot<K, C, PAST_T>(st, hit, pl % K);
    }
}

// Geometry of one pair (all wave-uniform).
struct Geo {
    int n, m;
    int a0;        // lowest diagonal held (band edge, or -m: the boundary row)
    int a0w;       // the first diagonal of this wave's slots (a0 for wave 0)
    int dlo, dhi;  // diagonals with interior cells
    int r_last;    // last non-empty anti-diagonal
    int a1;        // highest band diagonal
};

struct Track {
    int G, gi, gj;        // global maximum (Eq. 7); gi/gj valid once resolved
    int endS, endI, endJ; // local maximum where the sweep ended
    int zd;
    // where G was taken, kept lazily: the anti-diagonal, the wave holding
    // the cell and the frame value; the holding wave parks that
    // anti-diagonal's class values in LDS until the cell is needed
    int g_r, g_base, g_ma;  // g_base: diagonal of lane 0's slot 0 in the holding wave (several waves)
    bool g_open;  // G moved since its cell was last resolved
    bool g_set;   // G has moved off the origin
    // one wave per pair: G in the score frame of the anti-diagonal being
    // decided (advanced by e per anti-diagonal), so the decisions compare
    // frame values and never convert back to scores; G itself is
    // g_ma + q - e * g_r (g_r = -1 and g_ma the frame value of 0 on
    // anti-diagonal -1 while G is at the origin)
    int gf;
    int g_res;  // one wave per pair: g_r when G's cell was last resolved
};

// LDS of one pair's workgroup: the park of the wave holding the global
// maximum (slot-major, so 64 lanes write 64 consecutive words), and with
// several waves per pair the exchange every two anti-diagonals, double
// buffered: the owned edge diagonals each wave hands its neighbours' ghosts
// and each wave's maxima.
// Base staging rings of one wave (one per sequence): the byte of base
// position x sits at ring[x mod BYTES]. A block's windows span at most
// 32K + 16 positions of each sequence (every lane's K/2 + 4 bases, aligned
// to words); the ring is refilled 64 words (256 bases) at a time, one word
// per lane, whenever the next block's windows reach past what it holds, so
// it also holds a refill's worth beyond the windows. A lane reads its window
// as K/8 + 3 words from one ring offset; the ring's first MIRROR words are
// copied past its end, so such a read never wraps.
template <int K>
struct Ring {
    static constexpr int BYTES = K <= 4 ? 512 : K <= 16 ? 1024 : 2048;
    static constexpr int WORDS = BYTES / 4;
    static constexpr int MIRROR = K / 8 + 2;
    static_assert(WORDS >= 8 * K + 4 + WAVE, "a block's windows and one refill must fit the ring");
};

// One sequence's bases in HBM: its first 2-bit word, the stream's N bitmap
// (or null) and the bit of its first base there, its length.
struct SeqSource {
    const uint32_t *words;
    const uint32_t *nmask;
    int64_t nbit0;
    int64_t len;
};

template <int K, int NW>
struct PairLds {
    int park[K * WAVE];  // park[s * 64 + lane] = A of slot s
    // each wave's staged bases: [wave][0 target, 1 query], and where they
    // come from (read only when a ring is refilled, so the sweep keeps no
    // registers for them)
    uint32_t ring[NW][2][Ring<K>::WORDS + Ring<K>::MIRROR];
    SeqSource src[NW][2];
    // several waves (double-buffered by exchange): the owned edge diagonals
    // a wave hands its neighbours (A, E, X, F, Y of two slots each way) and
    // the wave maxima of the exchange's two anti-diagonals
    int up[2][NW][2][5];
    int dn[2][NW][2][5];
    int ma[2][NW][2];
    int ma2[NW];         // wave maxima of an anti-diagonal redone with masks
    int flag;            // a rare decision's outcome, for every wave
    int idx;             // pair index handed to every wave
};

// Interior diagonals of anti-diagonal r, clipped to its parity.
__device__ __forceinline__ void diag_window(const Geo &g, int r, int &vlo, int &vhi) {
    vlo = max(g.dlo, max(-r, r - 2 * g.m + 2));
    vhi = min(g.dhi, min(r, 2 * g.n - 2 - r));
    vlo += (vlo - r) & 1;
    vhi -= (vhi - r) & 1;
}

// Frame value (A = H - q, stored + e*r) of the boundary cells (-1, r+1) and
// (r+1, -1) of anti-diagonal r: H = -gamma(r+2).
__device__ __forceinline__ int ring_a(const DpArgs &P, int r) {
    const int l = r + 2;
    const int gap = min(P.q1 + l * P.e1, P.oe2 + (l - 1) * P.e2);
    return -gap - P.q1 + P.e1 * r;
}

// Smallest-i cell attaining the frame value MA among the class-C slots of
// anti-diagonal r whose diagonals lie in [vlo, vhi] (lowest lane first, then
// lowest slot: i grows with the diagonal). Called by the wave holding MA.
template <int K, int C>
__device__ __forceinline__ void locate(const PairState<K> &st, const Geo &g, int lm, int MA, int r,
                                       int vlo, int vhi, int &mi, int &mj) {
    const uint64_t bal = __ballot(lm == MA);
    const int L = __builtin_ctzll(bal);
    const int dL = g.a0w + L * K;
    int found = C;
#pragma unroll
    for (int s = K - 2 + C; s >= C; s -= 2) {
        const int x = __builtin_amdgcn_readlane(st.A[s], L);
        if (x == MA && dL + s >= vlo && dL + s <= vhi) found = s;
    }
    const int dm = dL + found;
    mi = (r + dm) >> 1;
    mj = (r - dm) >> 1;
}

// The cell of the global maximum, from the values its wave parked: the
// lowest (lane, slot) of g_r's class holding g_ma on an interior diagonal of
// anti-diagonal g_r. Any wave of the pair can run it once the park is
// visible to it.
template <int K, int NW>
__device__ __forceinline__ void park_cell(const Track &tr, const Geo &g, const PairLds<K, NW> &S, int lane,
                                          int &gi, int &gj) {
    int vlo, vhi;
    diag_window(g, tr.g_r, vlo, vhi);
    // the holding window (one wave: the current one, see take_max) and the
    // class of anti-diagonal g_r in it: slot s holds a diagonal of g_r's
    // parity when s = g_r - base (mod 2)
    const int gb = NW == 1 ? g.a0w : tr.g_base;
    const int cls = (tr.g_r - gb) & 1;
    const int dl = gb + lane * K + cls;  // this lane's first class slot
    int hit = K;
#pragma unroll
    for (int t = K / 2 - 1; t >= 0; --t) {
        const int v = S.park[(cls + 2 * t) * WAVE + lane];
        const int d = dl + 2 * t;
        if (v == tr.g_ma && d >= vlo && d <= vhi) hit = t;
    }
    const int L = __builtin_ctzll(__ballot(hit < K));
    const int t = __builtin_amdgcn_readlane(hit, L);
    const int dm = gb + L * K + cls + 2 * t;
    gi = (tr.g_r + dm) >> 1;
    gj = (tr.g_r - dm) >> 1;
}

// New global maximum: the wave holding it parks the class-C values of all
// its lanes (no lane selection on the hot path; the cell is found lazily).
template <int K, int C, int NW>
__device__ __forceinline__ void park_class(const PairState<K> &st, PairLds<K, NW> &S, int lane) {
#pragma unroll
    for (int s = C; s < K; s += 2) S.park[s * WAVE + lane] = st.A[s];
}

// This wave's lane maximum of the class-C slots of anti-diagonal r over the
// interior diagonals [vlo, vhi] (masked), or over every slot (the band is
// interior on this anti-diagonal). NEG_MAX when the wave holds none.
template <int K, int C, int NW>
__device__ __forceinline__ int lane_max(const PairState<K> &st, const Geo &g, int vlo, int vhi, bool masked) {
    constexpr int H = K / 2;  // class slots C, C+2, ...
    int v[H];
    if (masked) {
        // this wave's slots inside [vlo, vhi]: a lane range per slot
        const int u = max(vlo - g.a0w, 0);
        const int vv = min(vhi - g.a0w, WAVE * K - 1);
        if (u <= vv) {
            const int qu = u / K, ru = u % K, qv = vv / K, rv = vv % K;
            const uint64_t lo0 = lanes_from(qu), lo1 = lanes_from(qu + 1);
            const uint64_t hi0 = lanes_upto(qv), hi1 = lanes_upto(qv - 1);
            const int negmax = NEG_MAX;
#pragma unroll
            for (int t = 0; t < H; ++t) {
                const int sl = C + 2 * t;
                const uint64_t msk = (ru > sl ? lo1 : lo0) & (rv >= sl ? hi0 : hi1);
                v[t] = select_by_lanes(msk, st.A[sl], negmax);
            }
        } else {
#pragma unroll
            for (int t = 0; t < H; ++t) v[t] = NEG_MAX;
        }
    } else {
#pragma unroll
        for (int t = 0; t < H; ++t) v[t] = st.A[C + 2 * t];
    }
    // balanced v_max3 tree: depth 2-3 instead of a chain of H/2
    int w3[(H + 2) / 3];
#pragma unroll
    for (int t = 0; t < (H + 2) / 3; ++t) {
        const int a = v[3 * t];
        const int b = 3 * t + 1 < H ? v[3 * t + 1] : a;
        const int c = 3 * t + 2 < H ? v[3 * t + 2] : a;
        w3[t] = max(max(a, b), c);
    }
    int lm = w3[0];
#pragma unroll
    for (int t = 1; t < (H + 2) / 3; t += 2) {
        const int b = w3[t];
        const int c = t + 1 < (H + 2) / 3 ? w3[t + 1] : b;
        lm = max(max(lm, b), c);
    }
    return lm;
}

// One wave per pair: the decisions for anti-diagonal r (class C) from its
// lane maxima lm and wave maximum MA (frame value of the local maximum M of
// Eq. 6). They run one step late, after the update of anti-diagonal r+1,
// which leaves class C untouched. The common case takes only take_max (M
// above G: the global maximum of Eq. 7 moves, the class is parked so its
// cell can be found later); the end of the sweep and z-drop candidates
// (Eq. 5) go to finish_diag, which returns 0 to go on, 1 when the sweep
// ends at its last anti-diagonal and 2 on a z-drop.
template <int K, int C>
__device__ __forceinline__ void take_max(const PairState<K> &st, const Geo &g, Track &tr, int r, int lane,
                                         int MA, PairLds<K, 1> &S) {
    // (G's window is the current one: a one-wave pair resolves G's cell
    // before its window moves; its class follows from g_r)
    if (MA > tr.gf) {
        park_class<K, C, 1>(st, S, lane);
        tr.g_r = r;
        tr.g_ma = MA;
    }
    tr.gf = max(tr.gf, MA);
}

template <int K, int C>
__device__ __forceinline__ int finish_diag(const PairState<K> &st, const DpArgs &P, const Geo &g, Track &tr,
                                           int r, int lane, int lm, int MA, bool up, PairLds<K, 1> &S) {
    const bool last = r >= g.r_last;
    int vlo, vhi;
    diag_window(g, r, vlo, vhi);
    int mi, mj;
    locate<K, C>(st, g, lm, MA, r, vlo, vhi, mi, mj);
    tr.endS = MA + P.q1 - P.e1 * r;  // back to the true score
    tr.endI = mi;
    tr.endJ = mj;
    // G - M, in the frame of anti-diagonal r
    const int drop = tr.gf - MA;
    if (!up && P.Z >= 0 && drop > P.Z) {
        if (tr.g_r != tr.g_res) {
            int gi, gj;
            park_cell<K, 1>(tr, g, S, lane, gi, gj);
            tr.gi = gi;
            tr.gj = gj;
            tr.g_res = tr.g_r;
        }
        if (mi > tr.gi && mj > tr.gj) {
            int dd = (mi - tr.gi) - (mj - tr.gj);
            dd = dd < 0 ? -dd : dd;
            if (drop > P.Z + P.e2 * dd) return 2;
        }
    }
    return last ? 1 : 0;
}

// Several waves per pair: the decisions for anti-diagonal r (class C) after
// the exchange that published every wave's maximum of it (slot `k` of the
// exchange buffers `b`). All waves read the same maxima and take the same
// decisions. The rare events that need a cell (the last anti-diagonal, a
// z-drop candidate) are resolved by the wave holding the anti-diagonal
// maximum (the lowest such wave: the smallest diagonal, hence the smallest
// i): after a barrier that makes every park visible, it locates the cells,
// runs the test and writes the pair's result, then tells every wave the
// outcome through LDS and a second barrier. Returns true when done.
template <int K, int C, int NW>
__device__ __forceinline__ bool decide_mw(const PairState<K> &st, const DpArgs &P, const Geo &g, Track &tr,
                                          int r, int lm, int lane, int wv, PairLds<K, NW> &S, int p, int b,
                                          int k, bool ring) {
    // LDS loads land in VGPRs: readfirstlane keeps the decisions scalar
    int MA = __builtin_amdgcn_readfirstlane(S.ma[b][0][k]);
    int vstar = 0;
#pragma unroll
    for (int v = 1; v < NW; ++v) {
        const int x = __builtin_amdgcn_readfirstlane(S.ma[b][v][k]);
        if (x > MA) {
            MA = x;
            vstar = v;
        }
    }
    const bool last = r >= g.r_last;
    int vlo = 0, vhi = 0;
    bool masked = false;
    if (__builtin_expect(ring && MA == ring_a(P, r), 0)) {
        // a boundary cell may hold the maximum: redo the anti-diagonal masked
        masked = true;
        diag_window(g, r, vlo, vhi);
        lm = vlo <= vhi ? lane_max<K, C, NW>(st, g, vlo, vhi, true) : NEG_MAX;
        const int MAw = wave_max(lm);
        if (lane == 0) S.ma2[wv] = MAw;
        __syncthreads();
        MA = __builtin_amdgcn_readfirstlane(S.ma2[0]);
        vstar = 0;
#pragma unroll
        for (int v = 1; v < NW; ++v) {
            const int x = __builtin_amdgcn_readfirstlane(S.ma2[v]);
            if (x > MA) {
                MA = x;
                vstar = v;
            }
        }
        __syncthreads();  // S.ma2 is reused by the next redo
    }
    if (MA <= LIVE_MIN) return last;  // no interior cell on this anti-diagonal
    const int M = MA + P.q1 - P.e1 * r;  // back to the true score
    const bool up = M > tr.G;
    if (up) {
        if (wv == vstar) park_class<K, C, NW>(st, S, lane);
        tr.G = M;
        tr.g_r = r;
        tr.g_base = g.a0 + vstar * wave_stride(K);
        tr.g_ma = MA;
        tr.g_set = true;
    }
    const bool cand = !up && P.Z >= 0 && tr.G - M > P.Z;
    if (!(cand || last)) return false;
    __syncthreads();  // every park so far is visible to the wave resolving
    if (wv == vstar) {
        if (!masked) diag_window(g, r, vlo, vhi);
        int mi, mj, gi = -1, gj = -1;
        locate<K, C>(st, g, lm, MA, r, vlo, vhi, mi, mj);
        if (up) {
            gi = mi;
            gj = mj;
        } else if (tr.g_set) {
            park_cell<K, NW>(tr, g, S, lane, gi, gj);
        }
        bool drop = false;
        if (cand && mi > gi && mj > gj) {
            int dd = (mi - gi) - (mj - gj);
            dd = dd < 0 ? -dd : dd;
            drop = tr.G - M > P.Z + P.e2 * dd;
        }
        if (drop || last) {
            if (lane < 7) {
                const int v[7] = {tr.G, gi, gj, M, mi, mj, drop ? 1 : 0};
                int val = v[0];
#pragma unroll
                for (int t = 1; t < 7; ++t) val = (lane == t) ? v[t] : val;
                reinterpret_cast<int32_t *>(P.out + p)[lane] = val;
            }
        }
        if (lane == 0) S.flag = (drop || last) ? 1 : 0;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(S.flag) != 0;
}

// Several waves per pair, at an exchange: each wave hands its neighbours
// the owned diagonals next to their ghosts -- slots K-4, K-3 of lane 63 go
// up, slots 2, 3 of lane 0 go down -- with their latest values.
template <int K, int NW>
__device__ __forceinline__ void publish_ghosts(const PairState<K> &st, PairLds<K, NW> &S, int b, int lane,
                                               int wv) {
    if (wv < NW - 1 && lane == WAVE - 1) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            S.up[b][wv][t][0] = st.A[K - 4 + t];
            S.up[b][wv][t][1] = st.E[K - 4 + t];
            S.up[b][wv][t][2] = st.X[K - 4 + t];
            S.up[b][wv][t][3] = st.F[K - 4 + t];
            S.up[b][wv][t][4] = st.Y[K - 4 + t];
        }
    }
    if (wv > 0 && lane == 0) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            S.dn[b][wv][t][0] = st.A[2 + t];
            S.dn[b][wv][t][1] = st.E[2 + t];
            S.dn[b][wv][t][2] = st.X[2 + t];
            S.dn[b][wv][t][3] = st.F[2 + t];
            S.dn[b][wv][t][4] = st.Y[2 + t];
        }
    }
}

// ... and, after the barrier, each wave refreshes its ghosts: slots 0, 1 of
// lane 0 from the wave below, slots K-2, K-1 of lane 63 from the wave above.
template <int K, int NW>
__device__ __forceinline__ void read_ghosts(PairState<K> &st, const PairLds<K, NW> &S, int b, int lane,
                                            int wv) {
    if (wv > 0 && lane == 0) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            st.A[t] = S.up[b][wv - 1][t][0];
            st.E[t] = S.up[b][wv - 1][t][1];
            st.X[t] = S.up[b][wv - 1][t][2];
            st.F[t] = S.up[b][wv - 1][t][3];
            st.Y[t] = S.up[b][wv - 1][t][4];
        }
    }
    if (wv < NW - 1 && lane == WAVE - 1) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            st.A[K - 2 + t] = S.dn[b][wv + 1][t][0];
            st.E[K - 2 + t] = S.dn[b][wv + 1][t][1];
            st.X[K - 2 + t] = S.dn[b][wv + 1][t][2];
            st.F[K - 2 + t] = S.dn[b][wv + 1][t][3];
            st.Y[K - 2 + t] = S.dn[b][wv + 1][t][4];
        }
    }
}


// Bit T set for every step T of a block (0..7) with lo <= T <= hi.
__device__ __forceinline__ uint32_t step_bits(int lo, int hi) {
    lo = max(lo, 0);
    hi = min(hi, 7);
    return lo > hi ? 0u : ((0xFFu >> (7 - hi)) & (0xFFu << lo));
}

// One wave per pair, 8 anti-diagonals r0 .. r0+7. Step T finishes
// anti-diagonal r-1 (its clamps, lane maxima and wave reduction) in the
// same straight-line code as the update of anti-diagonal r, so the serial
// reduction hides among the independent cell updates; the decisions for r-1
// follow. The last anti-diagonal's decisions therefore come one step after
// it; the extra anti-diagonal computed meanwhile is never looked at.
//
// The lane maxima are unmasked: the wall and the cells leaving the
// rectangle are clamped to -inf, cells before row/column -1 never leave
// -inf, and the only other finite cells outside the rectangle are the two
// boundary cells (-1, r+1), (r+1, -1) while they are in the band. When the
// wave maximum equals their value the anti-diagonal is redone with masks.
template <int K>
__device__ __forceinline__ bool run_block1(PairState<K> &st, const DpArgs &P, const Geo &g, Track &tr,
                                           int r0, int lane, uint64_t wall_lanes, int wall_pos,
                                           PairLds<K, 1> &S) {
    // Which steps of the block need the wall clamp, an exit-cell clamp or
    // the boundary-cell check, as bit masks over T, worked out once per
    // block: step T finishes anti-diagonal r0+T-1, whose cell i = n sits at
    // slot position pi0 - T and whose cell j = m at pj0 + T.
    const int t1 = 1 - r0;  // first step with an anti-diagonal to finish
    const int pi0 = 2 * g.n - r0 + 1 - g.a0w;
    const int pj0 = r0 - 1 - 2 * g.m - g.a0w;
    // the cell (n, -1) is clamped too when the band reaches the target's end
    // (a1 = n: no wall then, see align_pair)
    const int a1x = g.a1 + (g.a1 == g.n ? 1 : 0);
    const uint32_t bits_i = step_bits(max(max(t1, 2 * g.n - r0 + 1 - a1x), pi0 - WAVE * K + 1), pi0);
    const uint32_t bits_j = step_bits(max(max(t1, g.a0 + 2 * g.m + 1 - r0), -pj0), WAVE * K - 1 - pj0);
    const uint32_t bits_w = wall_lanes != 0 ? ((wall_pos & 1) ? 0x55u : 0xAAu) & step_bits(t1, 7) : 0u;
    const uint32_t bits_ring = step_bits(t1, max(g.a1, -g.a0) - r0 - 1);
    const int ring_r0 = P.ring_b0 + P.ring_d * r0;  // boundary value's linear piece at r0
    const uint32_t bits_c = bits_w | bits_i | bits_j;  // steps with any clamp
    const uint32_t bits_dec = step_bits(t1, 7);        // steps with decisions to take
    // steps still to run: anti-diagonal r >= 0 and the pair not ended. The
    // end clears it (no return from inside the unrolled steps, which would
    // cost every step flow bookkeeping), so the block's later steps do
    // nothing and the block reports the end when it returns.
    uint32_t bits_run = step_bits(-r0, 7);
    const int Zc = P.Z >= 0 ? P.Z : 0x7fffffff;        // z-drop threshold, none when Z < 0
    const int end0 = r0 - g.r_last;                    // step T decides r_last when end0 + T > 0
#define GA_STEP1(T)                                                                        \
    {                                                                                      \
        constexpr int C = (T) & 1;                                                         \
        constexpr int CP = C ^ 1;                                                          \
        constexpr int KC = (T) >> 1;                                                       \
        const int r = r0 + (T);                                                            \
        if (bits_run & (1u << (T))) {                                                      \
            const int rp = r - 1;                                                          \
            if (bits_c & (1u << (T))) {                                                    \
                if (bits_w & (1u << (T))) clamp_wall<K, CP>(st, wall_lanes, wall_pos);     \
                if (bits_i & (1u << (T))) clamp_cell<K, CP, true>(st, pi0 - (T));          \
                if (bits_j & (1u << (T))) clamp_cell<K, CP, false>(st, pj0 + (T));         \
            }                                                                              \
            int lm = lane_max<K, CP, 1>(st, g, 0, 0, false);                               \
            int MA = wave_max(lm);                                                         \
            dp_step<K, C, KC, (K < 32)>(st, P);                                            \
            if (bits_dec & (1u << (T))) {                                                  \
                if (__builtin_expect((bits_ring & (1u << (T))) &&                          \
                                     MA == max(P.ring_a0, ring_r0 + P.ring_d * ((T) - 1)), 0)) { \
                    /* a boundary cell may hold the maximum: redo it masked */             \
                    int vlo, vhi;                                                          \
                    diag_window(g, rp, vlo, vhi);                                          \
                    lm = lane_max<K, CP, 1>(st, g, vlo, vhi, true);                        \
                    MA = wave_max(lm);                                                     \
                }                                                                          \
                tr.gf += P.e1;  /* G's frame value on anti-diagonal rp */                 \
                /* M above G: Eq. 7's maximum moves (never for an anti-diagonal   */       \
                /* with no interior cell: its MA is below every frame value)      */       \
                take_max<K, CP>(st, g, tr, rp, lane, MA, S);                               \
                /* the last anti-diagonal, or G - M above Z (then M is not above  */       \
                /* G: Zc >= 0), as one signed test: no overflow, G - M < 2^31    */       \
                if (__builtin_expect(max(end0 + (T), tr.gf - MA - Zc) > 0, 0)) {           \
                    if (MA > LIVE_MIN) {  /* the anti-diagonal has an interior cell */     \
                        /* M above G here exactly when G moved to this anti-diagonal */    \
                        const int rc = finish_diag<K, CP>(st, P, g, tr, rp, lane, lm, MA,  \
                                                          tr.g_r == rp, S);                \
                        if (rc) {                                                          \
                            tr.zd = rc >> 1;                                               \
                            bits_run = 0;                                                  \
                        }                                                                  \
                    }                                                                      \
                }                                                                          \
            }                                                                              \
        }                                                                                  \
    }
    GA_STEP1(0)
    GA_STEP1(1)
    GA_STEP1(2)
    GA_STEP1(3)
    GA_STEP1(4)
    GA_STEP1(5)
    GA_STEP1(6)
    GA_STEP1(7)
#undef GA_STEP1
    return bits_run == 0;
}

// Several waves per pair, 8 anti-diagonals r0 .. r0+7 in four exchanges of
// two. Each wave updates its slots (ghosts included) for both
// anti-diagonals with -inf beyond its edge lanes -- a ghost fed -inf is at
// most its true value, and the two ghost diagonals keep every owned
// diagonal exact for two anti-diagonals -- then publishes its owned edge
// diagonals and both wave maxima, meets the others at one barrier,
// refreshes its ghosts and takes the decisions of both anti-diagonals in
// order. Ghost values never exceed the true ones, so counting them in a
// wave maximum changes nothing (the owner counts the true value).
template <int K, int NW>
__device__ __forceinline__ bool run_block(PairState<K> &st, const DpArgs &P, const Geo &g,
                                          Track &tr, int r0, int lane, int wv, uint64_t wall_lanes,
                                          int wall_pos, PairLds<K, NW> &S, int p) {
    // the steps that need each clamp and the boundary-cell check, as bit
    // masks over T worked out once per block (step T updates anti-diagonal
    // r0+T: its cell i = n at slot position pi0 - T of this wave, its cell
    // j = m at pj0 + T)
    const int t0 = -r0;
    const int pi0 = 2 * g.n - r0 - g.a0w;
    const int pj0 = r0 - 2 * g.m - g.a0w;
    const int a1x = g.a1 + (g.a1 == g.n ? 1 : 0);  // (n, -1) too when a1 = n (no wall)
    const uint32_t bits_i = step_bits(max(max(t0, 2 * g.n - r0 - a1x), pi0 - WAVE * K + 1), pi0);
    const uint32_t bits_j = step_bits(max(max(t0, g.a0 + 2 * g.m - r0), -pj0), WAVE * K - 1 - pj0);
    const uint32_t bits_w = wall_lanes != 0 ? ((wall_pos & 1) ? 0xAAu : 0x55u) & step_bits(t0, 7) : 0u;
    const uint32_t bits_ring = step_bits(t0, max(g.a1, -g.a0) - r0 - 2);
#define GA_HSTEP(T, LM, MAW)                                                          \
    {                                                                                 \
        constexpr int C = (T) & 1;                                                    \
        constexpr int KC = (T) >> 1;                                                  \
        if (r0 + (T) >= 0) {                                                          \
            dp_step<K, C, KC>(st, P);                                  \
            if (bits_w & (1u << (T))) clamp_wall<K, C>(st, wall_lanes, wall_pos);     \
            if (bits_i & (1u << (T))) clamp_cell<K, C, true>(st, pi0 - (T));          \
            if (bits_j & (1u << (T))) clamp_cell<K, C, false>(st, pj0 + (T));         \
            LM = lane_max<K, C, NW>(st, g, 0, 0, false);                              \
            MAW = wave_max(LM);                                                       \
        }                                                                             \
    }
#define GA_EXCHANGE(T)                                                                \
    {                                                                                 \
        int lm0 = NEG_MAX, lm1 = NEG_MAX, ma0 = NEG_MAX, ma1 = NEG_MAX;               \
        GA_HSTEP(T, lm0, ma0)                                                         \
        GA_HSTEP((T) + 1, lm1, ma1)                                                   \
        const int b = ((r0 + (T)) >> 1) & 1;                                          \
        publish_ghosts<K, NW>(st, S, b, lane, wv);                                    \
        if (lane == 0) {                                                              \
            S.ma[b][wv][0] = ma0;                                                     \
            S.ma[b][wv][1] = ma1;                                                     \
        }                                                                             \
        __syncthreads();                                                              \
        read_ghosts<K, NW>(st, S, b, lane, wv);                                       \
        if (r0 + (T) >= 0 &&                                                          \
            decide_mw<K, 0, NW>(st, P, g, tr, r0 + (T), lm0, lane, wv, S, p, b, 0,    \
                                (bits_ring & (1u << (T))) != 0))                      \
            return true;                                                              \
        if (r0 + (T) + 1 >= 0 &&                                                      \
            decide_mw<K, 1, NW>(st, P, g, tr, r0 + (T) + 1, lm1, lane, wv, S, p, b, 1, \
                                (bits_ring & (1u << ((T) + 1))) != 0))                \
            return true;                                                              \
    }
    GA_EXCHANGE(0)
    GA_EXCHANGE(2)
    GA_EXCHANGE(4)
    GA_EXCHANGE(6)
#undef GA_EXCHANGE
#undef GA_HSTEP
    return false;
}

// Raw words holding the block's base windows T[I0 .. I0+K/2+4) and
// Q[J0-K/2+1 .. J0+4) of this lane, read from the wave's rings. Positions
// outside a sequence read whatever the ring holds there; they only feed
// cells outside the rectangle, which never reach an interior cell.
template <int K>
struct Windows {
    static constexpr int NW = K / 8 + 3;
    uint32_t RT[NW], RQ[NW];
    int to, qo;  // byte misalignment of the first word
};

template <int K>
__device__ __forceinline__ void load_windows(Windows<K> &wd, const uint32_t *ring_t, const uint32_t *ring_q,
                                             int r0, int d0) {
    constexpr int KH = K / 2;
    constexpr int MASK = Ring<K>::WORDS - 1;
    const int ts = (r0 + d0) >> 1;           // I0
    const int qs = ((r0 - d0) >> 1) - KH + 1;  // J0 - K/2 + 1
    const uint32_t *tw = ring_t + ((ts >> 2) & MASK);
    const uint32_t *qw = ring_q + ((qs >> 2) & MASK);
#pragma unroll
    for (int k = 0; k < Windows<K>::NW; ++k) {
        wd.RT[k] = tw[k];
        wd.RQ[k] = qw[k];
    }
    wd.to = ts & 3;
    wd.qo = qs & 3;
}

// Four 2-bit codes (bits 0..7) and their N bits (bits 0..3) -> four bytes
// (0..3, N = 4): the codes spread to byte lanes in two shift-or-mask steps,
// the N bits by one multiply whose four shifted copies never overlap.
__device__ __forceinline__ uint32_t expand4(uint32_t c8, uint32_t n4) {
    const uint32_t y = (c8 | (c8 << 12)) & 0x000F000Fu;
    const uint32_t codes = (y | (y << 6)) & 0x03030303u;
    return codes | (((n4 * 0x00204081u) & 0x01010101u) << 2);
}

// Make the ring of one sequence hold the ring words [wlo, whi) (word x =
// positions 4x .. 4x+3). The ring holds the words below `filled`
// (wave-uniform); when the block needs more, lanes fill the next 64 words
// at once, one each (bases past the sequence are left as they are), until
// it holds enough. Rare: once every 64 words of advance. The source comes
// from LDS, where the wave put it when the pair started.
template <int K>
__device__ __forceinline__ void refill(uint32_t *ring, const SeqSource *src, int &filled, int wlo, int whi,
                                    int lane) {
    constexpr int WORDS = Ring<K>::WORDS, MIRROR = Ring<K>::MIRROR;
    const uint32_t *words = src->words;
    const uint32_t *nmask = src->nmask;
    const int64_t nbit0 = src->nbit0;
    const int wend = (int)((src->len + 3) >> 2);
    if (filled < wlo) filled = wlo;  // nothing below the windows is needed
    do {
        const int x = filled + lane;
        if (x < wend) {
            const uint32_t w = words[x >> 2];
            uint32_t n4 = 0;
            if (nmask) {
                const int64_t bit = nbit0 + 4 * (int64_t)x;
                n4 = (nmask[bit >> 5] >> (int)(bit & 31)) & 0xFu;
            }
            const uint32_t v = expand4((w >> (8 * (x & 3))) & 0xFFu, n4);
            const int i = x & (WORDS - 1);
            ring[i] = v;
            if (i < MIRROR) ring[WORDS + i] = v;
        }
        filled += WAVE;
    } while (filled < whi);
}

// Stage the bases the windows of the block at anti-diagonal r need, for a
// wave whose lane 0 holds diagonal b first: target positions
// [I0, I0 + 32K + 4) and query positions [J0 - 32K + 1, J0 + 4) of lane
// 0's I0, J0, clipped to the sequences. `ft`, `fq`: the rings' watermarks.
template <int K>
__device__ __forceinline__ void stage_block(const Geo &g, uint32_t *ring_t, uint32_t *ring_q,
                                            const SeqSource *src, int &ft, int &fq, int r, int b, int lane) {
    const int I0 = (r + b) >> 1, J0 = (r - b) >> 1;
    {
        const int lo = max(I0, 0), hi = min(I0 + 32 * K + 4, g.n);
        if (lo < hi && ((hi + 3) >> 2) > ft) refill<K>(ring_t, src, ft, lo >> 2, (hi + 3) >> 2, lane);
    }
    {
        const int lo = max(J0 - 32 * K + 1, 0), hi = min(J0 + 4, g.m);
        if (lo < hi && ((hi + 3) >> 2) > fq) refill<K>(ring_q, src + 1, fq, lo >> 2, (hi + 3) >> 2, lane);
    }
    __builtin_amdgcn_wave_barrier();  // the ring writes precede the window reads
}

// v_bitop3 truth table of (x, y, m) -> m ? (x | y) : (x ^ y), built the way
// the instruction indexes it: operand bits (x, y, m) form the index with x as
// the most significant bit, i.e. the table is f applied to 0xF0, 0xCC, 0xAA.
constexpr uint32_t CLS_TT = (((0xF0u | 0xCCu) & 0xAAu) | ((0xF0u ^ 0xCCu) & ~0xAAu)) & 0xFFu;

template <int K>
__device__ __forceinline__ void build_scores(PairState<K> &st, const Windows<K> &wd, const DpArgs &P) {
    constexpr int KH = K / 2;
    constexpr int NW = Windows<K>::NW;
    uint32_t TW[NW - 1], QW[NW - 1];
#pragma unroll
    for (int k = 0; k < NW - 1; ++k) {
        TW[k] = __builtin_amdgcn_alignbyte(wd.RT[k + 1], wd.RT[k], (uint32_t)wd.to);
        QW[k] = __builtin_amdgcn_alignbyte(wd.RQ[k + 1], wd.RQ[k], (uint32_t)wd.qo);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int c = s & 1, sp = s >> 1;
        const uint32_t t4 = window4(TW, c + sp);       // T[I0+c+sp .. +4)
        const uint32_t q4 = window4(QW, KH - 1 - sp);  // Q[J0-sp .. +4)
        // class byte: t ^ q in bits 0-1, (t | q) & 4 (either is N) in bit 2,
        // one v_bitop3 with the bit-2 mask as third operand
        const uint32_t cls = __builtin_amdgcn_bitop3_b32(t4, q4, 0x04040404u, CLS_TT);
        st.S4[s] = __builtin_amdgcn_perm(P.lut_hi, P.lut_lo, cls);
    }
}

// A sliding wave's first diagonal for the block of anti-diagonals r0 ..
// r0+7 (then anti-diagonal r0-1, finished in that block, too), moved from
// `base` by whole lanes. Sliding down (n <= m) it keeps the boundary cell
// (-1, r+1) on diagonal -r-2 in the window, stopping at a0 (base stays a
// multiple of K above a0, so lane 0's -inf fill becomes the band wall there);
// below the window every cell is before column -1, hence -inf. Sliding up it
// keeps the boundary cell (r+1, -1) on diagonal r+2, or the band wall a1+1,
// in the window; below it every cell is past the query end. The class
// choice guarantees the other end of the window still covers every cell
// that can be finite (see class_for).
template <int K>
__device__ __forceinline__ int window_base(const Geo &g, int slide, int base, int r0) {
    if (slide < 0) {
        while (base - K >= g.a0 && base > -r0 - 9) base -= K;
    } else if (slide > 0) {
        const int need = min(g.a1 + 1, r0 + 9);
        while (base + WAVE * K - 1 < need) base += K;
    }
    return base;
}

// Move the window by `step` lanes (-2, -1, 1 or 2): down (step < 0: lane l
// takes lane l+step's slots, the lowest lanes start at -inf) or up (lane l
// takes lane l+step's, the highest lanes at -inf). Each state array goes
// through LDS: row l+2 of `rows` takes lane l's K slots, then every lane
// reads the row `step` away; rows 0, 1 and 66, 67 hold -inf for the lanes
// with no source on that side. Staging costs no registers beyond the
// state, and the rows are reused array after array; a two-lane move (a
// 4-slot window moves two lanes per block) costs one round trip.
// A sliding window's workgroup is one wave, whose LDS operations complete
// in order: a wave-level scheduling barrier keeps the compiler from moving
// the reads above the writes (or the next array's writes above the reads),
// and no workgroup barrier is needed.
template <int K>
__device__ __forceinline__ void shift_array(typename PairState<K>::VecK &a, int *rows, int lane, int step) {
    int4 *own = reinterpret_cast<int4 *>(rows + (lane + 2) * K);
#pragma unroll
    for (int q = 0; q < K / 4; ++q) own[q] = make_int4(a[4 * q], a[4 * q + 1], a[4 * q + 2], a[4 * q + 3]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // every row is staged before any lane reads its neighbour's
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int4 *from = reinterpret_cast<const int4 *>(rows + (lane + 2 + step) * K);
#pragma unroll
    for (int q = 0; q < K / 4; ++q) {
        const int4 v = from[q];
        a[4 * q] = v.x;
        a[4 * q + 1] = v.y;
        a[4 * q + 2] = v.z;
        a[4 * q + 3] = v.w;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // every lane has read before the next array is staged
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int K>
__device__ __forceinline__ void shift_lanes(PairState<K> &st, int *rows, int lane, int step) {
    static_assert(K % 4 == 0, "rows are staged 16 bytes at a time");
    shift_array<K>(st.A, rows, lane, step);
    shift_array<K>(st.E, rows, lane, step);
    shift_array<K>(st.X, rows, lane, step);
    shift_array<K>(st.F, rows, lane, step);
    shift_array<K>(st.Y, rows, lane, step);
}

// Geometry of pair p (band edges, interior diagonals, last anti-diagonal);
// returns the band's width D in diagonals. a0w is left at a0.
__device__ __forceinline__ int pair_geo(const DpArgs &P, int p, Geo &g) {
    g.n = P.t_len[p];
    g.m = P.q_len[p];
    const int n = g.n, m = g.m, w = P.w;
    int a1;
    if (w >= 0) {
        g.a0 = max(-w, -m);
        a1 = min(w, n);
    } else {
        g.a0 = -m;
        a1 = n;
    }
    g.a0w = g.a0;
    g.dlo = max(g.a0, 1 - m);
    g.dhi = min(a1, n - 1);
    {
        const int dc = min(max(n - m, g.dlo), g.dhi);
        g.r_last = min(2 * n - 2 - dc, 2 * m - 2 + dc);
    }
    g.a1 = a1;
    return a1 - g.a0 + 1;
}

// The right wall of a window whose lane 0 starts at diagonal g.a0w: the slot
// of diagonal a1+1 if the window holds it. When the band reaches the
// target's end (a1 = n) every cell on that diagonal lies past the target's
// end: the exit-cell clamp of (n, -1) keeps it at -inf instead, with no
// clamp on the other steps.
template <int K>
__device__ __forceinline__ void place_wall(const Geo &g, int &wall_pos, uint64_t &wall_lanes) {
    const int Dw = g.a1 + 1 - g.a0w;
    const bool has_wall = Dw >= 0 && Dw < WAVE * K && g.a1 < g.n;
    wall_pos = has_wall ? Dw % K : 0;
    wall_lanes = has_wall ? (1ull << (Dw / K)) : 0ull;
}

// The state before the first anti-diagonal, for the lane whose slots start
// at diagonal d0: the origin (-1,-1) on anti-diagonal -2, (-1,0) and (0,-1)
// on anti-diagonal -1 (runs of length 1), every other slot -inf; values in
// the drifting frame.
template <int K>
__device__ __forceinline__ void init_state(PairState<K> &st, const DpArgs &P, const Geo &g, int d0) {
    const int gap1 = min(P.oe1, P.oe2);
    const int a_origin = -2 * P.e1 - P.q1;
    const int a_ring = -gap1 - P.e1 - P.q1;
    st.eA = st.eE = st.eX = st.fA = st.fF = st.fY = NEG;
#pragma unroll
    for (int s = 0; s < K; ++s) {
        const int d = d0 + s;
        const bool held = d >= g.a0 && d <= g.a1;
        st.A[s] = NEG;
        st.E[s] = NEG;
        st.X[s] = NEG;
        st.F[s] = NEG;
        st.Y[s] = NEG;
        if (held && d == 0) st.A[s] = a_origin;
        if (held && d == -1) {  // (-1,0): horizontal run of length 1
            st.A[s] = a_ring;
            st.F[s] = -P.oe1 - P.e1;
            st.Y[s] = -P.oe2 - P.e2;
        }
        if (held && d == 1) {  // (0,-1): vertical run of length 1
            st.A[s] = a_ring;
            st.E[s] = -P.oe1 - P.e1;
            st.X[s] = -P.oe2 - P.e2;
        }
    }
}

// One wave per pair: resolve the cell of the global maximum if its class is
// still parked (before the park is reused, or at the end).
template <int K>
__device__ __forceinline__ void settle_max(Track &tr, const Geo &g, const PairLds<K, 1> &S, int lane) {
    if (tr.g_r != tr.g_res) {
        int gi, gj;
        park_cell<K, 1>(tr, g, S, lane, gi, gj);
        tr.gi = gi;
        tr.gj = gj;
        tr.g_res = tr.g_r;
    }
}

// One wave per pair: the pair's result (Eq. 7's maximum and its cell, where
// the sweep ended, whether z-drop ended it), one field per lane.
template <int K>
__device__ __forceinline__ void write_result(const DpArgs &P, int p, Track &tr, const Geo &g,
                                             const PairLds<K, 1> &S, int lane) {
    settle_max<K>(tr, g, S, lane);
    if (lane < 7) {
        const int G = tr.g_ma + P.q1 - P.e1 * tr.g_r;
        const int v[7] = {G, tr.gi, tr.gj, tr.endS, tr.endI, tr.endJ, tr.zd};
        int val = v[0];
#pragma unroll
        for (int k = 1; k < 7; ++k) val = (lane == k) ? v[k] : val;
        reinterpret_cast<int32_t *>(P.out + p)[lane] = val;
    }
}

template <int K, int NW, bool SL>
__device__ void align_pair(const DpArgs &P, int p, int lane, int wv, PairLds<K, NW> &S, int *rows) {
    Geo g;
    const int D = pair_geo(P, p, g);
    const int n = g.n, m = g.m;
    g.a0w = g.a0 + wv * wave_stride(K);
    // one wave on a band wider than it holds: the window slides (class_for)
    const int slide = (SL && D > WAVE * K) ? (n <= m ? -1 : 1) : 0;
    int r0 = (g.a0 & 1) ? -1 : -2;  // blocks of 8 anti-diagonals start on the class of slot 0
    if (slide < 0) g.a0w = g.a0 + K * max(0, (-r0 - 9 - g.a0) / K);
    int wall_pos = 0;
    uint64_t wall_lanes = 0;
    place_wall<K>(g, wall_pos, wall_lanes);

    const int d0 = g.a0w + lane * K;
    PairState<K> st;
    init_state<K>(st, P, g, d0);
    // G = 0 at the origin, in the frame of anti-diagonal -1 (the first
    // decision, for anti-diagonal 0, advances it)
    Track tr{0, -1, -1, 0, -1, -1, 0, -1, 0, -P.q1 - P.e1, false, false, -P.q1 - P.e1, -1};

    // this wave's base rings and their sources, filled for the first block
    uint32_t *ring_t = S.ring[wv][0], *ring_q = S.ring[wv][1];
    if (lane == 0) {
        const int64_t to = P.t_off[p], qo = P.q_off[p];
        S.src[wv][0] = SeqSource{P.tw + to, P.tn, 16 * to, n};
        S.src[wv][1] = SeqSource{P.qw + qo, P.qn, 16 * qo, m};
    }
    __builtin_amdgcn_wave_barrier();
    int ft = -(1 << 30), fq = -(1 << 30);
    stage_block<K>(g, ring_t, ring_q, S.src[wv], ft, fq, r0, g.a0w, lane);
    Windows<K> wd;
    load_windows<K>(wd, ring_t, ring_q, r0, d0);
    int base_next = g.a0w;
    for (;;) {
        if (slide != 0 && base_next != g.a0w) {
            if constexpr (NW == 1) settle_max<K>(tr, g, S, lane);  // G's cell, while its window is current
            // move the window to this block's base, two lanes at a time
            const int dir = base_next < g.a0w ? -1 : 1;
            int lanes = min((base_next - g.a0w) * dir / K, WAVE);  // whole lanes by construction
            while (lanes > 0) {
                const int k = lanes >= 2 ? 2 : 1;
                shift_lanes<K>(st, rows, lane, dir * k);
                lanes -= k;
            }
            g.a0w = base_next;
            place_wall<K>(g, wall_pos, wall_lanes);
        }
        build_scores<K>(st, wd, P);
        base_next = slide != 0 ? window_base<K>(g, slide, g.a0w, r0 + 8) : g.a0w;
        stage_block<K>(g, ring_t, ring_q, S.src[wv], ft, fq, r0 + 8, base_next, lane);
        load_windows<K>(wd, ring_t, ring_q, r0 + 8, base_next + lane * K);  // next block, in flight
        bool done;
        if constexpr (NW == 1)
            done = run_block1<K>(st, P, g, tr, r0, lane, wall_lanes, wall_pos, S);
        else
            done = run_block<K, NW>(st, P, g, tr, r0, lane, wv, wall_lanes, wall_pos, S, p);
        if (done) break;
        r0 += 8;
    }
    if constexpr (NW == 1) write_result<K>(P, p, tr, g, S, lane);
    // (several waves: the wave that ended the sweep has written the result)
}

// ---------------------------------------------------------------------------
// Narrow start and end triangles. A band of D diagonals needs K slots per
// lane only while an anti-diagonal's finite cells span more than a narrower
// class holds. Near the origin those cells lie between the boundary cells
// (-1, r+1) and (r+1, -1), 2r+5 diagonals; near the end, between the cells
// leaving the rectangle. A one-wave pair of the wide class KB therefore runs
// its first and last anti-diagonals with KT < KB slots per lane on a window
// of 64*KT diagonals placed over them, and the middle with KB slots over the
// whole band. The cells and decisions are those of the wide sweep: every
// slot outside the narrow window holds -inf in the wide sweep at those
// anti-diagonals (before row/column -1, outside the band, or past a cell
// that left the rectangle), and the window's edge lanes see -inf beyond it.
// The state moves between the two slot layouts through LDS, between blocks.

// LDS of a pair that changes layout: the views of both layouts share the
// storage (each phase stages its own rings), and the move between layouts
// goes through the wide layout's park, indexed by diagonal - a0.
template <int KB, int KT>
union SplitLds {
    PairLds<KB, 1> wide;
    PairLds<KT, 1> narrow;
};

// Copy one state array from layout KF (lane 0 at diagonal a0 + f_off) to
// layout KD (lane 0 at a0 + d_off) through `stage` (64*max(KF, KD) words,
// word x = diagonal a0 + x); destination slots the source does not hold
// start at -inf. Both windows lie inside [a0, a0 + 64*max(KF, KD)).
template <int KF, int KD>
__device__ __forceinline__ void move_array(const typename PairState<KF>::VecK &from,
                                           typename PairState<KD>::VecK &to, int *stage, int f_off, int d_off,
                                           int lane) {
    int *dst = stage + d_off + lane * KD;  // even offset: 8-byte aligned pairs
    if constexpr (KD > KF) {
#pragma unroll
        for (int q = 0; q < KD / 2; ++q) reinterpret_cast<int2 *>(dst)[q] = make_int2(NEG, NEG);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    int *src = stage + f_off + lane * KF;
#pragma unroll
    for (int q = 0; q < KF / 2; ++q) reinterpret_cast<int2 *>(src)[q] = make_int2(from[2 * q], from[2 * q + 1]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // every source slot is staged before any lane reads
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < KD / 2; ++q) {
        const int2 v = reinterpret_cast<const int2 *>(dst)[q];
        to[2 * q] = v.x;
        to[2 * q + 1] = v.y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();  // every lane has read before the next array is staged
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KF, int KD>
__device__ __forceinline__ void move_state(const PairState<KF> &from, PairState<KD> &to, int *stage, int f_off,
                                           int d_off, int lane) {
    // the stage reuses the park and the rings: their last reads come first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    move_array<KF, KD>(from.A, to.A, stage, f_off, d_off, lane);
    move_array<KF, KD>(from.E, to.E, stage, f_off, d_off, lane);
    move_array<KF, KD>(from.X, to.X, stage, f_off, d_off, lane);
    move_array<KF, KD>(from.F, to.F, stage, f_off, d_off, lane);
    move_array<KF, KD>(from.Y, to.Y, stage, f_off, d_off, lane);
    to.eA = to.eE = to.eX = to.fA = to.fF = to.fY = NEG;
}

// One wave sweeps blocks of 8 anti-diagonals from r0 with K slots per lane,
// lane 0 at diagonal `base`, up to the block starting at r_stop. Returns
// true when the pair has ended (last anti-diagonal or z-drop); else false
// with r0 = r_stop. The rings are staged afresh for this layout. (The stop
// is worked out before the sweep: one scalar is all the loop carries beyond
// the one-layout sweep's state.)
template <int K>
__device__ __forceinline__ bool sweep_window(PairState<K> &st, const DpArgs &P, Geo &g, Track &tr, int &r0,
                                             int base, int lane, PairLds<K, 1> &S, int p, int r_stop) {
    g.a0w = base;
    int wall_pos = 0;
    uint64_t wall_lanes = 0;
    place_wall<K>(g, wall_pos, wall_lanes);
    uint32_t *ring_t = S.ring[0][0], *ring_q = S.ring[0][1];
    if (lane == 0) {
        const int64_t to = P.t_off[p], qo = P.q_off[p];
        S.src[0][0] = SeqSource{P.tw + to, P.tn, 16 * to, g.n};
        S.src[0][1] = SeqSource{P.qw + qo, P.qn, 16 * qo, g.m};
    }
    __builtin_amdgcn_wave_barrier();
    int ft = -(1 << 30), fq = -(1 << 30);
    stage_block<K>(g, ring_t, ring_q, S.src[0], ft, fq, r0, base, lane);
    Windows<K> wd;
    load_windows<K>(wd, ring_t, ring_q, r0, base + lane * K);
    for (;;) {
        build_scores<K>(st, wd, P);
        stage_block<K>(g, ring_t, ring_q, S.src[0], ft, fq, r0 + 8, base, lane);
        load_windows<K>(wd, ring_t, ring_q, r0 + 8, base + lane * K);  // next block, in flight
        if (run_block1<K>(st, P, g, tr, r0, lane, wall_lanes, wall_pos, S)) return true;
        r0 += 8;
        if (r0 >= r_stop) return false;
    }
}

// A pair of the one-wave class KB whose triangles run with KT slots per
// lane. The narrow window's lane 0 sits at bs (start) or be (end), at most
// 64*(KB-KT) above a0, so the window lies inside the wide one.
template <int KB, int KT>
__device__ void align_pair_split(const DpArgs &P, int p, int lane, SplitLds<KB, KT> &U) {
    static_assert(KT < KB && KT % 2 == 0, "the narrow layout has fewer slots, whole slot pairs");
    Geo g;
    pair_geo(P, p, g);
    const int a0 = g.a0, a1 = g.a1;
    constexpr int CAP = WAVE * KT;           // diagonals of the narrow window
    constexpr int SPAN = WAVE * (KB - KT);  // its highest start above a0
    int *stage = U.wide.park;
    // start window: centred on diagonal 0 (or ending at the band's top),
    // at or above a0 and of a0's parity, like every layout's slot 0
    int bs = min(-CAP / 2, a1 + 1 - CAP);
    bs = min(max(bs, a0), a0 + SPAN);
    bs -= (bs - a0) & 1;
    // the block from anti-diagonal r fits it when the boundary cells of its
    // last anti-diagonal (diagonals -(r+9), r+9) do, or the band edge comes
    // first: r <= r_fit
    constexpr int NEVER = 1 << 30;
    const int r_fit = min(bs == a0 ? NEVER : -bs - 9, a1 <= bs + CAP - 1 ? NEVER : bs + CAP - 10);
    // end window for the block from r: the state holds anti-diagonals r-2
    // and r-1, whose finite cells lie in [lo, hi] and never leave it later
    // (boundary cells while any is in the band, else the interior cells).
    // Cells of r-1 leaving the rectangle, still to be clamped, may fall
    // outside: they start at -inf there, as the clamp would leave them.
    // [lo, hi] only shrinks as r grows, so once a block fits, all later do.
    auto end_base = [&](int r, int &be) {
        const int lo = (-r >= a0) ? a0 : max(g.dlo, r - 2 * g.m);
        const int hi = (r <= a1) ? a1 : min(g.dhi, 2 * g.n - r);
        be = min(lo - ((lo - a0) & 1), a0 + SPAN);
        return hi <= be + CAP - 1;
    };
    // G = 0 at the origin, in the frame of anti-diagonal -1
    Track tr{0, -1, -1, 0, -1, -1, 0, -1, 0, -P.q1 - P.e1, false, false, -P.q1 - P.e1, -1};
    int r0 = (a0 & 1) ? -1 : -2;
    PairState<KB> sw;
    if (r0 <= r_fit) {
        PairState<KT> sn;
        init_state<KT>(sn, P, g, bs + lane * KT);
        const int r_stop = r0 + 8 * ((r_fit - r0) / 8 + 1);  // first block past r_fit
        if (sweep_window<KT>(sn, P, g, tr, r0, bs, lane, U.narrow, p, r_stop)) {
            write_result<KT>(P, p, tr, g, U.narrow, lane);
            return;
        }
        settle_max<KT>(tr, g, U.narrow, lane);
        move_state<KT, KB>(sn, sw, stage, bs - a0, 0, lane);
    } else {
        init_state<KB>(sw, P, g, a0 + lane * KB);
    }
    int be = a0;
    if (!end_base(r0, be)) {
        // the first block whose state fits the end window: the block from
        // r_last + 2 holds only the last anti-diagonal's single cell, so it
        // fits; binary search between
        int klo = 1, khi = (g.r_last + 2 - r0 + 7) / 8;
        int tmp;
        while (klo < khi) {
            const int k = (klo + khi) >> 1;
            if (end_base(r0 + 8 * k, tmp))
                khi = k;
            else
                klo = k + 1;
        }
        if (sweep_window<KB>(sw, P, g, tr, r0, a0, lane, U.wide, p, r0 + 8 * klo)) {
            write_result<KB>(P, p, tr, g, U.wide, lane);
            return;
        }
        settle_max<KB>(tr, g, U.wide, lane);
        end_base(r0, be);
    }
    PairState<KT> se;
    move_state<KB, KT>(sw, se, stage, 0, be - a0, lane);
    sweep_window<KT>(se, P, g, tr, r0, be, lane, U.narrow, p, NEVER);
    write_result<KT>(P, p, tr, g, U.narrow, lane);
}

// Waves per SIMD each kernel is compiled for (its register budget: 512 per
// SIMD lane over the resident waves). The one-wave K=32 kernel fits two
// waves in 256 registers only with the iterative ILP scheduler the library
// is built with (252); the default one left it at one wave per SIMD, its
// excess in accumulation registers.
template <int K, int NW, bool SL>
struct Occ {
    static constexpr int value = K <= 8 ? 4 : (K <= 16 ? 3 : 2);
};

// Each workgroup of NW waves takes pairs of its group from the list through
// an atomic head until the group is exhausted: persistent (a grid of
// resident workgroups over a cost-ordered list) or one workgroup per pair
// (the bucketed schedule).
// KT > 0: one-wave fixed class whose start and end triangles run with KT
// slots per lane (align_pair_split).
template <int K, int NW, bool SL, int KT>
__global__ __launch_bounds__(WAVE * NW, (Occ<K, NW, SL>::value)) void ga_dp_kernel(DpArgs P) {
    static_assert(!SL || NW == 1, "a sliding window runs on one wave");
    static_assert(KT == 0 || (NW == 1 && !SL), "narrow triangles on one fixed wave");
    __shared__ std::conditional_t<(KT > 0), SplitLds<K, KT>, PairLds<K, NW>> S;
    // lane-shift staging of a sliding window: two -inf rows on each side
    __shared__ __align__(16) int rows[SL ? (WAVE + 4) * K : 4];
    const int lane = threadIdx.x & (WAVE - 1);
    if constexpr (SL) {
        if (lane < 2 * K) {
            rows[lane] = NEG;
            rows[(WAVE + 2) * K + lane] = NEG;
        }
    }
    const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int count = P.counters[CNT_COUNT + P.group];
    const int32_t *list = P.list + P.counters[CNT_START + P.group];
    for (;;) {
        int idx = 0;
        if constexpr (NW == 1) {
            if (lane == 0) idx = atomicAdd(&P.counters[CNT_HEAD + P.group], 1);
            idx = __builtin_amdgcn_readfirstlane(idx);
        } else {
            if (threadIdx.x == 0) S.idx = atomicAdd(&P.counters[CNT_HEAD + P.group], 1);
            __syncthreads();
            idx = __builtin_amdgcn_readfirstlane(S.idx);
            __syncthreads();  // every wave has read S.idx before the next pair overwrites it
        }
        if (idx >= count) break;
        const int p = list[idx];
        if constexpr (KT > 0)
            align_pair_split<K, KT>(P, p, lane, S);
        else
            align_pair<K, NW, SL>(P, p, lane, wv, S, rows);
    }
}

// Integer VALU peak probe: every lane runs CAL_CHAINS independent chains of
// v_max3_i32 / v_add_u32 pairs (inline asm, so nothing folds), enough
// independent work per wave to hide issue latency. One lane-op per
// instruction per lane.
constexpr int CAL_CHAINS = 8;
constexpr int CAL_WAVES_PER_SIMD = 8;

__global__ __launch_bounds__(256) void ga_valu_probe(int32_t iters, int32_t *sink) {
    int a[CAL_CHAINS];
#pragma unroll
    for (int k = 0; k < CAL_CHAINS; ++k) a[k] = (int)threadIdx.x + k;
    const int x = (int)blockIdx.x, y = -(int)threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < CAL_CHAINS; ++k) {
            asm volatile("v_max3_i32 %0, %0, %1, %2" : "+v"(a[k]) : "v"(x), "v"(y));
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[k]) : "v"(x));
        }
    }
    int acc = 0;
#pragma unroll
    for (int k = 0; k < CAL_CHAINS; ++k) acc ^= a[k];
    if (acc == 0x7fffffff) sink[0] = acc;  // keeps the chains live; practically never stores
}

__global__ void ga_zero_i32(int32_t *x, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

// Work planning. A wave's time on a pair is proportional to the number of
// anti-diagonals it sweeps, whatever the band's occupancy, so pairs are
// ordered by n + m, longest first, within each slot class: the persistent
// waves then finish on short pairs instead of waiting on one long straggler.
// Counting sort over cost buckets of PLAN_SHIFT anti-diagonals: classify and
// histogram, an exclusive scan in descending bucket order, then a scatter.
constexpr int PLAN_BUCKETS = 4096;  // per group; the last bucket takes every longer pair
constexpr int PLAN_SHIFT = 5;
constexpr int PLAN_BINS = NGROUP * PLAN_BUCKETS;

struct PlanArgs {
    int64_t n_pairs;
    const int64_t *t_off, *q_off;
    const int32_t *t_len, *q_len;
    int64_t t_nwords, q_nwords;
    int32_t max_len;
    int32_t w;
    int32_t bucketed;  // schedule: 0 persistent, 1 bucketed
    int32_t ordered;   // persistent: order each class longest first
    uint32_t mask;     // kernel classes allowed
    uint64_t order;    // the order classes are tried in (class_for)
    int32_t *counters;
    int32_t *hist;    // [PLAN_BINS] pairs per (group, cost bucket)
    int32_t *cursor;  // [PLAN_BINS] next list position per (group, cost bucket)
    int32_t *keys;    // [n_pairs] group * PLAN_BUCKETS + cost bucket, or -1 when finished here
    int32_t *lists;   // [n_pairs] the pairs, grouped
    int32_t *err;
    ga_result_t *out;
};

// Add 1 to ctr[key] for every lane of the wave with key >= 0, with one
// atomic per distinct key in the wave (a batch's pairs crowd into few
// (class, cost bucket) keys, and contended atomics on one address
// serialise). Returns, for such a lane, the counter's old value plus the
// lane's rank among the wave's lanes with its key, so the values handed out
// are distinct. Every lane of the wave must take part.
__device__ __forceinline__ int wave_counter_inc(int32_t *ctr, int key) {
    const int lane = __lane_id();
    uint64_t todo = __ballot(key >= 0);
    int pos = -1;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int k = __shfl(key, leader);
        const uint64_t same = __ballot(key == k) & todo;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctr[k], (int)__popcll(same));
        base = __shfl(base, leader);
        if ((same >> lane) & 1ull) pos = base + (int)__popcll(same & ((1ull << lane) - 1ull));
        todo &= ~same;
    }
    return pos;
}

// Validate each pair, finish invalid and empty pairs, and give the rest a
// (group, cost bucket) key. Persistent schedule: the group is the cheapest
// class that runs the pair (class_for) and the cost bucket orders each group
// longest first. Bucketed schedule: the group is the power-of-two bucket of
// max(n, m), with no ordering inside it. The key of pair p is -1 when the
// pair is finished here (invalid, empty or held by no allowed class; its
// result is written).
__device__ __forceinline__ int plan_key(const PlanArgs &A, int64_t p) {
    const int32_t n = A.t_len[p], m = A.q_len[p];
    const int64_t to = A.t_off[p], qo = A.q_off[p];
    const bool bad = n < 0 || m < 0 || n > A.max_len || m > A.max_len || to < 0 || qo < 0 ||
                     to + (n + 15) / 16 > A.t_nwords || qo + (m + 15) / 16 > A.q_nwords;
    int key = -1;
    if (bad) {
        atomicOr(A.err, 1);
        A.out[p] = ga_result_t{0, -1, -1, 0, -1, -1, -1};
    } else if (n == 0 || m == 0) {
        A.out[p] = ga_result_t{0, -1, -1, 0, -1, -1, 0};
    } else {
        int group, bucket = 0;
        if (A.bucketed) {
            group = 32 - __clz((unsigned)max(n, m));  // max(n, m) < 2^group
            if (bucket_class(group, A.w, A.mask) < 0) group = -1;
        } else {
            int slide;
            group = class_for(n, m, A.w, &slide, A.mask, A.order);
            bucket = A.ordered ? min((n + m) >> PLAN_SHIFT, PLAN_BUCKETS - 1) : 0;
        }
        if (group < 0) {
            atomicOr(A.err, 2);
            A.out[p] = ga_result_t{0, -1, -1, 0, -1, -1, -1};
        } else {
            key = group * PLAN_BUCKETS + bucket;
        }
    }
    return key;
}

__global__ void ga_plan_classify(PlanArgs A) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int key = -1;
    if (p < A.n_pairs) {
        key = plan_key(A, p);
        A.keys[p] = key;
    }
    wave_counter_inc(A.hist, key);
}

// One workgroup of 1024 threads: list positions of every (group, cost
// bucket), groups in order and cost buckets descending inside a group
// (exclusive scan), and the groups' sizes and starts.
__global__ __launch_bounds__(1024) void ga_plan_scan(PlanArgs A) {
    constexpr int PER = PLAN_BUCKETS / 1024;  // buckets per thread, in descending order
    __shared__ int part[1024];
    const int t = threadIdx.x;
    int start = 0;
    for (int c = 0; c < NGROUP; ++c) {
        const int *h = A.hist + c * PLAN_BUCKETS;
        // thread t owns descending ranks t*PER .. t*PER+PER-1, i.e. buckets B-1-rank
        int v[PER], sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            v[k] = h[PLAN_BUCKETS - 1 - (t * PER + k)];
            sum += v[k];
        }
        part[t] = sum;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int x = t >= d ? part[t - d] : 0;
            __syncthreads();
            part[t] += x;
            __syncthreads();
        }
        int run = start + part[t] - sum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            A.cursor[c * PLAN_BUCKETS + PLAN_BUCKETS - 1 - (t * PER + k)] = run;
            run += v[k];
        }
        const int total = part[1023];
        if (t == 1023) {
            A.counters[CNT_COUNT + c] = total;
            A.counters[CNT_START + c] = start;
        }
        start += total;
        __syncthreads();
    }
}

__global__ void ga_plan_scatter(PlanArgs A) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int key = p < A.n_pairs ? A.keys[p] : -1;
    const int pos = wave_counter_inc(A.cursor, key);
    if (key >= 0) A.lists[pos] = (int32_t)p;
}

// ---- packing: ASCII -> 2-bit stream + N bitmap (input packing, Section 2.2)

__global__ void ga_word_counts(const int32_t *len, int64_t n, int64_t *cnt) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) cnt[p] = (len[p] > 0 ? (int64_t)len[p] + 15 : 0) / 16;
}

// In-place exclusive prefix sum of x[0..n) by one workgroup of 1024 threads;
// total[0] receives the sum.
__global__ __launch_bounds__(1024) void ga_exclusive_scan(int64_t *x, int64_t n, int64_t *total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t lo = t * chunk, hi = min(n, lo + chunk);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += x[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;  // exclusive prefix of this chunk
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t v = x[i];
        x[i] = run;
        run += v;
    }
    if (t == 1023) total[0] = part[1023];
}

__device__ __forceinline__ uint32_t base2bit(uint8_t c, bool &is_n) {
    switch (c) {
    case 'A': case 'a': is_n = false; return 0;
    case 'C': case 'c': is_n = false; return 1;
    case 'G': case 'g': is_n = false; return 2;
    case 'T': case 't': is_n = false; return 3;
    default: is_n = true; return 0;
    }
}

// One workgroup per sequence; thread per output word.
__global__ void ga_pack_kernel(const uint8_t *ascii, const int64_t *off, const int32_t *len,
                               const int64_t *word_off, int64_t nwords, uint32_t *words,
                               uint32_t *nmask, int32_t *err) {
    const int64_t p = blockIdx.x;
    const int32_t L = len[p];
    const int64_t wo = word_off[p];
    const int64_t nw = L > 0 ? ((int64_t)L + 15) / 16 : 0;
    const uint8_t *src = ascii + off[p];
    for (int64_t k = threadIdx.x; k < nw; k += blockDim.x) {
        const int64_t gw = wo + k;
        if (gw < 0 || gw >= nwords) {
            atomicOr(err, 4);
            continue;
        }
        uint32_t v = 0, nb = 0;
        const uint8_t *s16 = src + 16 * k;
        if (16 * k + 16 <= L && (reinterpret_cast<uintptr_t>(s16) & 15) == 0) {
            // a whole word of bases at an aligned address: one 16-byte load
            // (one bus transaction when the bytes sit in host memory)
            const uint4 q = *reinterpret_cast<const uint4 *>(s16);
            const uint32_t w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                bool is_n;
                v |= base2bit((uint8_t)(w4[b >> 2] >> (8 * (b & 3))), is_n) << (2 * b);
                nb |= (is_n ? 1u : 0u) << b;
            }
        } else {
            for (int b = 0; b < 16; ++b) {
                const int64_t pos = 16 * k + b;
                if (pos >= L) break;
                bool is_n;
                v |= base2bit(s16[b], is_n) << (2 * b);
                nb |= (is_n ? 1u : 0u) << b;
            }
        }
        words[gw] = v;
        if (nb) atomicOr(&nmask[gw >> 1], nb << (16 * (gw & 1)));
    }
}

// Probe pairs for the autotuner: pair p has a target of n random bases and
// a query of m bases copying the target's first m with about one
// substitution in 16 (no N). Bases come from an integer hash of the pair,
// word and base indices (the lowbias32 mixer of C. Wellons).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void ga_probe_fill(int64_t n_pairs, int32_t n, int32_t m, uint32_t *t_words, uint32_t *q_words,
                              int64_t *t_off, int64_t *q_off, int32_t *t_len, int32_t *q_len) {
    const int64_t tw = ((int64_t)n + 15) / 16, qw = ((int64_t)m + 15) / 16;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n_pairs * tw) return;
    const int64_t p = idx / tw, k = idx % tw;
    const uint32_t v = mix32((uint32_t)p * 0x9e3779b9u ^ mix32((uint32_t)k + 0x5bd1e995u));
    t_words[idx] = v;
    if (k < qw) {
        uint32_t x = 0;
        for (int b = 0; b < 16; ++b) {
            const uint32_t h = mix32(v ^ ((uint32_t)b * 0x27d4eb2fu) ^ (uint32_t)k);
            if ((h & 15u) == 0) x |= (1u + (h >> 4) % 3u) << (2 * b);
        }
        q_words[p * qw + k] = v ^ x;
    }
    if (k == 0) {
        t_off[p] = p * tw;
        q_off[p] = p * qw;
        t_len[p] = n;
        q_len[p] = m;
    }
}

// Layout of one call's planning workspace for n pairs: the counters, the
// histogram and cursors of the cost buckets (cleared or written by the
// planning kernels on every call), one key and one list entry per pair.
constexpr size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
constexpr size_t WS_HIST = round_up(sizeof(int32_t) * CNT_WORDS, 256);
constexpr size_t WS_CURSOR = WS_HIST + sizeof(int32_t) * PLAN_BINS;
constexpr size_t WS_KEYS = WS_CURSOR + sizeof(int32_t) * PLAN_BINS;
constexpr size_t ws_lists(size_t n) { return round_up(WS_KEYS + sizeof(int32_t) * n, 256); }
constexpr size_t ws_bytes(size_t n) { return ws_lists(n) + sizeof(int32_t) * n; }

}  // namespace

// --------------------------------------------------------------- host side

// The allocation-free entry point's workspace (ga_align_batch_noalloc): one
// call's planning workspace for up to GA_NOALLOC_MAX_PAIRS pairs (about
// 9 MiB), a file-scope device array of which each GPU holds its own copy
// until the process ends. Host code never uses the array's name as an
// address: ga_context_create looks up this device's copy once
// (hipGetSymbolAddress, with the device current) and every later use goes
// through that pointer.
static __device__ __align__(256) unsigned char scratch[ws_bytes(GA_NOALLOC_MAX_PAIRS)];
constexpr int SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[SCRATCH_DEVICES];  // this device's copy of `scratch`, once looked up

// Stage events of a timed call: start, end of planning, then a start and
// an end per launch (recorded on the stream the launch runs on).
constexpr int NEVENTS = 2 + 2 * NGROUP;
// The persistent launches run on up to four streams at once (the caller's
// and three of the context's), joined back into the caller's stream. A
// launch holds its stream until its last pair ends, so the class holding
// the band's full width (2w + 1 diagonals, where the longest pairs of a
// batch land) launches first, on lane 0, ahead of everything: its longest
// pairs start at once and nothing waits behind them. The other classes
// spread over lanes 1-3 so the heavy classes of a mixed batch (sliding K=4
// and K=8, K=4, K=16) land on different streams, the multi-wave classes
// first on each (usually empty, they end at once instead of waiting behind
// a full grid of another class for the resources of their wide
// workgroups).
constexpr int MAX_LANES = 4;
constexpr int LANE_OF[NCLASS] = {3, 2, 3, 0, 1, 2, 3, 1, 2, 3, 3, 1, 2, 1, 3};
constexpr int LAUNCH_ORDER[NCLASS] = {10, 9, 8, 7, 14, 12, 13, 0, 1, 2, 3, 4, 5, 6, 11};

struct ga_context {
    int device;
    int num_cu;
    int blocks_per_cu[NCLASS];  // resident workgroups of each slot class's kernel per CU
    void *ws;          // workspace
    size_t ws_size;
    int32_t *d_err;    // device error latch
    int timing;        // record stage events in ga_align_batch
    int timed_last;    // the last ga_align_batch recorded them
    int schedule;      // GA_SCHED_*
    uint32_t class_mask;  // kernel classes the planner may use
    uint64_t class_order; // the order the planner tries them in (autotune table)
    float class_cost[NCLASS];  // measured ns per pair and anti-diagonal (0: not tuned)
    float class_lat[NCLASS];   // measured ns per anti-diagonal of one pair in a small batch
    uint64_t order_lat;        // the classes by that latency, for batches of up to lat_pairs pairs
    int lat_pairs;             // 0: no latency order (not tuned)
    int n_launch_last;              // launches of the last timed call
    int lanes;                      // streams the persistent launches spread over
    hipStream_t side[MAX_LANES - 1];
    hipEvent_t fork_ev, join_ev[MAX_LANES - 1];
    int launch_class[NGROUP];       // their kernel classes
    int32_t *h_counts;              // pinned host copy of the group sizes (bucketed schedule)
    hipEvent_t ev[NEVENTS];
    void *scratch;                  // this device's copy of `scratch` (null: not available)
};

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int ensure_ws(ga_context *ctx, size_t need) {
    if (ctx->ws_size >= need) return GA_OK;
    if (ctx->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    size_t sz = align_up(need + need / 4, 1 << 20);
    if (hipMalloc(&ctx->ws, sz) != hipSuccess) {
        (void)hipGetLastError();
        return GA_ENOMEM;
    }
    ctx->ws_size = sz;
    return GA_OK;
}

// Makes `dev` current for the scope of a call; touches the device setting
// only when another device is current.
struct SetDevice {
    int prev = -1;
    bool changed = false;
    explicit SetDevice(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~SetDevice() {
        if (changed && prev >= 0) hipSetDevice(prev);
    }
};

template <int K, int NW, bool SL, int KT = 0>
void launch_dp(const DpArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((ga_dp_kernel<K, NW, SL, KT>), dim3(grid), dim3(WAVE * NW), 0, s, a);
}

void launch_class(int c, const DpArgs &a, int grid, hipStream_t s) {
    switch (c) {
    case 0: launch_dp<4, 1, false>(a, grid, s); break;
    case 1: launch_dp<8, 1, false>(a, grid, s); break;
    case 2: launch_dp<16, 1, false, TRI_K16>(a, grid, s); break;
    case 3: launch_dp<24, 1, false, TRI_K24>(a, grid, s); break;
    case 4: launch_dp<32, 1, false>(a, grid, s); break;
    case 5: launch_dp<8, 1, true>(a, grid, s); break;
    case 6: launch_dp<16, 1, true>(a, grid, s); break;
    case 7: launch_dp<24, 2, false>(a, grid, s); break;
    case 8: launch_dp<32, 2, false>(a, grid, s); break;
    case 9: launch_dp<32, 3, false>(a, grid, s); break;
    case 10: launch_dp<32, 4, false>(a, grid, s); break;
    case 11: launch_dp<4, 1, true>(a, grid, s); break;
    case 12: launch_dp<8, 2, false>(a, grid, s); break;
    case 13: launch_dp<4, 2, false>(a, grid, s); break;
    default: launch_dp<4, 4, false>(a, grid, s); break;
    }
}

template <int K, int NW, bool SL, int KT = 0>
int blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ga_dp_kernel<K, NW, SL, KT>, WAVE * NW, 0) != hipSuccess) {
        (void)hipGetLastError();
        nb = 0;
    }
    return nb > 0 ? nb : 1;
}

}  // namespace

extern "C" {

const char *ga_strerror(int code) {
    switch (code) {
    case GA_OK: return "ok";
    case GA_EINVAL: return "invalid argument (null pointer, negative size or parameter, or range guard)";
    case GA_ENOMEM: return "device workspace allocation failed";
    case GA_EHIP: return "HIP launch or runtime error";
    case GA_EUNSUPPORTED: return "parameters outside what the kernels implement";
    case GA_EDEVICE: return "a device-side check failed (pair outside the declared bounds)";
    default: return "unknown error";
    }
}

int ga_context_create(ga_context_t **out, int device) {
    if (!out) return GA_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return GA_EINVAL;
    }
    SetDevice sd(device);
    ga_context *ctx = (ga_context *)calloc(1, sizeof(ga_context));
    if (!ctx) return GA_ENOMEM;
    ctx->device = device;
    ctx->class_mask = ALL_CLASSES;
    ctx->class_order = DEFAULT_ORDER;
    ctx->lanes = MAX_LANES;
    if (hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        ctx->num_cu = 256;
    // persistent grids: as many workgroups as the registers let reside
    ctx->blocks_per_cu[0] = blocks_per_cu<4, 1, false>();
    ctx->blocks_per_cu[1] = blocks_per_cu<8, 1, false>();
    ctx->blocks_per_cu[2] = blocks_per_cu<16, 1, false, TRI_K16>();
    ctx->blocks_per_cu[3] = blocks_per_cu<24, 1, false, TRI_K24>();
    ctx->blocks_per_cu[4] = blocks_per_cu<32, 1, false>();
    ctx->blocks_per_cu[5] = blocks_per_cu<8, 1, true>();
    ctx->blocks_per_cu[6] = blocks_per_cu<16, 1, true>();
    ctx->blocks_per_cu[7] = blocks_per_cu<24, 2, false>();
    ctx->blocks_per_cu[8] = blocks_per_cu<32, 2, false>();
    ctx->blocks_per_cu[9] = blocks_per_cu<32, 3, false>();
    ctx->blocks_per_cu[10] = blocks_per_cu<32, 4, false>();
    ctx->blocks_per_cu[11] = blocks_per_cu<4, 1, true>();
    ctx->blocks_per_cu[12] = blocks_per_cu<8, 2, false>();
    ctx->blocks_per_cu[13] = blocks_per_cu<4, 2, false>();
    ctx->blocks_per_cu[14] = blocks_per_cu<4, 4, false>();
    if (hipMalloc(&ctx->d_err, sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        free(ctx);
        return GA_ENOMEM;
    }
    if (hipMemset(ctx->d_err, 0, sizeof(int32_t)) != hipSuccess) {
        hipFree(ctx->d_err);
        free(ctx);
        return GA_EHIP;
    }
    // this device's copy of the allocation-free entry point's scratch
    if (device < SCRATCH_DEVICES) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_dev[device]) {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
                (void)hipGetLastError();
                ptr = nullptr;
            }
            g_scratch_dev[device] = ptr;
        }
        ctx->scratch = g_scratch_dev[device];
    }
    *out = ctx;
    return GA_OK;
}

int ga_context_destroy(ga_context_t *ctx) {
    if (!ctx) return GA_EINVAL;
    SetDevice sd(ctx->device);
    hipDeviceSynchronize();
    if (ctx->ev[0])
        for (int k = 0; k < NEVENTS; ++k) hipEventDestroy(ctx->ev[k]);
    for (int k = 0; k < MAX_LANES - 1; ++k) {
        if (ctx->side[k]) hipStreamDestroy(ctx->side[k]);
        if (ctx->join_ev[k]) hipEventDestroy(ctx->join_ev[k]);
    }
    if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
    if (ctx->ws) hipFree(ctx->ws);
    if (ctx->d_err) hipFree(ctx->d_err);
    if (ctx->h_counts) hipHostFree(ctx->h_counts);
    free(ctx);
    return GA_OK;
}

int ga_context_check(ga_context_t *ctx, void *stream) {
    if (!ctx) return GA_EINVAL;
    SetDevice sd(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) return GA_EHIP;
    int32_t flag = 0;
    if (hipMemcpy(&flag, ctx->d_err, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) return GA_EHIP;
    if (flag) {
        if (hipMemset(ctx->d_err, 0, sizeof(int32_t)) != hipSuccess) return GA_EHIP;
        return GA_EDEVICE;
    }
    return GA_OK;
}

int ga_context_set_timing(ga_context_t *ctx, int enable) {
    if (!ctx) return GA_EINVAL;
    SetDevice sd(ctx->device);
    if (enable && !ctx->ev[0]) {
        for (int k = 0; k < NEVENTS; ++k)
            if (hipEventCreate(&ctx->ev[k]) != hipSuccess) return GA_EHIP;
    }
    ctx->timing = enable ? 1 : 0;
    return GA_OK;
}

int ga_context_timing(ga_context_t *ctx, float *ms, int n) {
    if (!ctx || !ms || n < 1) return GA_EINVAL;
    if (!ctx->timed_last) return GA_EINVAL;
    SetDevice sd(ctx->device);
    for (int l = 0; l < ctx->n_launch_last; ++l)
        if (hipEventSynchronize(ctx->ev[3 + 2 * l]) != hipSuccess) return GA_EHIP;
    if (hipEventSynchronize(ctx->ev[1]) != hipSuccess) return GA_EHIP;
    for (int k = 0; k < n; ++k) ms[k] = 0.f;
    float t = 0.f;
    if (hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]) != hipSuccess) return GA_EHIP;
    ms[0] = t;
    for (int l = 0; l < ctx->n_launch_last; ++l) {
        if (hipEventElapsedTime(&t, ctx->ev[2 + 2 * l], ctx->ev[3 + 2 * l]) != hipSuccess) return GA_EHIP;
        const int c = ctx->launch_class[l];
        if (1 + c < n) ms[1 + c] += t;
    }
    return GA_OK;
}

int ga_context_set_schedule(ga_context_t *ctx, int schedule) {
    if (!ctx || (schedule != GA_SCHED_PERSISTENT && schedule != GA_SCHED_BUCKETED &&
                 schedule != GA_SCHED_UNORDERED))
        return GA_EINVAL;
    ctx->schedule = schedule;
    return GA_OK;
}

int ga_host_device_pointer(void *host, void **dev) {
    if (!host || !dev) return GA_EINVAL;
    *dev = nullptr;
    if (hipHostGetDevicePointer(dev, host, 0) != hipSuccess) {
        (void)hipGetLastError();
        *dev = nullptr;
        return GA_EINVAL;
    }
    return GA_OK;
}

int ga_context_set_lanes(ga_context_t *ctx, int lanes) {
    if (!ctx || lanes < 1 || lanes > MAX_LANES) return GA_EINVAL;
    ctx->lanes = lanes;
    return GA_OK;
}

int ga_context_set_classes(ga_context_t *ctx, uint32_t mask) {
    if (!ctx || mask == 0 || (mask & ~ALL_CLASSES) != 0) return GA_EINVAL;
    ctx->class_mask = mask;
    return GA_OK;
}

int ga_context_pair_class(const ga_context_t *ctx, int32_t n, int32_t m, int32_t w) {
    if (!ctx || n <= 0 || m <= 0) return -1;
    int slide;
    return class_for(n, m, w, &slide, ctx->class_mask, ctx->class_order);
}

// Anti-diagonals a full sweep of an (n, m) pair at band w visits (the last
// one with an interior cell, plus one), as the kernels' geometry has it.
static int64_t sweep_steps(int64_t n, int64_t m, int64_t w) {
    const int64_t a0 = w >= 0 ? (-w > -m ? -w : -m) : -m;
    const int64_t a1 = w >= 0 ? (w < n ? w : n) : n;
    const int64_t dlo = a0 > 1 - m ? a0 : 1 - m;
    const int64_t dhi = a1 < n - 1 ? a1 : n - 1;
    int64_t dc = n - m;
    if (dc < dlo) dc = dlo;
    if (dc > dhi) dc = dhi;
    const int64_t x = 2 * n - 2 - dc, y = 2 * m - 2 + dc;
    return (x < y ? x : y) + 1;
}

}  // extern "C"

namespace {

// Pairs of the autotuner's latency probe (each alone on its CU).
constexpr int LAT_PROBE = 64;

// The class order a call of n_pairs pairs plans with: by measured latency
// for a batch too small to fill the GPU (its time is its longest sweep),
// else by throughput cost.
uint64_t batch_order(const ga_context *ctx, int64_t n_pairs) {
    return ctx->lat_pairs > 0 && n_pairs <= ctx->lat_pairs ? ctx->order_lat : ctx->class_order;
}

// The classes ordered by a measured cost, cheapest first (insertion sort;
// ties keep the default order), as order nibbles.
uint64_t order_by(const float *cost) {
    int ord[NCLASS];
    for (int k = 0; k < NCLASS; ++k) ord[k] = (int)((DEFAULT_ORDER >> (4 * k)) & 0xFull);
    for (int k = 1; k < NCLASS; ++k)
        for (int j = k; j > 0 && cost[ord[j]] < cost[ord[j - 1]]; --j) {
            const int t = ord[j];
            ord[j] = ord[j - 1];
            ord[j - 1] = t;
        }
    uint64_t order = 0;
    for (int k = 0; k < NCLASS; ++k) order |= (uint64_t)ord[k] << (4 * k);
    return order;
}

}  // namespace

extern "C" {

int ga_context_autotune(ga_context_t *ctx, float *ns_per_step, int n_out, void *stream) {
    if (!ctx || n_out < 0 || (n_out > 0 && !ns_per_step)) return GA_EINVAL;
    SetDevice sd(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const uint32_t mask0 = ctx->class_mask;
    const int sched0 = ctx->schedule, timing0 = ctx->timing;
    ctx->schedule = GA_SCHED_PERSISTENT;
    ctx->class_order = DEFAULT_ORDER;
    int rc = ga_context_set_timing(ctx, 1);
    const ga_scoring_t sc{2, 4, 4, 2, 24, 1, 1};
    float cost[NCLASS], lat[NCLASS];
    ctx->lat_pairs = 0;
    for (int c = 0; c < NCLASS && rc == GA_OK; ++c) {
        // a probe each class runs in the shape the cheapest-first rule gives it
        const int K = class_k(c), cap = class_cap(c);
        int n, m, w;
        if (class_slides(c)) {
            m = (cap - 11 - K) / 2 - 4;  // the short side's span fits the window
            n = 8 * cap;
            w = 2 * cap;                 // the band does not
        } else {
            const int lo = WAVE * K * (class_nw(c) - 1);
            const int D = lo + (cap - lo) * 7 / 8;
            w = (D - 1) / 2;
            n = m = 2 * w + 1024;
        }
        const int64_t pairs = 2 * (int64_t)ctx->blocks_per_cu[c] * ctx->num_cu;
        const int64_t tw = ((int64_t)n + 15) / 16, qw = ((int64_t)m + 15) / 16;
        char *buf = nullptr;
        const size_t o_q = align_up(sizeof(uint32_t) * pairs * tw, 256);
        const size_t o_to = o_q + align_up(sizeof(uint32_t) * pairs * qw, 256);
        const size_t o_qo = o_to + align_up(sizeof(int64_t) * pairs, 256);
        const size_t o_tl = o_qo + align_up(sizeof(int64_t) * pairs, 256);
        const size_t o_ql = o_tl + align_up(sizeof(int32_t) * pairs, 256);
        const size_t o_out = o_ql + align_up(sizeof(int32_t) * pairs, 256);
        const size_t total = o_out + sizeof(ga_result_t) * pairs;
        if (hipMalloc(&buf, total) != hipSuccess) {
            (void)hipGetLastError();
            rc = GA_ENOMEM;
            break;
        }
        ga_batch_t bt{};
        bt.n_pairs = pairs;
        bt.t_words_dev = (const uint32_t *)buf;
        bt.t_nwords = pairs * tw;
        bt.q_words_dev = (const uint32_t *)(buf + o_q);
        bt.q_nwords = pairs * qw;
        bt.t_off_dev = (const int64_t *)(buf + o_to);
        bt.q_off_dev = (const int64_t *)(buf + o_qo);
        bt.t_len_dev = (const int32_t *)(buf + o_tl);
        bt.q_len_dev = (const int32_t *)(buf + o_ql);
        bt.max_len = n > m ? n : m;
        const int64_t nthr = pairs * tw;
        hipLaunchKernelGGL(ga_probe_fill, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, pairs, n, m,
                           (uint32_t *)buf, (uint32_t *)(buf + o_q), (int64_t *)(buf + o_to),
                           (int64_t *)(buf + o_qo), (int32_t *)(buf + o_tl), (int32_t *)(buf + o_ql));
        ctx->class_mask = 1u << c;
        float ms[1 + NCLASS] = {};
        for (int rep = 0; rep < 2 && rc == GA_OK; ++rep)  // the first run warms up
            rc = ga_align_batch(ctx, &bt, &sc, w, -1, (ga_result_t *)(buf + o_out), s);
        if (rc == GA_OK) rc = ga_context_timing(ctx, ms, 1 + NCLASS);
        if (rc == GA_OK) rc = ga_context_check(ctx, s);
        const double steps = (double)sweep_steps(n, m, w);
        cost[c] = (float)(ms[1 + c] * 1e6 / ((double)pairs * steps));
        // latency: a batch of LAT_PROBE pairs, each alone on its CU, times
        // one pair's sweep
        bt.n_pairs = LAT_PROBE;
        float ml[1 + NCLASS] = {};
        for (int rep = 0; rep < 2 && rc == GA_OK; ++rep)
            rc = ga_align_batch(ctx, &bt, &sc, w, -1, (ga_result_t *)(buf + o_out), s);
        if (rc == GA_OK) rc = ga_context_timing(ctx, ml, 1 + NCLASS);
        if (rc == GA_OK) rc = ga_context_check(ctx, s);
        lat[c] = (float)(ml[1 + c] * 1e6 / steps);
        (void)hipFree(buf);
    }
    ctx->class_mask = mask0;
    ctx->schedule = sched0;
    const int rc2 = ga_context_set_timing(ctx, timing0);
    if (rc == GA_OK) rc = rc2;
    if (rc != GA_OK) return rc;
    ctx->class_order = order_by(cost);
    ctx->order_lat = order_by(lat);
    ctx->lat_pairs = 2 * ctx->num_cu;
    for (int c = 0; c < NCLASS; ++c) {
        ctx->class_cost[c] = cost[c];
        ctx->class_lat[c] = lat[c];
    }
    for (int c = 0; c < n_out && c < NCLASS; ++c) ns_per_step[c] = cost[c];
    return GA_OK;
}

int ga_context_class_latency(const ga_context_t *ctx, float *ns_per_step, int n) {
    if (!ctx || n < 0 || (n > 0 && !ns_per_step)) return GA_EINVAL;
    if (!ctx->lat_pairs) return GA_EINVAL;
    for (int c = 0; c < n && c < NCLASS; ++c) ns_per_step[c] = ctx->class_lat[c];
    return GA_OK;
}

int ga_context_set_latency_pairs(ga_context_t *ctx, int32_t n_pairs) {
    if (!ctx || n_pairs < 0) return GA_EINVAL;
    if (!ctx->order_lat) return GA_EINVAL;  // not autotuned
    ctx->lat_pairs = n_pairs;
    return GA_OK;
}

int ga_context_batch_class(const ga_context_t *ctx, int32_t n, int32_t m, int32_t w, int64_t n_pairs) {
    if (!ctx || n <= 0 || m <= 0) return -1;
    int slide;
    return class_for(n, m, w, &slide, ctx->class_mask, batch_order(ctx, n_pairs));
}

int ga_pair_class(int32_t n, int32_t m, int32_t w) {
    if (n <= 0 || m <= 0) return -1;
    int slide;
    return class_for(n, m, w, &slide);
}

int ga_pair_class_in(int32_t n, int32_t m, int32_t w, uint32_t mask) {
    if (n <= 0 || m <= 0) return -1;
    int slide;
    return class_for(n, m, w, &slide, mask & ALL_CLASSES);
}

int64_t ga_pack_words(const int32_t *len_host, int64_t n) {
    if (!len_host || n < 0) return -1;
    int64_t total = 0;
    for (int64_t p = 0; p < n; ++p) total += len_host[p] > 0 ? ((int64_t)len_host[p] + 15) / 16 : 0;
    return total;
}

int ga_pack(ga_context_t *ctx, const uint8_t *ascii_dev, const int64_t *off_dev, const int32_t *len_dev,
            int64_t n, int64_t nwords, uint32_t *words_dev, int64_t *word_off_dev, uint32_t *nmask_dev,
            void *stream) {
    if (!ctx || n < 0 || nwords < 0) return GA_EINVAL;
    if (n == 0) return GA_OK;
    if (!ascii_dev || !off_dev || !len_dev || !word_off_dev) return GA_EINVAL;
    if (nwords > 0 && (!words_dev || !nmask_dev)) return GA_EINVAL;
    SetDevice sd(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_ws(ctx, 64);
    if (rc != GA_OK) return rc;
    int64_t *total = (int64_t *)ctx->ws;
    const int TB = 256;
    hipLaunchKernelGGL(ga_word_counts, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, s, len_dev, n,
                       word_off_dev);
    hipLaunchKernelGGL(ga_exclusive_scan, dim3(1), dim3(1024), 0, s, word_off_dev, n, total);
    const int64_t nmw = (nwords + 1) / 2;
    if (nmw > 0)
        hipLaunchKernelGGL(ga_zero_i32, dim3((unsigned)((nmw + TB - 1) / TB)), dim3(TB), 0, s,
                           (int32_t *)nmask_dev, nmw);
    hipLaunchKernelGGL(ga_pack_kernel, dim3((unsigned)n), dim3(64), 0, s, ascii_dev, off_dev, len_dev,
                       word_off_dev, nwords, words_dev, nmask_dev, ctx->d_err);
    return hipGetLastError() == hipSuccess ? GA_OK : GA_EHIP;
}

int ga_calibrate_valu(ga_context_t *ctx, double *lane_ops_per_s, void *stream) {
    if (!ctx || !lane_ops_per_s) return GA_EINVAL;
    SetDevice sd(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_ws(ctx, 256);
    if (rc != GA_OK) return rc;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return GA_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return GA_EHIP;
    }
    const int threads = 256;  // 4 waves per workgroup
    const int blocks = ctx->num_cu * 4 * CAL_WAVES_PER_SIMD / (threads / WAVE);
    const int iters = 20000;
    int32_t *sink = (int32_t *)ctx->ws;
    hipLaunchKernelGGL(ga_valu_probe, dim3(blocks), dim3(threads), 0, s, 100, sink);  // warm up
    hipEventRecord(e0, s);
    hipLaunchKernelGGL(ga_valu_probe, dim3(blocks), dim3(threads), 0, s, iters, sink);
    hipEventRecord(e1, s);
    float ms = 0.f;
    const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (!ok || ms <= 0.f) return GA_EHIP;
    const double ops = (double)blocks * threads * iters * CAL_CHAINS * 2;
    *lane_ops_per_s = ops / (ms * 1e-3);
    return GA_OK;
}

int64_t ga_count_cells(int32_t n, int32_t m, int32_t w, int32_t r_end) {
    if (n <= 0 || m <= 0 || r_end < 0) return 0;
    int64_t total = 0;
    for (int64_t r = 0; r <= r_end && r <= (int64_t)n + m - 2; ++r) {
        int64_t lo = r - (m - 1) > 0 ? r - (m - 1) : 0;
        int64_t hi = r < n - 1 ? r : n - 1;
        if (w >= 0) {
            const int64_t t = r - w, u = r + w;
            const int64_t lb = t >= 0 ? (t + 1) / 2 : -((-t) / 2);
            const int64_t ub = u / 2;
            if (lb > lo) lo = lb;
            if (ub < hi) hi = ub;
        }
        if (hi >= lo) total += hi - lo + 1;
    }
    return total;
}

}  // extern "C"

namespace {

// Host validation of an alignment call (GA_OK, GA_EINVAL or GA_EUNSUPPORTED).
int validate_call(const ga_context_t *ctx, const ga_batch_t *bt, const ga_scoring_t *sc, int32_t w, int32_t Z,
                  const ga_result_t *out_dev) {
    if (!ctx || !bt || !sc || bt->n_pairs < 0) return GA_EINVAL;
    if (bt->n_pairs == 0) return GA_OK;
    if (!out_dev || !bt->t_off_dev || !bt->q_off_dev || !bt->t_len_dev || !bt->q_len_dev) return GA_EINVAL;
    if (bt->t_nwords < 0 || bt->q_nwords < 0 || bt->max_len < 0) return GA_EINVAL;
    if ((bt->t_nwords > 0 && !bt->t_words_dev) || (bt->q_nwords > 0 && !bt->q_words_dev)) return GA_EINVAL;
    if (sc->a < 0 || sc->b < 0 || sc->q < 0 || sc->e < 0 || sc->q2 < 0 || sc->e2 < 0 || sc->ambig < 0)
        return GA_EINVAL;
    {
        // the per-cell score table holds S + q + 2e in signed bytes
        const int64_t fold = (int64_t)sc->q + 2 * (int64_t)sc->e;
        if (sc->a + fold > 127 || fold - sc->b < -128 || fold - sc->ambig < -128) return GA_EUNSUPPORTED;
    }
    {
        const int64_t oe1 = (int64_t)sc->q + sc->e, oe2 = (int64_t)sc->q2 + sc->e2;
        int64_t P = sc->a;
        if (sc->b > P) P = sc->b;
        if (sc->ambig > P) P = sc->ambig;
        if (oe1 > P) P = oe1;
        if (oe2 > P) P = oe2;
        const int64_t L = 2 * (int64_t)bt->max_len + 2;
        const int64_t guard = L * (P + sc->a + sc->e + sc->e2) + (Z > 0 ? Z : 0);
        if (guard >= (int64_t)1 << 29) return GA_EINVAL;
    }
    {
        const int64_t wl = w < 0 ? bt->max_len : (w < bt->max_len ? w : bt->max_len);
        if (2 * wl + 1 > MAX_DIAGONALS) return GA_EUNSUPPORTED;
    }
    return GA_OK;
}

// The context's side streams and their fork/join events, made on first
// use by an allocating call with more than one lane. (Made only then: a
// context that never needs them -- a serving slot on one lane -- must not
// add streams, which would share the GPU's few hardware queues with the
// streams that matter.)
int make_side_streams(ga_context *ctx) {
    if (ctx->fork_ev) return GA_OK;
    bool ok = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < MAX_LANES - 1; ++k)
        ok = hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&ctx->join_ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (ctx->fork_ev) hipEventDestroy(ctx->fork_ev);
        ctx->fork_ev = nullptr;
        for (int k = 0; k < MAX_LANES - 1; ++k) {
            if (ctx->side[k]) hipStreamDestroy(ctx->side[k]);
            if (ctx->join_ev[k]) hipEventDestroy(ctx->join_ev[k]);
            ctx->side[k] = nullptr;
            ctx->join_ev[k] = nullptr;
        }
        return GA_EHIP;
    }
    return GA_OK;
}

// The planning and alignment launches of one validated, non-empty call on
// the device current, with `ws` the call's planning workspace
// (ws_bytes(n_pairs) bytes of device memory). The persistent launches
// spread over the context's lanes when its side streams exist, else all
// run on `s`.
int align_launch(ga_context *ctx, const ga_batch_t *bt, const ga_scoring_t *sc, int32_t w, int32_t Z,
                 ga_result_t *out_dev, hipStream_t s, char *ws) {
    const int64_t np = bt->n_pairs;
    const size_t off_cursor = WS_CURSOR;
    int32_t *counters = (int32_t *)ws;
    int32_t *lists = (int32_t *)(ws + ws_lists((size_t)np));
    const int TB = 256;
    const bool timed = ctx->timing != 0;
    ctx->timed_last = timed ? 1 : 0;
    if (timed) hipEventRecord(ctx->ev[0], s);
    // counters and the bucket histogram are contiguous: one fill clears both
    hipLaunchKernelGGL(ga_zero_i32, dim3((unsigned)((off_cursor / 4 + TB - 1) / TB)), dim3(TB), 0, s,
                       counters, (int64_t)(off_cursor / 4));
    PlanArgs pa;
    pa.n_pairs = np;
    pa.t_off = bt->t_off_dev;
    pa.q_off = bt->q_off_dev;
    pa.t_len = bt->t_len_dev;
    pa.q_len = bt->q_len_dev;
    pa.t_nwords = bt->t_nwords;
    pa.q_nwords = bt->q_nwords;
    pa.max_len = bt->max_len;
    pa.w = w;
    pa.bucketed = ctx->schedule == GA_SCHED_BUCKETED ? 1 : 0;
    pa.ordered = ctx->schedule == GA_SCHED_PERSISTENT ? 1 : 0;
    pa.mask = ctx->class_mask;
    pa.order = batch_order(ctx, np);
    pa.counters = counters;
    pa.hist = (int32_t *)(ws + WS_HIST);
    pa.cursor = (int32_t *)(ws + WS_CURSOR);
    pa.keys = (int32_t *)(ws + WS_KEYS);
    pa.lists = lists;
    pa.err = ctx->d_err;
    pa.out = out_dev;
    hipLaunchKernelGGL(ga_plan_classify, dim3((unsigned)((np + TB - 1) / TB)), dim3(TB), 0, s, pa);
    hipLaunchKernelGGL(ga_plan_scan, dim3(1), dim3(1024), 0, s, pa);
    hipLaunchKernelGGL(ga_plan_scatter, dim3((unsigned)((np + TB - 1) / TB)), dim3(TB), 0, s, pa);
    if (timed) hipEventRecord(ctx->ev[1], s);

    DpArgs da;
    da.tw = bt->t_words_dev;
    da.qw = bt->q_words_dev;
    da.tn = bt->t_nmask_dev;
    da.qn = bt->q_nmask_dev;
    da.t_off = bt->t_off_dev;
    da.q_off = bt->q_off_dev;
    da.t_len = bt->t_len_dev;
    da.q_len = bt->q_len_dev;
    da.counters = counters;
    da.out = out_dev;
    da.w = w;
    da.Z = Z;
    da.q1 = sc->q;
    da.c2 = (sc->q2 + sc->e2) - (sc->q + sc->e);
    da.d2 = sc->e2 - sc->e;
    da.e1 = sc->e;
    da.e2 = sc->e2;
    da.oe1 = sc->q + sc->e;
    da.oe2 = sc->q2 + sc->e2;
    // -gamma(r+2) - q + e*r = max(-2q - 2e, -(q2 + e2) - e2 - q + r*(e - e2))
    da.ring_a0 = -2 * sc->q - 2 * sc->e;
    da.ring_b0 = -(sc->q2 + sc->e2) - sc->e2 - sc->q;
    da.ring_d = sc->e - sc->e2;
    {
        const int fold = sc->q + 2 * sc->e;  // frame drift over the diagonal step
        const uint32_t A = (uint32_t)(uint8_t)(int8_t)(sc->a + fold);
        const uint32_t B = (uint32_t)(uint8_t)(int8_t)(fold - sc->b);
        const uint32_t N = (uint32_t)(uint8_t)(int8_t)(fold - sc->ambig);
        da.lut_lo = A | (B << 8) | (B << 16) | (B << 24);
        da.lut_hi = N | (N << 8) | (N << 16) | (N << 24);
    }
    da.list = lists;
    int nl = 0;
    if (ctx->schedule == GA_SCHED_BUCKETED) {
        // plain per-length-bucket launches, for comparison: wait for the
        // group sizes, then one fixed-shape launch per non-empty bucket with
        // one workgroup per pair
        if (!ctx->h_counts) {
            if (hipHostMalloc((void **)&ctx->h_counts, sizeof(int32_t) * NGROUP) != hipSuccess) {
                (void)hipGetLastError();
                ctx->h_counts = nullptr;
                return GA_ENOMEM;
            }
        }
        if (hipMemcpyAsync(ctx->h_counts, counters + CNT_COUNT, sizeof(int32_t) * NGROUP, hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return GA_EHIP;
        for (int g = 0; g < NGROUP; ++g) {
            const int cnt = ctx->h_counts[g];
            const int c = cnt > 0 ? bucket_class(g, w, ctx->class_mask) : -1;
            if (c < 0) continue;
            da.group = g;
            if (timed) hipEventRecord(ctx->ev[2 + 2 * nl], s);
            launch_class(c, da, cnt, s);
            if (timed) hipEventRecord(ctx->ev[3 + 2 * nl], s);
            ctx->launch_class[nl] = c;
            ++nl;
        }
    } else {
        // fork the context's streams off the caller's, launch each class on
        // its lane, join them back: the classes' launches overlap, so the
        // tail of one (its last long pairs) runs beside the others
        const int L = ctx->fork_ev ? ctx->lanes : 1;
        hipStream_t lane_s[MAX_LANES] = {s, s, s, s};
        if (L > 1) {
            if (hipEventRecord(ctx->fork_ev, s) != hipSuccess) return GA_EHIP;
            for (int k = 1; k < L; ++k) {
                if (hipStreamWaitEvent(ctx->side[k - 1], ctx->fork_ev, 0) != hipSuccess) return GA_EHIP;
                lane_s[k] = ctx->side[k - 1];
            }
        }
        int slide;
        const int full = class_for(bt->max_len, bt->max_len, w, &slide, ctx->class_mask, pa.order);
        const uint32_t reach = reachable_classes(bt->max_len, w, ctx->class_mask, pa.order);
        for (int k = -1; k < NCLASS; ++k) {
            const int c = k < 0 ? full : LAUNCH_ORDER[k];
            if (c < 0 || (k >= 0 && c == full) || !((reach >> c) & 1u)) continue;
            const int64_t want = (int64_t)ctx->num_cu * ctx->blocks_per_cu[c];
            const int grid = (int)(np < want ? np : want);
            hipStream_t ls = lane_s[k < 0 ? 0 : LANE_OF[c] % L];
            da.group = c;
            if (timed) hipEventRecord(ctx->ev[2 + 2 * nl], ls);
            launch_class(c, da, grid, ls);
            if (timed) hipEventRecord(ctx->ev[3 + 2 * nl], ls);
            ctx->launch_class[nl] = c;
            ++nl;
        }
        for (int k = 1; k < L; ++k) {
            if (hipEventRecord(ctx->join_ev[k - 1], ctx->side[k - 1]) != hipSuccess ||
                hipStreamWaitEvent(s, ctx->join_ev[k - 1], 0) != hipSuccess)
                return GA_EHIP;
        }
    }
    ctx->n_launch_last = nl;
    return hipGetLastError() == hipSuccess ? GA_OK : GA_EHIP;
}

}  // namespace

extern "C" {

int ga_align_batch(ga_context_t *ctx, const ga_batch_t *bt, const ga_scoring_t *sc, int32_t w, int32_t Z,
                   ga_result_t *out_dev, void *stream) {
    int rc = validate_call(ctx, bt, sc, w, Z, out_dev);
    if (rc != GA_OK || bt->n_pairs == 0) return rc;
    SetDevice sd(ctx->device);
    rc = ensure_ws(ctx, ws_bytes((size_t)bt->n_pairs));
    if (rc == GA_OK && ctx->lanes > 1 && ctx->schedule != GA_SCHED_BUCKETED) rc = make_side_streams(ctx);
    if (rc != GA_OK) return rc;
    return align_launch(ctx, bt, sc, w, Z, out_dev, (hipStream_t)stream, (char *)ctx->ws);
}

struct ga_graph {
    int device;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

int ga_graph_capture(ga_context_t *ctx, const ga_batch_t *bt, const ga_scoring_t *sc, int32_t w, int32_t Z,
                     ga_result_t *out_dev, void *stream, ga_graph_t **graph) {
    if (!graph) return GA_EINVAL;
    *graph = nullptr;
    int rc = validate_call(ctx, bt, sc, w, Z, out_dev);
    if (rc != GA_OK) return rc;
    if (!stream || bt->n_pairs == 0 || ctx->timing || ctx->schedule == GA_SCHED_BUCKETED) return GA_EINVAL;
    SetDevice sd(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    // everything the call needs exists before capture: the workspace at this
    // batch's size and the side streams
    rc = ensure_ws(ctx, ws_bytes((size_t)bt->n_pairs));
    if (rc == GA_OK && ctx->lanes > 1) rc = make_side_streams(ctx);
    if (rc != GA_OK) return rc;
    ga_graph *g = (ga_graph *)calloc(1, sizeof(ga_graph));
    if (!g) return GA_ENOMEM;
    g->device = ctx->device;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        free(g);
        return GA_EHIP;
    }
    rc = align_launch(ctx, bt, sc, w, Z, out_dev, s, (char *)ctx->ws);
    const bool ended = hipStreamEndCapture(s, &g->graph) == hipSuccess;
    if (rc == GA_OK && (!ended || !g->graph)) rc = GA_EHIP;
    if (rc == GA_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) rc = GA_EHIP;
    if (rc != GA_OK) {
        (void)hipGetLastError();
        if (g->graph) hipGraphDestroy(g->graph);
        free(g);
        return rc;
    }
    *graph = g;
    return GA_OK;
}

int ga_graph_launch(ga_graph_t *g, void *stream) {
    if (!g || !g->exec) return GA_EINVAL;
    SetDevice sd(g->device);
    return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? GA_OK : GA_EHIP;
}

int ga_graph_destroy(ga_graph_t *g) {
    if (!g) return GA_EINVAL;
    SetDevice sd(g->device);
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    free(g);
    return GA_OK;
}

int ga_align_batch_noalloc(ga_context_t *ctx, const ga_batch_t *bt, const ga_scoring_t *sc, int32_t w,
                           int32_t Z, ga_result_t *out_dev, void *stream) {
    int rc = validate_call(ctx, bt, sc, w, Z, out_dev);
    if (rc != GA_OK || bt->n_pairs == 0) return rc;
    if (bt->n_pairs > GA_NOALLOC_MAX_PAIRS) return GA_EINVAL;
    if (ctx->schedule == GA_SCHED_BUCKETED) return GA_EUNSUPPORTED;  // it waits for the host
    if (!ctx->scratch) return GA_EHIP;
    SetDevice sd(ctx->device);
    return align_launch(ctx, bt, sc, w, Z, out_dev, (hipStream_t)stream, (char *)ctx->scratch);
}

}  // extern "C"
