// Wavefront primitives shared by the search and index-build kernels of
// libnsg.so: storage-format decoding, LDS pool merge, visited filter and the
// row-gather distance routine.  One 64-lane wave works on one query.
#pragma once
#include "common.hpp"

namespace nsg {

#define KEY_MASK 0xFFFFFFFF7FFFFFFFull
#define CHECKED_BIT 0x80000000ull
#define KEY_NONE 0xFFFFFFFFFFFFFFFFull

// ------------------------------------------------------------------------
// storage formats: decode one 16-byte chunk into EPC floats
// ------------------------------------------------------------------------
template <int DT> struct Fmt;
template <> struct Fmt<NSG_F32> {
    static constexpr int EPC = 4;
    __device__ static inline void dec(const uint4 r, float *o) {
        o[0] = __uint_as_float(r.x); o[1] = __uint_as_float(r.y);
        o[2] = __uint_as_float(r.z); o[3] = __uint_as_float(r.w);
    }
};
template <> struct Fmt<NSG_BF16> {
    static constexpr int EPC = 8;
    __device__ static inline void dec(const uint4 r, float *o) {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(w[i] << 16);
            o[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
        }
    }
};
template <> struct Fmt<NSG_F16> {
    static constexpr int EPC = 8;
    __device__ static inline void dec(const uint4 r, float *o) {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[i] & 0xFFFFu));
            o[2 * i + 1] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w[i] >> 16));
        }
    }
};
// OCP FP8 E4M3 (bias 7, no infinities, S.1111.111 is NaN) by the packed
// hardware conversion, two bytes per instruction (it equals the field-by-field
// definition on all 256 codes, checked on gfx950 by a GPU test).
template <> struct Fmt<NSG_E4M3> {
    static constexpr int EPC = 16;
    __device__ static inline void dec(const uint4 r, float *o) {
        const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);   // bytes 0, 1
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);    // bytes 2, 3
            o[4 * i] = lo[0];
            o[4 * i + 1] = lo[1];
            o[4 * i + 2] = hi[0];
            o[4 * i + 3] = hi[1];
        }
    }
};

// ------------------------------------------------------------------------
// wave primitives
// ------------------------------------------------------------------------
// Order LDS accesses between the lanes of one wave.  A wave's LDS operations
// complete in issue order, so only compiler reordering has to be prevented:
// a code-motion barrier plus a compiler memory clobber, no memory fence (a
// fence would also wait for outstanding global loads).
__device__ inline void wave_sync() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

__device__ inline uint64_t mk_key(float d, uint32_t id) {
    return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)id;
}
__device__ inline float key_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ inline uint32_t key_id(uint64_t k) { return (uint32_t)(k & 0x7FFFFFFFu); }

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of
// a group receives its group's sum.  Within a row of 16 lanes the steps are
// DPP moves (mirror, half-mirror, quad permutations), across rows lane
// shuffles.
template <int CTRL>
__device__ inline float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int G>
__device__ inline float group_sum(float s) {
    if (G >= 64) s += __shfl_xor(s, 32);
    if (G >= 32) s += __shfl_xor(s, 16);
    if (G >= 16) s += dpp_mov<0x140>(s);   // row_mirror: lane l <-> 15 - l
    if (G >= 8) s += dpp_mov<0x141>(s);    // row_half_mirror: lane l <-> 7 - l
    if (G >= 4) s += dpp_mov<0x4E>(s);     // quad_perm [2,3,0,1]
    if (G >= 2) s += dpp_mov<0xB1>(s);     // quad_perm [1,0,3,2]
    return s;
}

// Visited filter: a direct-mapped table of node ids.  Exchanging u into its
// slot returns the previous occupant: u itself means u was seen; anything else
// means it was not (or was evicted by a colliding id, i.e. forgotten, which
// only costs a recomputation).  It never reports an unseen node as seen.
__device__ inline bool hash_insert(uint32_t *tab, int bits, uint32_t u) {
    const uint32_t h = (u * 2654435761u) >> (32 - bits);
    return atomicExch(&tab[h], u) != u;
}

__device__ inline uint64_t readlane64(uint64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v & 0xFFFFFFFFu), l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t readfirstlane64(uint64_t v) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v & 0xFFFFFFFFu));
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Merge the M keys staged in sbuf[0..M) (KEY_NONE = empty) into the sorted
// pool of `size` entries (size and Lcur wave-uniform), keeping the first Lcur.
//
// The staged keys are read back as wave-uniform values, so every step is a
// fixed, unrolled set of independent compares and ballots (no loop whose trip
// count depends on the data).  A staged key is dropped if an earlier staged
// key equals it (a node recorded twice) or if the pool holds it (a node the
// visited filter forgot; the pool entry keeps its checked flag): lane j looks
// at the pool entry at key j's lower bound, the only place an equal key can
// sit.  For each kept key j: lb_j = #pool keys below it; pool entry i moves to
// i + #{kept keys below it} (chunks last first, so nothing is overwritten
// before it is read) and key j goes to lb_j + #{kept keys below it}.
// Positions at or beyond Lcur are not written.
template <int M>
__device__ int merge_staged(uint64_t *pool, int size, int Lcur, const uint64_t *sbuf, int lane,
                            int *first_ins) {
    uint64_t bk[M];
#pragma unroll
    for (int j = 0; j < M; ++j) bk[j] = readfirstlane64(sbuf[j]);
    const uint64_t mine = lane < M ? sbuf[lane] : KEY_NONE;
    uint64_t dup = 0;
#pragma unroll
    for (int j = 0; j < M - 1; ++j) dup |= __ballot(mine == bk[j]) & (~0ull << (j + 1));
    uint32_t keep = (uint32_t)(__ballot(mine != KEY_NONE) & ~dup);
    const int nch = (size + 63) >> 6;
    int lb[M];
#pragma unroll
    for (int j = 0; j < M; ++j) lb[j] = 0;
    for (int c = 0; c < nch; ++c) {
        const int i = (c << 6) + lane;
        const uint64_t pk = i < size ? (pool[i] & KEY_MASK) : KEY_NONE;
#pragma unroll
        for (int j = 0; j < M; ++j) lb[j] += __popcll(__ballot(pk < bk[j]));
    }
    int mylb = 0;
#pragma unroll
    for (int j = 0; j < M; ++j) mylb = lane == j ? lb[j] : mylb;
    bool eq = false;
    if (lane < M && ((keep >> lane) & 1u) && mylb < size) eq = (pool[mylb] & KEY_MASK) == mine;
    keep &= ~(uint32_t)__ballot(eq);
    if (!keep) return size;
    int p0 = size;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const bool kj = (keep >> j) & 1u;
        if (!kj) bk[j] = KEY_NONE;   // a dropped key shifts nothing
        p0 = (kj && lb[j] < p0) ? lb[j] : p0;
    }
    if (p0 >= Lcur) return size;
    // pool entries [p0, size) move right, last chunk first
    for (int c = nch - 1; c >= 0 && (c << 6) + 63 >= p0; --c) {
        const int i = (c << 6) + lane;
        const bool act = i >= p0 && i < size;
        const uint64_t v = act ? pool[i] : 0ull;
        const uint64_t vk = v & KEY_MASK;
        int sh = 0;
#pragma unroll
        for (int j = 0; j < M; ++j) sh += bk[j] < vk ? 1 : 0;
        wave_sync();
        if (act && i + sh < Lcur) pool[i + sh] = v;
        wave_sync();
    }
    // kept staged keys: lane j places key j
    int pos = mylb;
#pragma unroll
    for (int j = 0; j < M; ++j) pos += bk[j] < mine ? 1 : 0;
    if (lane < M && ((keep >> lane) & 1u) && pos < Lcur) pool[pos] = mine;
    wave_sync();
    *first_ins = p0;
    const int ns = size + __popc(keep);
    return ns < Lcur ? ns : Lcur;
}

// Merge up to 64 candidate keys (one per lane, KEY_NONE = empty) into the
// sorted pool: the non-empty keys are staged, in lane order, in groups of at
// most 16 in sbuf (16 entries of LDS owned by the caller) and merged group by
// group.  Returns the new size; *first_ins receives the smallest position
// written (size if nothing was inserted).
__device__ int merge_pool(uint64_t *pool, int size, int Lcur, uint64_t key, uint64_t *sbuf,
                          int lane, int *first_ins) {
    *first_ins = size;
    const bool surv = key != KEY_NONE;
    const uint64_t sm = __ballot(surv);
    if (!sm) return size;
    const int m = __popcll(sm);
    const int idx = __popcll(sm & ((1ull << lane) - 1ull));
    for (int g = 0; g * 16 < m; ++g) {
        const int mg = m - g * 16 < 16 ? m - g * 16 : 16;
        const int M = mg <= 4 ? 4 : (mg <= 8 ? 8 : 16);
        if (lane < M) sbuf[lane] = KEY_NONE;
        wave_sync();
        if (surv && (idx >> 4) == g) sbuf[idx & 15] = key;
        wave_sync();
        int fi = size;
        if (M == 4)
            size = merge_staged<4>(pool, size, Lcur, sbuf, lane, &fi);
        else if (M == 8)
            size = merge_staged<8>(pool, size, Lcur, sbuf, lane, &fi);
        else
            size = merge_staged<16>(pool, size, Lcur, sbuf, lane, &fi);
        *first_ins = fi < *first_ins ? fi : *first_ins;
        wave_sync();
    }
    return size;
}

// ------------------------------------------------------------------------
// register-resident pool (search)
// ------------------------------------------------------------------------
// Lane l of pk[c] holds the key of pool entry 64c + l; bit l of the
// wave-uniform mask unc[c] is set when that entry is in the pool (position <
// size) and not yet checked.  The pool is sorted by key, so Algorithm 1's
// "first unchecked" is a scalar bit scan of unc, and an insertion is one
// compare + ballot per chunk (the rank) followed by a one-lane shift of the
// chunks at or above it.
// Positions at or beyond size hold KEY_NONE until the pool first fills, and
// afterwards keys pushed out at the end (never read: every reader stops at
// size).  Such a key is larger than every key in the pool and than every key
// the merge may still insert (a key enters only below the current L-th key,
// and the L-th key only decreases), so it never counts in a rank.
template <int NCH>
struct RegPool {
    uint64_t pk[NCH];
    uint64_t unc[NCH];
    int size;
};

// v_writelane_b32: the wave-uniform `value` replaces lane `lane` of `old`
// (the compiler intrinsic, bound by name; no builtin is exposed for it)
__device__ int amdgcn_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// whole-wave shift by one lane towards higher lanes (lane 0 receives 0)
__device__ __attribute__((always_inline)) inline uint64_t wave_shr64(uint64_t v) {
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v & 0xFFFFFFFFu), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), 0x138, 0xF, 0xF, true);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// v with lane l (wave-uniform) replaced by the wave-uniform value x
__device__ __attribute__((always_inline)) inline uint64_t writelane64(uint64_t v, uint64_t x, int l) {
    const int lo = amdgcn_writelane((int)(uint32_t)(x & 0xFFFFFFFFu), l, (int)(uint32_t)(v & 0xFFFFFFFFu));
    const int hi = amdgcn_writelane((int)(uint32_t)(x >> 32), l, (int)(uint32_t)(v >> 32));
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int NCH>
__device__ __attribute__((always_inline)) inline void rp_init(RegPool<NCH> &P) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        P.pk[c] = KEY_NONE;
        P.unc[c] = 0ull;
    }
    P.size = 0;
}

// key of entry pos (wave-uniform, < NCH * 64)
template <int NCH>
__device__ __attribute__((always_inline)) inline uint64_t rp_get(const RegPool<NCH> &P, int pos) {
    // read lane pos & 63 of every chunk, keep chunk pos >> 6 (scalar selects;
    // selecting the registers first would index the chunk array dynamically)
    const int cw = pos >> 6, l = pos & 63;
    uint64_t v = KEY_NONE;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const uint64_t x = readlane64(P.pk[c], l);
        v = cw == c ? x : v;
    }
    return v;
}

// position of the first unchecked entry (-1 if none); its key in *key
template <int NCH>
__device__ __attribute__((always_inline)) inline int rp_first_unchecked(const RegPool<NCH> &P, uint64_t *key) {
    int pos = -1;
#pragma unroll
    for (int c = NCH - 1; c >= 0; --c) pos = P.unc[c] ? (c << 6) + __builtin_ctzll(P.unc[c]) : pos;
    if (pos >= 0) *key = rp_get<NCH>(P, pos);
    return pos;
}

template <int NCH>
__device__ __attribute__((always_inline)) inline void rp_mark_checked(RegPool<NCH> &P, int pos) {
    const uint64_t bit = 1ull << (pos & 63);
    const int cw = pos >> 6;
#pragma unroll
    for (int c = 0; c < NCH; ++c) P.unc[c] &= cw == c ? ~bit : ~0ull;
}

// Insert the wave-uniform key s unless the pool holds it (a node the visited
// filter forgot) or it ranks at or beyond Lcur; the entry pushed to position
// Lcur, if any, leaves the pool.  Returns true if inserted.
template <int NCH>
__device__ __attribute__((always_inline)) inline bool rp_insert(RegPool<NCH> &P, uint64_t s, int Lcur, int lane) {
    int lt = 0;
    bool eq = false;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if ((c << 6) < P.size) {
            lt += __popcll(__ballot(P.pk[c] < s));
            eq |= __ballot(P.pk[c] == s) != 0ull;
        }
    }
    if (eq || lt >= Lcur) return false;
    const int top = P.size < Lcur ? P.size : Lcur - 1;   // last occupied position afterwards
#pragma unroll
    for (int c = NCH - 1; c >= 0; --c) {
        if ((c << 6) > top || (c << 6) + 63 < lt) continue;
        // chunk c-1 is still unmodified: its last entry moves into lane 0
        // (chunk 0's lane 0 is only ever the inserted key itself)
        uint64_t sh = wave_shr64(P.pk[c]);
        if (c > 0) sh = writelane64(sh, readlane64(P.pk[c > 0 ? c - 1 : 0], 63), 0);
        const uint64_t cbit = c > 0 ? (P.unc[c > 0 ? c - 1 : 0] >> 63) : 0ull;
        const int idx = (c << 6) + lane;
        const int lo = lt - (c << 6);
        const uint64_t nv = idx >= lt ? sh : P.pk[c];
        P.pk[c] = lo >= 0 ? writelane64(nv, s, lo) : nv;   // lo <= 63 here
        const uint64_t f = P.unc[c];
        uint64_t nf;
        if (lo < 0) {
            nf = (f << 1) | cbit;
        } else {
            const uint64_t below = (1ull << lo) - 1ull;     // lo <= 63 here
            nf = (f & below) | ((f << 1) & ~below) | (1ull << lo);
        }
        // an entry pushed to position Lcur leaves the pool
        const int cut = Lcur - (c << 6);
        if (cut < 64) nf &= (1ull << cut) - 1ull;        // cut >= 1 here
        P.unc[c] = nf;
    }
    P.size = P.size < Lcur ? P.size + 1 : Lcur;
    return true;
}

// write the pool to LDS (checked flag in the key's flag bit)
template <int NCH>
__device__ __attribute__((always_inline)) inline void rp_store(const RegPool<NCH> &P, uint64_t *pool, int lane) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int idx = (c << 6) + lane;
        if ((c << 6) < P.size && idx < P.size)
            pool[idx] = P.pk[c] | (((P.unc[c] >> lane) & 1ull) ? 0ull : CHECKED_BIT);
    }
}

// Rows the gathers read: n_rows rows of row_chunks 16-byte chunks each.  The
// allocation extends kRowTailBytes (zero-filled) past the last row, so every
// lane of a row group may read its full width of chunks at any row, also
// where the row holds fewer chunks (those reads are discarded, see
// gather_dist) without a per-lane condition on the load.
struct RowTable {
    const unsigned char *base;
    uint32_t row_bytes;   // row_chunks * 16
    uint32_t n_rows;
    int row_chunks;
};

// rows of one gather round
template <int LPR, int CPL>
struct GatherShape {
    static constexpr int RPP = 64 / LPR;                          // rows per pass
    static constexpr int U = (8 / CPL) > 0 ? (8 / CPL) : 1;       // passes per round
    static constexpr int ROWS = RPP * U;
};

// One round of NP passes of the gather: the row ids of the round are read
// from LDS and every row load is issued, then the passes are reduced (straight
// line code, so the loads of all passes are in flight together).  A lane
// whose row lies past the last one (r >= cnt) re-reads the last row, so no
// load needs a per-lane condition; its distance is not stored.  Chunks beyond
// a row's end contribute nothing: reduced formats carry a zero scale and a
// zero query there, FP32 rows (`part`) are zeroed explicitly.
template <int DT, int LPR, int CPL, int NP>
__device__ __attribute__((always_inline)) inline void gather_round(const RowTable &T, const unsigned char *lane_base,
                                                                   const float (&qv)[CPL][Fmt<DT>::EPC],
                                                                   const float (&sc)[CPL][Fmt<DT>::EPC],
                                                                   const uint32_t *cid, float *cdist, int r0,
                                                                   int cnt, int lane, bool part) {
    constexpr int EPC = Fmt<DT>::EPC;
    constexpr int RPP = GatherShape<LPR, CPL>::RPP;
    const int g = lane / LPR, li = lane % LPR;
    uint4 raw[NP][CPL];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        int r = r0 + u * RPP + g;
        r = r < cnt ? r : cnt - 1;
        uint32_t id = cid[r];
        id = id < T.n_rows ? id : 0u;   // never index past the table
        const unsigned char *rp = lane_base + (uint64_t)id * T.row_bytes;
#pragma unroll
        for (int c = 0; c < CPL; ++c) raw[u][c] = *reinterpret_cast<const uint4 *>(rp + c * LPR * 16);
    }
    // keep the reductions below every load of the round (the scheduler would
    // otherwise start one and wait for its data before the last loads issue)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            uint4 v = raw[u][c];
            if (part && li + c * LPR >= T.row_chunks) v = make_uint4(0u, 0u, 0u, 0u);
            float x[EPC];
            Fmt<DT>::dec(v, x);
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
                float xv = DT == NSG_F32 ? x[e] : sc[c][e] * x[e];
                float t = qv[c][e] - xv;
                acc = fmaf(t, t, acc);
            }
        }
        const float dsum = group_sum<LPR>(acc);
        const int r = r0 + u * RPP + g;
        if (li == 0 && r < cnt) cdist[r] = dsum;
    }
}

// Squared distances of q to the rows cid[0..cnt) -> cdist[0..cnt) (cnt >= 1).
// LPR lanes gather one row (lane li of the group reads chunks li + c * LPR,
// c < CPL, at compile-time offsets from one row address); a pass covers RPP
// rows.  Rounds take U passes while enough rows are left; the last round
// takes the fewest passes (1, 2, 4 or U) that cover its rows.
template <int DT, int LPR, int CPL>
__device__ inline void gather_dist(const RowTable &T, const float (&qv)[CPL][Fmt<DT>::EPC],
                                   const float (&sc)[CPL][Fmt<DT>::EPC], const uint32_t *cid, float *cdist,
                                   int cnt, int lane) {
    constexpr int RPP = GatherShape<LPR, CPL>::RPP;
    constexpr int U = GatherShape<LPR, CPL>::U;
    constexpr int U2 = U < 2 ? U : 2, U4 = U < 4 ? U : 4;
    const unsigned char *lane_base = T.base + (lane % LPR) * 16;
    const bool part = DT == NSG_F32 && LPR * CPL > T.row_chunks;   // wave-uniform
    for (int r0 = 0; r0 < cnt; r0 += U * RPP) {
        const int left = cnt - r0;
        if (left <= RPP)
            gather_round<DT, LPR, CPL, 1>(T, lane_base, qv, sc, cid, cdist, r0, cnt, lane, part);
        else if (U > 2 && left <= 2 * RPP)
            gather_round<DT, LPR, CPL, U2>(T, lane_base, qv, sc, cid, cdist, r0, cnt, lane, part);
        else if (U > 4 && left <= 4 * RPP)
            gather_round<DT, LPR, CPL, U4>(T, lane_base, qv, sc, cid, cdist, r0, cnt, lane, part);
        else
            gather_round<DT, LPR, CPL, U>(T, lane_base, qv, sc, cid, cdist, r0, cnt, lane, part);
    }
}

// Merge the candidates (cid[r], cdist[r]), r < cnt, into the pool: those
// below the current L-th key are inserted one by one (rp_insert drops keys the
// pool holds and keys pushed to rank Lcur or beyond).
template <int NCH>
__device__ __attribute__((always_inline)) inline void merge_cands(RegPool<NCH> &P, const uint32_t *cid,
                                                                  const float *cdist, int cnt, int Lcur,
                                                                  int lane) {
    for (int b = 0; b < cnt; b += 64) {
        const uint64_t worst = P.size >= Lcur ? rp_get<NCH>(P, Lcur - 1) : KEY_NONE;
        const int r = b + lane;
        uint64_t key = KEY_NONE;
        if (r < cnt) {
            const uint64_t kk = mk_key(cdist[r], cid[r]);
            if (kk < worst) key = kk;
        }
        uint64_t sm = __ballot(key != KEY_NONE);
        while (sm) {
            const int l = __builtin_ctzll(sm);
            sm &= sm - 1ull;
            rp_insert<NCH>(P, readlane64(key, l), Lcur, lane);
        }
    }
}

}  // namespace nsg
