// Re-sort of one species into supercell order (per-cell particle storage,
// arXiv:1608.01009 Section 3, grouped by supercells, Section 4.3).
//
// key = supercell * S^3 + cell-in-supercell (both x-fastest).  The keys are
// written by the push of the step that precedes the re-sort (or computed here
// from the positions when particles are loaded), then:
//   1. a stable LSD radix sort of (key, index) pairs, passes of <= 11-bit
//      digits (two passes up to 2^22 cells); each pass:
//        hist    per 4096-element block: digit histogram -> hist[digit][block]
//        scan    exclusive scan over hist in (digit, block) order
//        scatter per block: stable rank among equal digits (wave-level ballot
//                match, waves in element order), write to the slot;
//   2. supercell offsets from the sorted keys;
//   3. inside every supercell the cells' lists are interleaved in rounds:
//      round r holds the r-th particle of every cell with more than r, cells
//      in order, so that a wave working through a round touches 64 different
//      cells.  The result is the permutation perm (new index -> old index).
// The particle data are not moved by this global sort: the next push reads
// through perm, or the staged permutation moves them.  After a push, when no
// particle moved beyond the 27 supercells around its old one, the same order
// is built per supercell instead (the neighbourhood re-sort below), which
// with dense supercells also moves the data.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 256;          // 4 waves of 64
constexpr int kWaves = kBlock / 64;
constexpr int kRounds = 16;          // 64-element rounds per wave
constexpr int kTile = kBlock * kRounds;  // 4096 elements per block
constexpr int kMaxBits = 11;

__global__ void __launch_bounds__(kBlock) key_kernel(Geom g, int n, const double* x,
                                                     const double* y, const double* z,
                                                     const double* ux, const double* uy,
                                                     const double* uz, unsigned* key,
                                                     unsigned* err) {
    const int S = g.S;
    const int S3 = S * S * S;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double p[3] = {x[i], y[i], z[i]};
        int c[3];
        bool ok = isfinite(ux[i]) && isfinite(uy[i]) && isfinite(uz[i]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            // absorbing x: particles live in [0, n0 - 1)
            const double hi = (d == 0 && g.absorb_x) ? (double)(g.n[0] - 1) : (double)g.n[d];
            const bool in = p[d] >= 0.0 && p[d] < hi;   // false for NaN
            ok = ok && in;
            c[d] = in ? (int)floor(p[d]) : 0;
        }
        if (!ok) atomicOr(err, ERR_BADPOS);
        const int sc = c[0] / S + g.ns[0] * (c[1] / S + g.ns[1] * (c[2] / S));
        const int loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
        key[i] = (unsigned)(sc * S3 + loc);
    }
}

// Removed particles (key ncell) follow every supercell: their new slots
// [sc_off[nsc], n) take them in sorted (previous) order.
__global__ void __launch_bounds__(kBlock) tail_kernel(const unsigned* perm_sorted, int n,
                                                     const int* sc_end, unsigned* out) {
    for (int i = *sc_end + blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        out[i] = perm_sorted ? perm_sorted[i] : (unsigned)i;
}

template <int BITS>
__global__ void __launch_bounds__(kBlock) hist_kernel(const unsigned* key, int n, int shift,
                                                      int nblocks, unsigned* hist) {
    constexpr int D = 1 << BITS;
    __shared__ unsigned cnt[D];
    for (int d = threadIdx.x; d < D; d += kBlock) cnt[d] = 0;
    __syncthreads();
    const int b0 = blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(key[i] >> shift) & (D - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < D; d += kBlock) hist[d * nblocks + blockIdx.x] = cnt[d];
}

// Exclusive scan, three phases over chunks of kTile elements.  skip (when
// not null): the launch does nothing if *skip != 0 (a decision taken on the
// device by an earlier kernel of the stream).
__global__ void __launch_bounds__(kBlock) scan_reduce_kernel(const unsigned* in, int n,
                                                             unsigned* sums,
                                                             const unsigned* skip) {
    if (skip && *skip != 0u) return;
    __shared__ unsigned red[kBlock];
    const int b0 = blockIdx.x * kTile;
    unsigned s = 0;
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + r * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Block-wide exclusive scan of one value per thread (Hillis-Steele in LDS).
__device__ unsigned block_exscan(unsigned v, unsigned* tmp) {
    tmp[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const unsigned add = ((int)threadIdx.x >= o) ? tmp[threadIdx.x - o] : 0u;
        __syncthreads();
        tmp[threadIdx.x] += add;
        __syncthreads();
    }
    const unsigned incl = tmp[threadIdx.x];
    __syncthreads();
    return incl - v;
}

// Single workgroup: exclusive scan of up to kTile chunk sums, in place.
// Exclusive scan of the m block sums in one workgroup, kTile at a time with
// a running carry (m may exceed kTile for more than 2^24 histogram entries).
__global__ void __launch_bounds__(kBlock) scan_sums_kernel(unsigned* sums, int m,
                                                           const unsigned* skip) {
    if (skip && *skip != 0u) return;
    __shared__ unsigned tmp[kBlock];
    __shared__ unsigned carry_s;
    unsigned carry = 0;
    for (int c0 = 0; c0 < m; c0 += kTile) {
        unsigned local[kRounds];
        unsigned s = 0;
        for (int r = 0; r < kRounds; ++r) {
            const int i = c0 + threadIdx.x * kRounds + r;
            local[r] = (i < m) ? sums[i] : 0u;
            s += local[r];
        }
        unsigned run = block_exscan(s, tmp) + carry;
        for (int r = 0; r < kRounds; ++r) {
            const int i = c0 + threadIdx.x * kRounds + r;
            if (i < m) sums[i] = run;
            run += local[r];
        }
        if (threadIdx.x == kBlock - 1) carry_s = run;
        __syncthreads();
        carry = carry_s;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) scan_down_kernel(const unsigned* in, int n,
                                                           const unsigned* sums, unsigned* out,
                                                           const unsigned* skip) {
    if (skip && *skip != 0u) return;
    __shared__ unsigned tmp[kBlock];
    const int b0 = blockIdx.x * kTile;
    unsigned local[kRounds];
    unsigned s = 0;
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + threadIdx.x * kRounds + r;
        local[r] = (i < n) ? in[i] : 0u;
        s += local[r];
    }
    unsigned run = block_exscan(s, tmp) + sums[blockIdx.x];
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + threadIdx.x * kRounds + r;
        if (i < n) out[i] = run;
        run += local[r];
    }
}

// val_in == nullptr means the identity (val = element index).
template <int BITS>
__global__ void __launch_bounds__(kBlock) scatter_kernel(const unsigned* key_in,
                                                         const unsigned* val_in, int n, int shift,
                                                         int nblocks, const unsigned* offs,
                                                         unsigned* key_out, unsigned* val_out) {
    constexpr int D = 1 << BITS;
    __shared__ unsigned wcnt[kWaves][D];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * D; d += kBlock) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int wbase = blockIdx.x * kTile + w * (kRounds * 64);
    unsigned kk[kRounds], vv[kRounds], pos[kRounds];
    // rounds in element order: the ranks of a wave's later rounds follow its
    // earlier rounds, and wave w's elements precede wave w+1's
    for (int r = 0; r < kRounds; ++r) {
        const int i = wbase + r * 64 + lane;
        const bool valid = i < n;
        const unsigned k = valid ? key_in[i] : 0u;
        const unsigned dgt = (k >> shift) & (D - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const unsigned long long bb = __ballot(valid && ((dgt >> b) & 1u));
            peers &= ((dgt >> b) & 1u) ? bb : ~bb;
        }
        unsigned rank = 0, base = 0;
        if (valid) {
            rank = (unsigned)__popcll(peers & lt);
            base = wcnt[w][dgt];
        }
        // all lanes have read their base before the first peer lane adds
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcnt[w][dgt] = base + (unsigned)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        kk[r] = k;
        vv[r] = valid ? (val_in ? val_in[i] : (unsigned)i) : 0u;
        pos[r] = base + rank;
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, plus the block's global offset
    for (int d = threadIdx.x; d < D; d += kBlock) {
        unsigned run = offs[d * nblocks + blockIdx.x];
        for (int ww = 0; ww < kWaves; ++ww) {
            const unsigned c = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int r = 0; r < kRounds; ++r) {
        const int i = wbase + r * 64 + lane;
        if (i < n) {
            const unsigned dgt = (kk[r] >> shift) & (D - 1);
            const unsigned o = wcnt[w][dgt] + pos[r];
            key_out[o] = kk[r];
            val_out[o] = vv[r];
        }
    }
}

// sc_off[s] = first sorted index whose supercell is >= s; sc_off[nsc] = n.
__global__ void __launch_bounds__(kBlock) offsets_kernel(const unsigned* key, int n, int S3,
                                                         int nsc, int* sc_off) {
    // supercell of a key: a shift when S^3 is a power of two (S = 1, 2, 4)
    const int sh = (S3 & (S3 - 1)) == 0 ? __builtin_ctz((unsigned)S3) : -1;
    auto sc_of = [&](unsigned k) { return (int)(sh >= 0 ? k >> sh : k / (unsigned)S3); };
    for (int i = blockIdx.x * kBlock + threadIdx.x; i <= n; i += gridDim.x * kBlock) {
        const int prev = (i == 0) ? -1 : sc_of(key[i - 1]);
        const int cur = (i == n) ? nsc : sc_of(key[i]);
        for (int s = prev + 1; s <= cur; ++s) sc_off[s] = i;
    }
}

// One workgroup per supercell.  With cnt_l the particle count of cell l and
// rank the position of a particle among its cell's particles, its place in the
// round order is start + A[rank] + #{l < cell : cnt_l > rank}, where
// A[r] = sum_l min(cnt_l, r).  For up to kMaxRounds rounds the per-round
// masks of cells with cnt_l > r make that O(1) per particle.
constexpr int kMaxS3 = 256;
constexpr int kMaskWords = kMaxS3 / 64;
constexpr int kMaxRounds = 512;

__global__ void __launch_bounds__(kBlock) interleave_kernel(const unsigned* __restrict__ key,
                                                            const unsigned* __restrict__ perm_sorted,
                                                            const int* __restrict__ sc_off, int S3,
                                                            unsigned* __restrict__ out) {
    __shared__ int cnt[kMaxS3];
    __shared__ int cst[kMaxS3];
    __shared__ int rstart[kMaxRounds + 1];
    __shared__ unsigned long long rmask[kMaxRounds][kMaskWords];
    __shared__ int maxc_s;
    const int sc = blockIdx.x;
    const int s0 = sc_off[sc], s1 = sc_off[sc + 1];
    if (s0 >= s1) return;
    const unsigned kb = (unsigned)sc * (unsigned)S3;
    // cell starts straight from the sorted keys: the particle where the cell
    // changes starts every cell from the previous particle's cell + 1 to its
    // own (no atomics: consecutive lanes mostly share a cell); the cells after
    // the last particle start at s1
    for (int i = s0 + threadIdx.x; i < s1; i += kBlock) {
        const int loc = (int)(key[i] - kb);
        const int prev = (i == s0) ? -1 : (int)(key[i - 1] - kb);
        for (int l = prev + 1; l <= loc; ++l) cst[l] = i;
        if (i == s1 - 1)
            for (int l = loc + 1; l < S3; ++l) cst[l] = s1;
    }
    __syncthreads();
    for (int l = threadIdx.x; l < S3; l += kBlock) cnt[l] = (l + 1 < S3 ? cst[l + 1] : s1) - cst[l];
    __syncthreads();
    const int nwords = (S3 + 63) / 64;
    if (threadIdx.x < 64) {
        // wave 0: the largest count, 64 cells at a time
        const int lane = threadIdx.x;
        int mx = 0;
        for (int w = 0; w < nwords; ++w) {
            const int l = 64 * w + lane;
            const int c = l < S3 ? cnt[l] : 0;
            mx = c > mx ? c : mx;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int t = __shfl_xor(mx, o, 64);
            mx = t > mx ? t : mx;
        }
        if (lane == 0) maxc_s = mx;
        // round masks (cells with more than r particles, one ballot per 64
        // cells) and round starts (prefix of the round sizes)
        if (mx <= kMaxRounds) {
            int run = 0;
            for (int r = 0; r < mx; ++r) {
                if (lane == 0) rstart[r] = run;
                for (int w = 0; w < nwords; ++w) {
                    const int l = 64 * w + lane;
                    const unsigned long long m = __ballot(l < S3 && cnt[l] > r);
                    if (lane == 0) rmask[r][w] = m;
                    run += __popcll(m);
                }
            }
            if (lane == 0) rstart[mx] = run;
        }
    }
    __syncthreads();
    const int maxc = maxc_s;
    if (maxc <= kMaxRounds) {
        // independent iterations (out does not alias the inputs): unrolled so
        // that several key loads are in flight per lane
#pragma unroll 4
        for (int i = s0 + threadIdx.x; i < s1; i += kBlock) {
            const int loc = (int)(key[i] - kb);
            const int rank = i - cst[loc];
            int pos = s0 + rstart[rank];
            const int lw = loc >> 6, lb = loc & 63;
            for (int w = 0; w < lw; ++w) pos += __popcll(rmask[rank][w]);
            pos += __popcll(rmask[rank][lw] & ((1ull << lb) - 1ull));
            out[pos] = perm_sorted ? perm_sorted[i] : (unsigned)i;
        }
    } else {
        for (int i = s0 + threadIdx.x; i < s1; i += kBlock) {
            const int loc = (int)(key[i] - kb);
            const int rank = i - cst[loc];
            int pos = s0;
            for (int l = 0; l < S3; ++l) {
                const int c = cnt[l];
                pos += (c < rank ? c : rank) + ((l < loc && c > rank) ? 1 : 0);
            }
            out[pos] = perm_sorted ? perm_sorted[i] : (unsigned)i;
        }
    }
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Give each XCD a contiguous range of blocks: the gathered reads of one
// supercell's particles (old slots close to each other) then share one L2.
__device__ __forceinline__ int xcd_range_block(int b, int nb) {
    if ((nb & 7) != 0) return b;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

// dst[i] = src[perm[i]] for the six state arrays and the ids; each XCD takes
// a contiguous range of the new order, so that the gathered reads of the
// supercells in flight on it (old slots close to each other) share its L2.
__global__ void __launch_bounds__(kBlock) permute_kernel(int n, const unsigned* __restrict__ perm,
                                                         Parts src, Parts dst) {
    const int b = xcd_range_block((int)blockIdx.x, (int)gridDim.x);
    for (int i = b * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const unsigned j = perm[i];
        dst.x[i] = src.x[j];
        dst.y[i] = src.y[j];
        dst.z[i] = src.z[j];
        dst.ux[i] = src.ux[j];
        dst.uy[i] = src.uy[j];
        dst.uz[i] = src.uz[j];
        dst.id[i] = src.id[j];
    }
}

__global__ void __launch_bounds__(kBlock) permute_ids_kernel(int n,
                                                             const unsigned* __restrict__ perm,
                                                             const int64_t* __restrict__ src,
                                                             int64_t* __restrict__ dst) {
    const int b = xcd_range_block((int)blockIdx.x, (int)gridDim.x);
    for (int i = b * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        dst[i] = src[perm[i]];
}

// dst[i] = src[perm[i]] for the six state arrays and the ids, one workgroup
// per supercell of the new order: most of a supercell's particles were in
// the same supercell before (its old block [old_off[s], old_off[s + 1])),
// so each array's old block is first copied into LDS with coalesced reads,
// and the new block is then written with coalesced stores, its values taken
// from LDS or, for the particles that arrived from other supercells (and
// the part of an old block beyond the LDS buffer), from global memory.
constexpr int kStageBlock = 512;
constexpr int kStage = 4096;   // 8-byte values per array held in LDS (or 8192 4-byte ones)

// One array of the staged permutation: the old block staged in LDS (up to
// CAP elements), then dst[i] = src[perm[i]] for the new block, from LDS when
// the source is in the staged part.  The loads of a thread's elements are
// issued together (KB per round) before their values are used, so that their
// latencies overlap.
constexpr int kStageKB = 8;

template <class T, int CAP>
__device__ __forceinline__ void staged_move(const T* __restrict__ sp, T* __restrict__ dp,
                                            T* stage, const unsigned* __restrict__ perm, int o0,
                                            int ob, int n0, int n1) {
    constexpr int KB = kStageKB;
    const unsigned cap = (unsigned)min(ob, CAP);
    for (int b = 0; b < (int)cap; b += KB * kStageBlock) {
        T v[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const unsigned t = (unsigned)(b + k * kStageBlock) + threadIdx.x;
            if (t < cap) v[k] = sp[o0 + (int)t];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const unsigned t = (unsigned)(b + k * kStageBlock) + threadIdx.x;
            if (t < cap) stage[t] = v[k];
        }
    }
    __syncthreads();
    for (int b = n0; b < n1; b += KB * kStageBlock) {
        unsigned jj[KB];
        T v[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int i = b + k * kStageBlock + (int)threadIdx.x;
            jj[k] = i < n1 ? perm[i] : (unsigned)o0;
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const unsigned u = jj[k] - (unsigned)o0;
            if (u >= cap) v[k] = sp[jj[k]];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const unsigned u = jj[k] - (unsigned)o0;
            if (u < cap) v[k] = stage[u];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int i = b + k * kStageBlock + (int)threadIdx.x;
            if (i < n1) dp[i] = v[k];
        }
    }
}

// The same for a new block of at most kStageKB * kStageBlock elements whose
// sources jj (perm[n0 + k * kStageBlock + thread]) the caller loaded once for
// all the arrays.
template <class T, int CAP>
__device__ __forceinline__ void staged_move_pre(const T* __restrict__ sp, T* __restrict__ dp,
                                                T* stage, const unsigned (&jj)[kStageKB], int o0,
                                                int ob, int n0, int n1) {
    constexpr int KB = kStageKB;
    const unsigned cap = (unsigned)min(ob, CAP);
    for (int b = 0; b < (int)cap; b += KB * kStageBlock) {
        T v[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const unsigned t = (unsigned)(b + k * kStageBlock) + threadIdx.x;
            if (t < cap) v[k] = sp[o0 + (int)t];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const unsigned t = (unsigned)(b + k * kStageBlock) + threadIdx.x;
            if (t < cap) stage[t] = v[k];
        }
    }
    __syncthreads();
    T v[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const unsigned u = jj[k] - (unsigned)o0;
        if (u >= cap) v[k] = sp[jj[k]];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const unsigned u = jj[k] - (unsigned)o0;
        if (u < cap) v[k] = stage[u];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int i = n0 + k * kStageBlock + (int)threadIdx.x;
        if (i < n1) dp[i] = v[k];
    }
}

__global__ void __launch_bounds__(kStageBlock) staged_permute_kernel(
    const unsigned* __restrict__ perm, const int* __restrict__ old_off,
    const int* __restrict__ new_off, MoveArrays mv, const unsigned* skip) {
    if (skip && *skip != 0u) return;   // see scan_reduce_kernel
    __shared__ unsigned long long stage[kStage];
    const int s = xcd_range_block((int)blockIdx.x, (int)gridDim.x);
    const int n0 = new_off[s], n1 = new_off[s + 1];
    if (n0 >= n1) return;
    const int o0 = old_off[s];
    const int ob = old_off[s + 1] - o0;
    if (n1 - n0 <= kStageKB * kStageBlock) {
        // the order of the block read once for every array
        unsigned jj[kStageKB];
#pragma unroll
        for (int k = 0; k < kStageKB; ++k) {
            const int i = n0 + k * kStageBlock + (int)threadIdx.x;
            jj[k] = i < n1 ? perm[i] : (unsigned)o0;
        }
#pragma unroll 1
        for (int a = 0; a < mv.count; ++a) {
            if (mv.bytes[a] == 8)
                staged_move_pre<unsigned long long, kStage>(
                    (const unsigned long long*)mv.src[a], (unsigned long long*)mv.dst[a], stage,
                    jj, o0, ob, n0, n1);
            else
                staged_move_pre<unsigned, 2 * kStage>((const unsigned*)mv.src[a],
                                                      (unsigned*)mv.dst[a], (unsigned*)stage, jj,
                                                      o0, ob, n0, n1);
            __syncthreads();
        }
        return;
    }
#pragma unroll 1
    for (int a = 0; a < mv.count; ++a) {
        if (mv.bytes[a] == 8)
            staged_move<unsigned long long, kStage>((const unsigned long long*)mv.src[a],
                                                    (unsigned long long*)mv.dst[a], stage, perm,
                                                    o0, ob, n0, n1);
        else
            staged_move<unsigned, 2 * kStage>((const unsigned*)mv.src[a], (unsigned*)mv.dst[a],
                                              (unsigned*)stage, perm, o0, ob, n0, n1);
        __syncthreads();
    }
}

// ---- neighbourhood re-sort ------------------------------------------------
// Between re-sorts a particle drifts at most a few cells, so after a push its
// new supercell is almost always one of the 27 around (periodically) the
// supercell whose block of the current order holds it.  The order of the
// stable sort by (supercell, cell) followed by the round interleave is then
// built per supercell without a global sort:
//   classify   per old supercell s': the direction (one of 27) of every
//              particle's new supercell, counts per direction, and the
//              block's slots partitioned by direction in slot order (stable);
//              particles beyond the 27 are counted as distant;
//   sizes      per new supercell: the sum of the counts directed at it by
//              its (up to 27 distinct) neighbours; exclusive scan -> offsets;
//   interleave per new supercell s: its incoming slots are the segments
//              directed at it, taken in increasing order of the source
//              supercell (= increasing slot, since the current order is
//              grouped by supercell), which is the stable order; each
//              particle's rank among its cell's particles follows from a
//              running per-cell count, and its place in the rounds from the
//              per-round masks of cells with more than r particles.
constexpr int kNbrDirs = 28;     // 27 directions + distant
constexpr int kNbrStride = 32;   // ints per supercell in the count table
constexpr int kNbrDistant = 27;
constexpr int kNbrMaxRounds = 512;

struct NbrGeom {
    int ns[3];
    int nsc;
    int s3shift;   // log2(S^3)
    int sh0, sh1;  // log2 ns[0], log2 ns[1] when both are powers of two, else -1
    float rns0, rns1;
};

// floor(a / m) for 0 <= a < 2^24, m >= 1: the float quotient is within one
// of the exact one and is corrected by the remainder.
__device__ __forceinline__ int div_small(int a, int m, float rm) {
    int q = (int)((float)a * rm);
    const int r = a - q * m;
    q += (r >= m) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

struct I3 {
    int x, y, z;
};

template <bool POW2>
__device__ __forceinline__ I3 sc_coords(int s, const NbrGeom& q) {
    I3 c;
    if (POW2) {
        c.x = s & (q.ns[0] - 1);
        const int t = s >> q.sh0;
        c.y = t & (q.ns[1] - 1);
        c.z = t >> q.sh1;
    } else {
        const int t = div_small(s, q.ns[0], q.rns0);
        c.x = s - t * q.ns[0];
        c.z = div_small(t, q.ns[1], q.rns1);
        c.y = t - c.z * q.ns[1];
    }
    return c;
}

// Direction code of the periodic offset dest - src along an axis of m
// supercells (both in [0, m)): 0 (-1), 1 (0), 2 (+1), or 3 (farther).  With
// m = 2 both neighbours are the same supercell and take code 2.
__device__ __forceinline__ int axis_code(int dest, int src, int m) {
    int v = dest - src;
    v += v < 0 ? m : 0;
    return v == 0 ? 1 : (v == 1 ? 2 : (v == m - 1 ? 0 : 3));
}

__device__ __forceinline__ int wrap_axis(int v, int m) {
    v += v < 0 ? m : 0;
    return v >= m ? v - m : v;
}

// Lanes whose value v (bits below nbits) equals this lane's, among the valid.
__device__ __forceinline__ unsigned long long match_lanes(bool valid, unsigned v, int nbits) {
    unsigned long long peers = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
        const unsigned long long bb = __ballot(valid && ((v >> b) & 1u));
        peers &= ((v >> b) & 1u) ? bb : ~bb;
    }
    return peers;
}

constexpr int kNbrBlock = 512;
constexpr int kNbrWaves = kNbrBlock / 64;
constexpr int kNbrKeepDirs = 16384;   // directions of an old block kept in LDS
constexpr int kNbrKeep = 4096;        // incoming particles of a new supercell kept in LDS

// Each wave takes a contiguous chunk of [0, n) (whole rounds of 64, waves in
// order), so that per-wave counts and their exclusive prefix over the waves
// give stable positions without a workgroup barrier per round.
template <int WAVES>
__device__ __forceinline__ void wave_chunk(int n, int w, int* c0, int* c1) {
    const int per = ((n + WAVES * 64 - 1) / (WAVES * 64)) * 64;
    *c0 = min(n, w * per);
    *c1 = min(n, *c0 + per);
}

// The supercell that direction dir of supercell sc points to.
__device__ __forceinline__ int nbr_dest(const NbrGeom& q, I3 sc, int dir) {
    const int x = wrap_axis(sc.x + dir % 3 - 1, q.ns[0]);
    const int y = wrap_axis(sc.y + (dir / 3) % 3 - 1, q.ns[1]);
    const int z = wrap_axis(sc.z + dir / 9 - 1, q.ns[2]);
    return x + q.ns[0] * (y + q.ns[1] * z);
}

template <bool POW2>
__global__ void __launch_bounds__(kNbrBlock) nbr_classify_kernel(
    NbrGeom q, const unsigned* __restrict__ key, const int* __restrict__ old_off,
    int* __restrict__ cnt_out, unsigned* __restrict__ list, unsigned* __restrict__ size,
    unsigned* __restrict__ distant, unsigned* host_flag) {
    __shared__ unsigned char dirs[kNbrKeepDirs];
    __shared__ unsigned wcnt[kNbrWaves][kNbrStride];
    __shared__ unsigned tot[kNbrStride];
    __shared__ unsigned seg[kNbrStride];
    const int s = xcd_range_block((int)blockIdx.x, (int)gridDim.x);
    const int o0 = old_off[s];
    const int nb = old_off[s + 1] - o0;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const bool keep = nb <= kNbrKeepDirs;
    const I3 sc = sc_coords<POW2>(s, q);
    for (int t = threadIdx.x; t < kNbrWaves * kNbrStride; t += kNbrBlock) (&wcnt[0][0])[t] = 0u;
    __syncthreads();
    auto dir_of_key = [&](unsigned k) -> unsigned {
        const I3 d = sc_coords<POW2>((int)(k >> q.s3shift), q);
        const int cx = axis_code(d.x, sc.x, q.ns[0]);
        const int cy = axis_code(d.y, sc.y, q.ns[1]);
        const int cz = axis_code(d.z, sc.z, q.ns[2]);
        const bool far = (cx == 3) | (cy == 3) | (cz == 3);
        return far ? (unsigned)kNbrDistant : (unsigned)(cx + 3 * cy + 9 * cz);
    };
    auto dir_of = [&](int i) -> unsigned { return dir_of_key(key[i]); };
    int c0, c1;
    wave_chunk<kNbrWaves>(nb, w, &c0, &c1);
    // directions first (independent loads, several in flight), then the
    // per-wave counts per direction (the leader of each direction's lanes
    // adds; one wave writes its own row in program order)
    if (keep) {
        constexpr int KB = 8;
        for (int b = c0 + lane; b < c1; b += 64 * KB) {
            unsigned kv[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int t = b + 64 * k;
                if (t < c1) kv[k] = key[o0 + t];
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int t = b + 64 * k;
                if (t < c1) dirs[t] = (unsigned char)dir_of_key(kv[k]);
            }
        }
    }
    for (int t0 = c0; t0 < c1; t0 += 64) {
        const int t = t0 + lane;
        const bool valid = t < c1;
        const unsigned dir = valid ? (keep ? (unsigned)dirs[t] : dir_of(o0 + t)) : 0u;
        const unsigned long long peers = match_lanes(valid, dir, 5);
        if (valid && __popcll(peers & lt) == 0) wcnt[w][dir] += (unsigned)__popcll(peers);
    }
    __syncthreads();
    if (threadIdx.x < kNbrDirs) {
        unsigned a = 0;
        for (int ww = 0; ww < kNbrWaves; ++ww) a += wcnt[ww][threadIdx.x];
        tot[threadIdx.x] = a;
        // the new supercells' sizes, summed over their sources
        if (threadIdx.x < kNbrDistant && a > 0) atomicAdd(&size[nbr_dest(q, sc, threadIdx.x)], a);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned r = 0;
        for (int d = 0; d < kNbrDirs; ++d) {
            seg[d] = r;
            r += tot[d];
        }
        seg[kNbrDirs] = r;
        if (tot[kNbrDistant] > 0) {
            atomicAdd(distant, tot[kNbrDistant]);
            // and a flag for the host, written through to its pinned memory
            __hip_atomic_store(host_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    __syncthreads();
    // segment starts in the block per direction (and the block size last)
    if (threadIdx.x <= kNbrDirs) cnt_out[(size_t)s * kNbrStride + threadIdx.x] = (int)seg[threadIdx.x];
    if (threadIdx.x < kNbrDirs) {
        unsigned b = seg[threadIdx.x];
        for (int ww = 0; ww < kNbrWaves; ++ww) {
            const unsigned c = wcnt[ww][threadIdx.x];
            wcnt[ww][threadIdx.x] = b;
            b += c;
        }
    }
    __syncthreads();
    // the block's slots partitioned by direction, in slot order
    for (int t0 = c0; t0 < c1; t0 += 64) {
        const int t = t0 + lane;
        const bool valid = t < c1;
        const unsigned dir = valid ? (keep ? (unsigned)dirs[t] : dir_of(o0 + t)) : 0u;
        const unsigned long long peers = match_lanes(valid, dir, 5);
        const unsigned rank = valid ? (unsigned)__popcll(peers & lt) : 0u;
        const unsigned base = valid ? wcnt[w][dir] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcnt[w][dir] = base + (unsigned)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (valid) list[o0 + (int)(base + rank)] = (unsigned)(o0 + t);
    }
}

// The distinct neighbours that can send particles to supercell s: along an
// axis of m supercells the offsets -1, 0, +1 (m >= 3), 0, +1 (m = 2) or 0
// (m = 1).  For neighbour k (0..26 in x-fastest order of the offsets) it
// returns false if the offset is not used, else the source supercell and the
// direction code under which that source classified particles bound for s.
__device__ __forceinline__ bool nbr_source(const NbrGeom& q, I3 sc, int k, int* src, int* dir) {
    const int cx = k % 3 - 1, cy = (k / 3) % 3 - 1, cz = k / 9 - 1;
    auto used = [](int c, int m) { return c >= (m >= 3 ? -1 : 0) && c <= (m >= 2 ? 1 : 0); };
    if (!used(cx, q.ns[0]) || !used(cy, q.ns[1]) || !used(cz, q.ns[2])) return false;
    const int x = wrap_axis(sc.x - cx, q.ns[0]);
    const int y = wrap_axis(sc.y - cy, q.ns[1]);
    const int z = wrap_axis(sc.z - cz, q.ns[2]);
    *src = x + q.ns[0] * (y + q.ns[1] * z);
    *dir = axis_code(sc.x, x, q.ns[0]) + 3 * axis_code(sc.y, y, q.ns[1]) +
           9 * axis_code(sc.z, z, q.ns[2]);
    return true;
}

// Per new supercell: its incoming slots (the segments directed at it, in
// increasing order of the source supercell), their ranks in their cells and
// places in the rounds -> perm.
constexpr int kNbrMoveBlock = 512;
constexpr int kNbrMoveWaves = kNbrMoveBlock / 64;

__global__ void __launch_bounds__(kNbrMoveBlock) nbr_interleave_kernel(
    NbrGeom q, const unsigned* __restrict__ key, const int* __restrict__ old_off,
    const int* __restrict__ seg, const unsigned* __restrict__ list,
    const int* __restrict__ new_off, unsigned* __restrict__ tmp_j, unsigned* __restrict__ tmp_c,
    unsigned* __restrict__ perm, unsigned* __restrict__ err, const unsigned* skip) {
    if (skip && *skip != 0u) return;   // see scan_reduce_kernel
    __shared__ unsigned lj[kNbrKeep];
    __shared__ unsigned char lc[kNbrKeep];
    __shared__ int k_src[27], k_start[27], k_cnt[27];
    __shared__ int o_start[27], o_pre[28];
    __shared__ int nsrc_s;
    __shared__ unsigned wcnt[kNbrMoveWaves][64];
    __shared__ unsigned ccount[64];
    __shared__ int rstart[kNbrMaxRounds + 1];
    __shared__ unsigned long long rmask[kNbrMaxRounds];
    __shared__ int maxc_s;
    const int s = xcd_range_block((int)blockIdx.x, (int)gridDim.x);
    const int n0 = new_off[s], n1 = new_off[s + 1];
    if (n0 >= n1) return;
    const int S3 = 1 << q.s3shift;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const I3 sc = q.sh0 >= 0 ? sc_coords<true>(s, q) : sc_coords<false>(s, q);
    if (threadIdx.x < 27) {
        const int k = threadIdx.x;
        int src = -1, dir = 0;
        if (nbr_source(q, sc, k, &src, &dir)) {
            const int* c = seg + (size_t)src * kNbrStride;
            const int a = c[dir], b = c[dir + 1];
            k_start[k] = old_off[src] + a;
            k_cnt[k] = b - a;
        } else {
            src = -1;
            k_start[k] = 0;
            k_cnt[k] = 0;
        }
        k_src[k] = src;
    }
    for (int t = threadIdx.x; t < kNbrMoveWaves * 64; t += kNbrMoveBlock) (&wcnt[0][0])[t] = 0u;
    __syncthreads();
    if (threadIdx.x < 27 && k_src[threadIdx.x] >= 0) {
        // place of this source in increasing source order (sources distinct)
        const int me = k_src[threadIdx.x];
        int r = 0;
        for (int k = 0; k < 27; ++k) r += (k_src[k] >= 0 && k_src[k] < me) ? 1 : 0;
        o_start[r] = k_start[threadIdx.x];
        o_pre[r + 1] = k_cnt[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nsrc = 0;
        for (int k = 0; k < 27; ++k) nsrc += k_src[k] >= 0 ? 1 : 0;
        o_pre[0] = 0;
        for (int r = 0; r < nsrc; ++r) o_pre[r + 1] += o_pre[r];
        nsrc_s = nsrc;
        if (o_pre[nsrc] != n1 - n0) atomicOr(err, ERR_SORT);
    }
    __syncthreads();
    const int nsrc = nsrc_s;
    const int N = min(n1 - n0, o_pre[nsrc]);
    const unsigned kb = (unsigned)s << q.s3shift;
    // incoming slots and their cells, in LDS when they fit
    const bool keep = N <= kNbrKeep;
    unsigned* jb = keep ? lj : tmp_j + n0;
    unsigned char* cb = keep ? lc : (unsigned char*)(tmp_c + n0);
    int c0, c1;
    wave_chunk<kNbrMoveWaves>(N, w, &c0, &c1);
    {
        // the source segment holding t is the last r < nsrc with o_pre[r] <= t;
        // a lane's t grows by 64 per round, so after one binary search its
        // segment only moves forward
        int lo = 0;
        {
            const int t = c0 + lane;
            int hi = nsrc;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (o_pre[mid] <= t)
                    lo = mid;
                else
                    hi = mid;
            }
        }
        constexpr int KB = 8;
        bool bad = false;
        for (int b = c0 + lane; b < c1; b += 64 * KB) {
            int ix[KB];
            unsigned jv[KB], kv[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int t = b + 64 * k;
                while (lo + 1 < nsrc && o_pre[lo + 1] <= t) ++lo;
                ix[k] = o_start[lo] + (t - o_pre[lo]);
            }
            // the slots, then their keys: each group of loads issued together
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (b + 64 * k < c1) jv[k] = list[ix[k]];
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (b + 64 * k < c1) kv[k] = key[jv[k]];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int t = b + 64 * k;
                if (t < c1) {
                    unsigned cell = kv[k] - kb;
                    bad = bad || cell >= (unsigned)S3;
                    cell = cell < (unsigned)S3 ? cell : 0u;
                    jb[t] = jv[k];
                    cb[t] = (unsigned char)cell;
                }
            }
        }
        if (bad) atomicOr(err, ERR_SORT);
    }
    for (int t0 = c0; t0 < c1; t0 += 64) {
        const int t = t0 + lane;
        const bool valid = t < c1;
        const unsigned cell = valid ? (unsigned)cb[t] : 0u;
        const unsigned long long peers = match_lanes(valid, cell, q.s3shift);
        if (valid && __popcll(peers & lt) == 0) wcnt[w][cell] += (unsigned)__popcll(peers);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // per cell: the exclusive prefix over the waves, and the total
        unsigned b = 0;
        for (int ww = 0; ww < kNbrMoveWaves; ++ww) {
            const unsigned c = wcnt[ww][threadIdx.x];
            wcnt[ww][threadIdx.x] = b;
            b += c;
        }
        ccount[threadIdx.x] = b;
        const int c = (int)threadIdx.x < S3 ? (int)b : 0;
        int mx = c;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int t = __shfl_xor(mx, o, 64);
            mx = t > mx ? t : mx;
        }
        if (threadIdx.x == 0) maxc_s = mx;
        if (mx <= kNbrMaxRounds) {
            int acc = 0;
            for (int r = 0; r < mx; ++r) {
                const unsigned long long m = __ballot(c > r);
                if (threadIdx.x == 0) {
                    rmask[r] = m;
                    rstart[r] = acc;
                }
                acc += __popcll(m);
            }
        }
    }
    __syncthreads();
    const int maxc = maxc_s;
    for (int t0 = c0; t0 < c1; t0 += 64) {
        const int t = t0 + lane;
        const bool valid = t < c1;
        const unsigned cell = valid ? (unsigned)cb[t] : 0u;
        const unsigned j = valid ? jb[t] : 0u;
        const unsigned long long peers = match_lanes(valid, cell, q.s3shift);
        const unsigned rw = valid ? (unsigned)__popcll(peers & lt) : 0u;
        const unsigned base = valid ? wcnt[w][cell] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && rw == 0) wcnt[w][cell] = base + (unsigned)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        if (!valid) continue;
        const int rank = (int)(base + rw);
        int pos = 0;
        if (maxc <= kNbrMaxRounds) {
            pos = rstart[rank] + __popcll(rmask[rank] & ((1ull << cell) - 1ull));
        } else {
            for (int l = 0; l < S3; ++l) {
                const int cl = (int)ccount[l];
                pos += (cl < rank ? cl : rank) + ((l < (int)cell && cl > rank) ? 1 : 0);
            }
        }
        if (pos < N)
            perm[n0 + pos] = j;
        else
            atomicOr(err, ERR_SORT);
    }
}

int nblk(int64_t n, int per) {
    int64_t b = (n + per - 1) / per;
    return b < 1 ? 1 : (int)b;
}

int grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}

// With absorbing x a removed particle has key ncell (after every cell).
int key_bits(const Geom& g) {
    unsigned maxkey = (unsigned)g.ncell - (g.absorb_x ? 0u : 1u);
    int b = 0;
    while (b < 32 && (maxkey >> b) != 0u) ++b;
    return b;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct Scratch {
    unsigned* k0;
    unsigned* v0;
    unsigned* k1;
    unsigned* v1;
    unsigned* hist;
    unsigned* offs;
    unsigned* sums;
    int* nbr_cnt;        // nsc x kNbrStride segment starts per direction
    unsigned* nbr_size;  // nsc + 1 sizes
    unsigned* nbr_sums;  // block sums of their scan
    unsigned* nbr_far;   // particles beyond the 27 neighbours
};

Scratch carve(void* base, int64_t n, int nsc) {
    const int nb = nblk(n, kTile);
    const int64_t hn = (int64_t)(1 << kMaxBits) * nb;
    char* p = (char*)base;
    Scratch s;
    const size_t kb = align_up((size_t)(n > 0 ? n : 1) * 4);
    s.k0 = (unsigned*)p; p += kb;
    s.v0 = (unsigned*)p; p += kb;
    s.k1 = (unsigned*)p; p += kb;
    s.v1 = (unsigned*)p; p += kb;
    s.hist = (unsigned*)p; p += align_up((size_t)hn * 4);
    s.offs = (unsigned*)p; p += align_up((size_t)hn * 4);
    s.sums = (unsigned*)p; p += align_up((size_t)nblk(hn, kTile) * 4);
    s.nbr_cnt = (int*)p; p += align_up((size_t)nsc * kNbrStride * 4);
    s.nbr_size = (unsigned*)p; p += (size_t)(nsc + 1) * 4;
    s.nbr_far = (unsigned*)p; p = (char*)s.nbr_size + align_up((size_t)(nsc + 2) * 4);
    s.nbr_sums = (unsigned*)p;
    return s;
}

template <int BITS>
void radix_pass(const unsigned* kin, const unsigned* vin, unsigned* kout, unsigned* vout, int n,
                int shift, const Scratch& sc, hipStream_t s) {
    const int nb = nblk(n, kTile);
    const int hn = (1 << BITS) * nb;
    const int nsum = nblk(hn, kTile);
    hipLaunchKernelGGL((hist_kernel<BITS>), dim3(nb), dim3(kBlock), 0, s, kin, n, shift, nb,
                       sc.hist);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nsum), dim3(kBlock), 0, s, sc.hist, hn, sc.sums,
                       (const unsigned*)nullptr);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kBlock), 0, s, sc.sums, nsum,
                       (const unsigned*)nullptr);
    hipLaunchKernelGGL(scan_down_kernel, dim3(nsum), dim3(kBlock), 0, s, sc.hist, hn, sc.sums,
                       sc.offs, (const unsigned*)nullptr);
    hipLaunchKernelGGL((scatter_kernel<BITS>), dim3(nb), dim3(kBlock), 0, s, kin, vin, n, shift,
                       nb, sc.offs, kout, vout);
}

void radix_pass_bits(int bits, const unsigned* kin, const unsigned* vin, unsigned* kout,
                     unsigned* vout, int n, int shift, const Scratch& sc, hipStream_t s) {
    switch (bits) {
        case 1: radix_pass<1>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 2: radix_pass<2>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 3: radix_pass<3>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 4: radix_pass<4>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 5: radix_pass<5>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 6: radix_pass<6>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 7: radix_pass<7>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 8: radix_pass<8>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 9: radix_pass<9>(kin, vin, kout, vout, n, shift, sc, s); break;
        case 10: radix_pass<10>(kin, vin, kout, vout, n, shift, sc, s); break;
        default: radix_pass<11>(kin, vin, kout, vout, n, shift, sc, s); break;
    }
}

}  // namespace

size_t rebin_scratch_bytes(int64_t n, const Geom& g) {
    const int nb = nblk(n, kTile);
    const int64_t hn = (int64_t)(1 << kMaxBits) * nb;
    const size_t kb = align_up((size_t)(n > 0 ? n : 1) * 4);
    return 4 * kb + 2 * align_up((size_t)hn * 4) + align_up((size_t)nblk(hn, kTile) * 4) +
           align_up((size_t)g.nsc * kNbrStride * 4) + align_up((size_t)(g.nsc + 2) * 4) +
           align_up((size_t)nblk((int64_t)g.nsc + 1, kTile) * 4) + 256;
}

hipError_t launch_sort(const Geom& g, int64_t n64, const unsigned* keys, const Parts& src,
                       unsigned* perm, int* sc_off, void* scratch, unsigned* err, hipStream_t s) {
    const int n = (int)n64;
    const int S3 = g.S * g.S * g.S;
    if (S3 > kMaxS3) return hipErrorInvalidValue;
    if (n == 0) {
        hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(kBlock), 0, s, (const unsigned*)nullptr,
                           0, S3, g.nsc, sc_off);
        return hipGetLastError();
    }
    Scratch sc = carve(scratch, n, g.nsc);
    if (!keys) {
        hipLaunchKernelGGL(key_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, g, n, src.x, src.y,
                           src.z, src.ux, src.uy, src.uz, sc.k0, err);
        keys = sc.k0;
    }
    const int bits = key_bits(g);
    const int npass = (bits + kMaxBits - 1) / kMaxBits;
    // pass p reads the previous pass's output (the input keys and the
    // identity for p = 0) and writes (k1, v1) for even p, (k0, v0) for odd p
    const unsigned* kin = keys;
    const unsigned* vin = nullptr;  // identity
    unsigned* kbuf[2] = {sc.k1, sc.k0};
    unsigned* vbuf[2] = {sc.v1, sc.v0};
    int shift = 0;
    for (int p = 0; p < npass; ++p) {
        const int width = (bits - shift + (npass - p) - 1) / (npass - p);
        radix_pass_bits(width, kin, vin, kbuf[p & 1], vbuf[p & 1], n, shift, sc, s);
        kin = kbuf[p & 1];
        vin = vbuf[p & 1];
        shift += width;
    }
    if (npass == 0) {
        // a single cell: the sorted order is the input order
        hipLaunchKernelGGL(offsets_kernel, dim3(grid_for((int64_t)n + 1)), dim3(kBlock), 0, s,
                           keys, n, S3, g.nsc, sc_off);
        hipLaunchKernelGGL(interleave_kernel, dim3(g.nsc), dim3(kBlock), 0, s, keys,
                           (const unsigned*)nullptr, sc_off, S3, perm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(offsets_kernel, dim3(grid_for((int64_t)n + 1)), dim3(kBlock), 0, s, kin, n,
                       S3, g.nsc, sc_off);
    hipLaunchKernelGGL(interleave_kernel, dim3(g.nsc), dim3(kBlock), 0, s, kin, vin, sc_off, S3,
                       perm);
    if (g.absorb_x)
        hipLaunchKernelGGL(tail_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, vin, n,
                           sc_off + g.nsc, perm);
    return hipGetLastError();
}

namespace {

// Start of a re-sort: the current supercell offsets copied as the old ones,
// and the neighbourhood re-sort's sizes and distant count cleared.
__global__ void __launch_bounds__(kBlock) resort_prep_kernel(const int* __restrict__ cur,
                                                             int* __restrict__ prev, int m_copy,
                                                             unsigned* __restrict__ zero,
                                                             int m_zero) {
    const int m = m_copy > m_zero ? m_copy : m_zero;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) {
        if (i < m_copy) prev[i] = cur[i];
        if (i < m_zero) zero[i] = 0u;
    }
}

}  // namespace

hipError_t launch_resort_prep(const Geom& g, int64_t n, const int* sc_off, int* sc_prev,
                              void* scratch, hipStream_t s) {
    Scratch sc = carve(scratch, n, g.nsc);
    const int m = g.nsc + 2;
    hipLaunchKernelGGL(resort_prep_kernel, dim3(nblk(m, kBlock)), dim3(kBlock), 0, s, sc_off,
                       sc_prev, g.nsc + 1, sc.nbr_size, m);
    return hipGetLastError();
}

hipError_t launch_sort_local(const Geom& g, int64_t n64, const unsigned* keys, const int* old_off,
                             unsigned* perm, int* sc_off, void* scratch, unsigned* err,
                             const MoveArrays* move, unsigned* far_host, unsigned* far_dev,
                             hipEvent_t ev, hipStream_t s, bool* done) {
    *done = false;
    const int n = (int)n64;
    const int S3 = g.S * g.S * g.S;
    if (n <= 0 || keys == nullptr || g.absorb_x || S3 > 64 || (S3 & (S3 - 1)) != 0 ||
        g.nsc >= (1 << 24))
        return hipSuccess;
    Scratch sc = carve(scratch, n, g.nsc);
    NbrGeom q;
    for (int a = 0; a < 3; ++a) q.ns[a] = g.ns[a];
    q.nsc = g.nsc;
    q.s3shift = __builtin_ctz((unsigned)S3);
    const bool pow2 = (g.ns[0] & (g.ns[0] - 1)) == 0 && (g.ns[1] & (g.ns[1] - 1)) == 0;
    q.sh0 = pow2 ? __builtin_ctz((unsigned)g.ns[0]) : -1;
    q.sh1 = pow2 ? __builtin_ctz((unsigned)g.ns[1]) : -1;
    q.rns0 = 1.0f / (float)g.ns[0];
    q.rns1 = 1.0f / (float)g.ns[1];
    // the sizes and the distant count were cleared by launch_resort_prep; the
    // classification raises *far_host (pinned host memory) if any particle is
    // distant
    *(volatile unsigned*)far_host = 0u;
    hipError_t e;
    if (pow2)
        hipLaunchKernelGGL(nbr_classify_kernel<true>, dim3(g.nsc), dim3(kNbrBlock), 0, s, q, keys,
                           old_off, sc.nbr_cnt, sc.k1, sc.nbr_size, sc.nbr_far, far_dev);
    else
        hipLaunchKernelGGL(nbr_classify_kernel<false>, dim3(g.nsc), dim3(kNbrBlock), 0, s, q, keys,
                           old_off, sc.nbr_cnt, sc.k1, sc.nbr_size, sc.nbr_far, far_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // The rest of the neighbourhood re-sort is queued behind the
    // classification: each of its kernels does nothing when the distant count
    // is not zero, and the host waits for the classification (and its flag)
    // only once they are queued, so the GPU does not idle through the wait.
    if ((e = hipEventRecord(ev, s)) != hipSuccess) return e;
    const unsigned* gate = sc.nbr_far;
    const int m = g.nsc + 1;
    const int nsum = nblk(m, kTile);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nsum), dim3(kBlock), 0, s, sc.nbr_size, m,
                       sc.nbr_sums, gate);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kBlock), 0, s, sc.nbr_sums, nsum, gate);
    hipLaunchKernelGGL(scan_down_kernel, dim3(nsum), dim3(kBlock), 0, s, sc.nbr_size, m,
                       sc.nbr_sums, (unsigned*)sc_off, gate);
    hipLaunchKernelGGL(nbr_interleave_kernel, dim3(g.nsc), dim3(kNbrMoveBlock), 0, s, q, keys,
                       old_off, (const int*)sc.nbr_cnt, (const unsigned*)sc.k1, (const int*)sc_off,
                       sc.k0, sc.v0, perm, err, gate);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (move && move->count > 0 &&
        (e = launch_staged_permute(g, n, perm, old_off, sc_off, *move, s, gate)) != hipSuccess)
        return e;
    if ((e = hipEventSynchronize(ev)) != hipSuccess) return e;
    // distant particles: the kernels above did nothing, the global sort takes over
    *done = *(volatile unsigned*)far_host == 0u;
    return hipSuccess;
}

hipError_t launch_permute(int64_t n, const unsigned* perm, const Parts& src, const Parts& dst,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, (int)n, perm, src,
                       dst);
    return hipGetLastError();
}

hipError_t launch_staged_permute(const Geom& g, int64_t n, const unsigned* perm, const int* old_off,
                                const int* new_off, const MoveArrays& mv, hipStream_t s,
                                const unsigned* skip) {
    if (n <= 0 || g.nsc <= 0 || mv.count == 0) return hipSuccess;
    if (mv.count > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(staged_permute_kernel, dim3(g.nsc), dim3(kStageBlock), 0, s, perm, old_off,
                       new_off, mv, skip);
    return hipGetLastError();
}

hipError_t launch_permute_ids(int64_t n, const unsigned* perm, const int64_t* src, int64_t* dst,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_ids_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, (int)n, perm,
                       src, dst);
    return hipGetLastError();
}

}  // namespace pic
