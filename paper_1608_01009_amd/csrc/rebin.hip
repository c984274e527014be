// Re-sort of one species into supercell order (per-cell particle storage,
// arXiv:1608.01009 Section 3, grouped by supercells, Section 4.3).
//
// key = supercell * S^3 + cell-in-supercell (both x-fastest), a stable sort
// by key, implemented as an LSD radix sort of (key, index) pairs with 8-bit
// digits.  Each pass:
//   hist    per 4096-element block: digit histogram -> hist[digit][block]
//   scan    exclusive scan over hist in (digit, block) order
//   scatter per block: stable rank of every element among equal digits
//           (wave-level ballot match, waves in order), write to its slot.
// Stability of each pass gives a stable sort overall.  The supercell offsets
// are taken from the sorted keys; then, inside every supercell, the cells'
// particle lists are interleaved in rounds (round r holds the r-th particle of
// every cell with more than r, in cell order), so that the 64 lanes of a wave
// working through a round touch 64 different cells.  The final permutation is
// applied to the SoA arrays and ids.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kBlock = 256;          // 4 waves of 64
constexpr int kWaves = kBlock / 64;
constexpr int kRounds = 16;          // 64-element rounds per wave
constexpr int kTile = kBlock * kRounds;  // 4096 elements per block
constexpr int kDigits = 256;

__global__ void __launch_bounds__(kBlock) key_kernel(Geom g, int n, const double* x,
                                                     const double* y, const double* z,
                                                     const double* ux, const double* uy,
                                                     const double* uz, unsigned* key,
                                                     unsigned* val, unsigned* err) {
    const int S = g.S;
    const int S3 = S * S * S;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double p[3] = {x[i], y[i], z[i]};
        int c[3];
        bool ok = isfinite(ux[i]) && isfinite(uy[i]) && isfinite(uz[i]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const bool in = p[d] >= 0.0 && p[d] < (double)g.n[d];   // false for NaN
            ok = ok && in;
            c[d] = in ? (int)floor(p[d]) : 0;
        }
        if (!ok) atomicOr(err, ERR_BADPOS);
        const int sc = c[0] / S + g.ns[0] * (c[1] / S + g.ns[1] * (c[2] / S));
        const int loc = c[0] % S + S * (c[1] % S + S * (c[2] % S));
        key[i] = (unsigned)(sc * S3 + loc);
        val[i] = (unsigned)i;
    }
}

__global__ void __launch_bounds__(kBlock) hist_kernel(const unsigned* key, int n, int shift,
                                                      int nblocks, unsigned* hist) {
    __shared__ unsigned cnt[kDigits];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int b0 = blockIdx.x * kTile;
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(key[i] >> shift) & (kDigits - 1)], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan, three phases over chunks of kTile elements.
__global__ void __launch_bounds__(kBlock) scan_reduce_kernel(const unsigned* in, int n,
                                                             unsigned* sums) {
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
__device__ unsigned block_exscan(unsigned v, unsigned* tmp, unsigned* total) {
    tmp[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const unsigned add = ((int)threadIdx.x >= o) ? tmp[threadIdx.x - o] : 0u;
        __syncthreads();
        tmp[threadIdx.x] += add;
        __syncthreads();
    }
    const unsigned incl = tmp[threadIdx.x];
    if (total) *total = tmp[kBlock - 1];
    __syncthreads();
    return incl - v;
}

// Single workgroup: exclusive scan of up to kTile chunk sums, in place.
__global__ void __launch_bounds__(kBlock) scan_sums_kernel(unsigned* sums, int m) {
    __shared__ unsigned tmp[kBlock];
    // each thread owns kRounds consecutive entries
    unsigned local[kRounds];
    unsigned s = 0;
    for (int r = 0; r < kRounds; ++r) {
        const int i = threadIdx.x * kRounds + r;
        local[r] = (i < m) ? sums[i] : 0u;
        s += local[r];
    }
    unsigned run = block_exscan(s, tmp, nullptr);
    for (int r = 0; r < kRounds; ++r) {
        const int i = threadIdx.x * kRounds + r;
        if (i < m) sums[i] = run;
        run += local[r];
    }
}

__global__ void __launch_bounds__(kBlock) scan_down_kernel(const unsigned* in, int n,
                                                           const unsigned* sums, unsigned* out) {
    __shared__ unsigned tmp[kBlock];
    const int b0 = blockIdx.x * kTile;
    // thread t owns the kRounds consecutive entries b0 + t*kRounds + r
    unsigned local[kRounds];
    unsigned s = 0;
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + threadIdx.x * kRounds + r;
        local[r] = (i < n) ? in[i] : 0u;
        s += local[r];
    }
    unsigned run = block_exscan(s, tmp, nullptr) + sums[blockIdx.x];
    for (int r = 0; r < kRounds; ++r) {
        const int i = b0 + threadIdx.x * kRounds + r;
        if (i < n) out[i] = run;
        run += local[r];
    }
}

__global__ void __launch_bounds__(kBlock) scatter_kernel(const unsigned* key_in,
                                                         const unsigned* val_in, int n, int shift,
                                                         int nblocks, const unsigned* offs,
                                                         unsigned* key_out, unsigned* val_out) {
    __shared__ unsigned wcnt[kWaves][kDigits];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < kWaves * kDigits; d += kBlock) (&wcnt[0][0])[d] = 0;
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
        const unsigned dgt = (k >> shift) & (kDigits - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
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
        vv[r] = valid ? val_in[i] : 0u;
        pos[r] = base + rank;
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, plus the block's global offset
    for (int d = threadIdx.x; d < kDigits; d += kBlock) {
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
            const unsigned dgt = (kk[r] >> shift) & (kDigits - 1);
            const unsigned o = wcnt[w][dgt] + pos[r];
            key_out[o] = kk[r];
            val_out[o] = vv[r];
        }
    }
}

__global__ void __launch_bounds__(kBlock) permute_kernel(int n, const unsigned* perm, Parts src,
                                                         Parts dst) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
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

// sc_off[s] = first sorted index whose supercell is >= s; sc_off[nsc] = n.
__global__ void __launch_bounds__(kBlock) offsets_kernel(const unsigned* key, int n, int S3,
                                                         int nsc, int* sc_off) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i <= n; i += gridDim.x * kBlock) {
        const int prev = (i == 0) ? -1 : (int)(key[i - 1] / (unsigned)S3);
        const int cur = (i == n) ? nsc : (int)(key[i] / (unsigned)S3);
        for (int s = prev + 1; s <= cur; ++s) sc_off[s] = i;
    }
}

// One workgroup per supercell: position of sorted element i in the round
// order, pos = start + sum_l min(cnt_l, rank) + #{l < cell : cnt_l > rank}.
constexpr int kMaxS3 = 512;

__global__ void __launch_bounds__(kBlock) interleave_kernel(const unsigned* key,
                                                            const unsigned* perm,
                                                            const int* sc_off, int S3,
                                                            unsigned* out) {
    __shared__ int cnt[kMaxS3];
    __shared__ int cst[kMaxS3];
    const int sc = blockIdx.x;
    const int s0 = sc_off[sc], s1 = sc_off[sc + 1];
    if (s0 >= s1) return;
    for (int l = threadIdx.x; l < S3; l += kBlock) cnt[l] = 0;
    __syncthreads();
    const unsigned kb = (unsigned)sc * (unsigned)S3;
    for (int i = s0 + threadIdx.x; i < s1; i += kBlock) atomicAdd(&cnt[key[i] - kb], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = s0;
        for (int l = 0; l < S3; ++l) {
            cst[l] = run;
            run += cnt[l];
        }
    }
    __syncthreads();
    for (int i = s0 + threadIdx.x; i < s1; i += kBlock) {
        const int loc = (int)(key[i] - kb);
        const int rank = i - cst[loc];
        int pos = s0;
        for (int l = 0; l < S3; ++l) {
            const int c = cnt[l];
            pos += (c < rank ? c : rank) + ((l < loc && c > rank) ? 1 : 0);
        }
        out[pos] = perm[i];
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

int key_bits(const Geom& g) {
    unsigned maxkey = (unsigned)g.ncell - 1u;
    int b = 0;
    while (b < 32 && (maxkey >> b) != 0u) ++b;
    return b;
}

// scratch layout (unsigned words)
struct Scratch {
    unsigned* k0;
    unsigned* v0;
    unsigned* k1;
    unsigned* v1;
    unsigned* hist;
    unsigned* offs;
    unsigned* sums;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

Scratch carve(void* base, int64_t n) {
    const int nb = nblk(n, kTile);
    const int64_t hn = (int64_t)kDigits * nb;
    char* p = (char*)base;
    Scratch s;
    const size_t kb = align_up((size_t)(n > 0 ? n : 1) * 4);
    s.k0 = (unsigned*)p; p += kb;
    s.v0 = (unsigned*)p; p += kb;
    s.k1 = (unsigned*)p; p += kb;
    s.v1 = (unsigned*)p; p += kb;
    s.hist = (unsigned*)p; p += align_up((size_t)hn * 4);
    s.offs = (unsigned*)p; p += align_up((size_t)hn * 4);
    s.sums = (unsigned*)p;
    return s;
}

}  // namespace

size_t rebin_scratch_bytes(int64_t n, const Geom& g) {
    (void)g;
    const int nb = nblk(n, kTile);
    const int64_t hn = (int64_t)kDigits * nb;
    const size_t kb = align_up((size_t)(n > 0 ? n : 1) * 4);
    return 4 * kb + 2 * align_up((size_t)hn * 4) + align_up((size_t)nblk(hn, kTile) * 4) + 256;
}

hipError_t launch_rebin(const Geom& g, int64_t n64, const Parts& src, const Parts& dst,
                        int* sc_off, void* scratch, unsigned* err, hipStream_t s) {
    const int n = (int)n64;
    const int S3 = g.S * g.S * g.S;
    if (n == 0) {
        hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(kBlock), 0, s, (const unsigned*)nullptr,
                           0, S3, g.nsc, sc_off);
        return hipGetLastError();
    }
    Scratch sc = carve(scratch, n);
    const int nb = nblk(n, kTile);
    const int hn = kDigits * nb;
    const int nsum = nblk(hn, kTile);
    if (nsum > kTile) return hipErrorInvalidValue;  // more than 2^24 histogram entries
    hipLaunchKernelGGL(key_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, g, n, src.x, src.y,
                       src.z, src.ux, src.uy, src.uz, sc.k0, sc.v0, err);
    const int bits = key_bits(g);
    unsigned *kin = sc.k0, *vin = sc.v0, *kout = sc.k1, *vout = sc.v1;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(hist_kernel, dim3(nb), dim3(kBlock), 0, s, kin, n, shift, nb, sc.hist);
        hipLaunchKernelGGL(scan_reduce_kernel, dim3(nsum), dim3(kBlock), 0, s, sc.hist, hn,
                           sc.sums);
        hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kBlock), 0, s, sc.sums, nsum);
        hipLaunchKernelGGL(scan_down_kernel, dim3(nsum), dim3(kBlock), 0, s, sc.hist, hn,
                           sc.sums, sc.offs);
        hipLaunchKernelGGL(scatter_kernel, dim3(nb), dim3(kBlock), 0, s, kin, vin, n, shift, nb,
                           sc.offs, kout, vout);
        unsigned* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    hipLaunchKernelGGL(offsets_kernel, dim3(grid_for((int64_t)n + 1)), dim3(kBlock), 0, s, kin, n,
                       S3, g.nsc, sc_off);
    if (S3 > kMaxS3) return hipErrorInvalidValue;
    hipLaunchKernelGGL(interleave_kernel, dim3(g.nsc), dim3(kBlock), 0, s, kin, vin, sc_off, S3,
                       kout);
    hipLaunchKernelGGL(permute_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, kout, src, dst);
    return hipGetLastError();
}

}  // namespace pic
