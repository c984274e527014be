// Host runtime and C ABI of libpic_hip.so (declared in include/pic.h).
//
// A context owns all device memory of one simulation: the SoA particle
// arrays of every species twice over (the re-sort writes into the other
// buffer), the supercell offsets, the six Yee field arrays, two J buffers
// (the step deposits into one while the other keeps the previous step's J for
// readout and is cleared by the Yee pass), the sort scratch and a device
// error word.  All work is queued on the context's stream; pic_step waits
// only for the final 4-byte error word.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pic.h"
#include "pic_internal.h"

using namespace pic;

namespace {

thread_local std::string g_create_error;

struct SpeciesState {
    SpeciesC c;
    int64_t capacity = 0;
    int64_t n = 0;
    Parts buf[2] = {};         // FP64 arrays (PIC_FP64)
    PartsM bufm[2] = {};       // packed arrays (PIC_FP32_MIXED)
    SpeciesM cm{};             // FP32 constants of the mixed-precision push
    int cur = 0;               // buffer holding the particles
    int* sc_off = nullptr;     // supercell offsets of the (new) order
    int* sc_prev = nullptr;    // supercell offsets of the order before the last re-sort
    unsigned* keys = nullptr;  // sort keys written by the push before a re-sort
    unsigned* perm = nullptr;  // re-sort order: new index -> index in buf[cur]
    bool pending = false;      // buf[cur] is still in the old order; apply perm
    bool moved = false;        // the re-sort ending this step moved the data (perm valid)
    bool loaded = false;
};

// Mean particles per supercell from which a re-sort also moves the particle
// data into the new order (the neighbourhood re-sort's staged move, or after
// the global sort the staged permutation) rather than leaving the order for
// the next push to read through.
constexpr int64_t kStagedPermuteMin = 1024;

enum Stage { ST_PUSH = 0, ST_PUSH_PERM = 1, ST_FAR = 2, ST_FDTD = 3, ST_SORT = 4, ST_TOTAL = 5,
             ST_N = 6 };

struct TimedRange {
    hipEvent_t a, b;
    int stage;
};

__global__ void iota_kernel(int64_t* id, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        id[i] = i;
}

// A saved state of the context: per species the particles in stored order
// (no pending re-sort) with ids and supercell offsets, E, B, the J of the
// last step, and the step counters.  Device memory owned by the checkpoint.
struct Checkpoint {
    int64_t steps = 0;
    int64_t rebins = 0;
    int since_sort = 0;
    std::vector<int64_t> n;
    std::vector<Parts> parts;
    std::vector<int*> sc_off;
    double* EBJ[9] = {};
    std::vector<void*> mem;
};

}  // namespace

struct pic_ctx {
    int device = 0;
    int precision = PIC_FP64;
    DetJ det{};              // deterministic J: integer accumulators (hi[0] == nullptr: off)
    double* stage[6] = {};   // mixed precision: FP64 staging of x, y, z, ux, uy, uz
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Geom g{};
    int R = 1;
    std::vector<SpeciesState> sp;
    double* E[3] = {};     // current fields
    double* B[3] = {};
    double* Eo[3] = {};    // second pair: the Yee update writes here, then the pairs swap
    double* Bo[3] = {};
    double* J[2][3] = {};
    int jcur = 0;     // J buffer holding the last step's current
    int jdep = 1;     // J buffer the next step deposits into (zero)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    unsigned* d_err = nullptr;
    unsigned long long* d_nfar = nullptr;
    int* far_q = nullptr;          // far-mover queue (capacity of the largest species)
    unsigned* far_n = nullptr;     // two queue counters, used alternately by launches
    int far_phase = 0;
    int pair_phase = 0;            // counters far_n[4..7] of the two-species launch
    unsigned* h_err = nullptr;
    unsigned* h_far = nullptr;     // pinned, coherent: raised by a re-sort's classification
    unsigned* d_far = nullptr;     // (distant particles); d_far is its device address
    hipEvent_t ev_sort = nullptr;  // recorded after that classification
    double* rho = nullptr;
    double* tmp = nullptr;
    double* G0 = nullptr;
    double* divB0 = nullptr;
    double* d_acc = nullptr;                 // W_E, W_B, then one kinetic sum per species
    double* d_live = nullptr;                // live particles per species (absorbing x)
    unsigned long long* d_max = nullptr;     // 2 words
    bool ref_dirty = true;
    bool any_loaded = false;
    int64_t steps = 0;
    int steps_since_sort = 0;
    int64_t rebins = 0;
    int timers = 0;        // 0 off, 1 every stage, 2 the stored-order push+deposit kernel only,
                           // 3 that kernel on one timed step in seven
    double t_ms[ST_N] = {};
    int64_t push_launches = 0;       // push+deposit launches in stored order
    int64_t push_perm_launches = 0;  // push+deposit launches reading through a re-sort order
    int64_t timed_steps = 0;
    std::vector<hipEvent_t> ev_free;
    std::vector<TimedRange> ranges;
    std::vector<void*> allocs;
    std::string err;
    double laser_amp = 0.0;            // laser sheet (absorbing x only)
    double laser_omega = 0.0;
    double laser_T = 0.0;
    int laser_plane = -1;              // -1: off
    bool recording = false;            // pic_record .. pic_backward
    int rec_every = 1;
    int64_t rec_start = 0;             // step count at pic_record
    std::vector<Checkpoint> ckpts;     // at rec_start, rec_start + rec_every, ...
};

namespace {

int fail(pic_ctx* c, int code, const std::string& msg) {
    c->err = msg;
    return code;
}

int hip_fail(pic_ctx* c, hipError_t e, const char* what) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE;
}

#define HIPCHK(ctx, expr)                                   \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

hipError_t dalloc(pic_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) c->allocs.push_back(*p);
    return e;
}

void free_checkpoint(Checkpoint& k) {
    for (void* p : k.mem) (void)hipFree(p);
    k.mem.clear();
}

void end_recording(pic_ctx* c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& k : c->ckpts) free_checkpoint(k);
    c->ckpts.clear();
    c->recording = false;
}

void release(pic_ctx* c) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    end_recording(c);
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->h_err) (void)hipHostFree(c->h_err);
    c->h_err = nullptr;
    if (c->h_far) (void)hipHostFree(c->h_far);
    c->h_far = nullptr;
    if (c->ev_sort) (void)hipEventDestroy(c->ev_sort);
    c->ev_sort = nullptr;
    for (auto& r : c->ranges) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    c->ranges.clear();
    for (auto e : c->ev_free) (void)hipEventDestroy(e);
    c->ev_free.clear();
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
}

hipEvent_t take_event(pic_ctx* c) {
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Timer mode 3 brackets the stored-order push of one timed step in
// kPushSampleStride (7, coprime with the usual re-sort periods, so that the
// samples fall on every step of a period in turn).  An event pair costs the
// stream about 5.6 us on each side of the bracketed kernel.
constexpr int64_t kPushSampleStride = 7;

bool push_sampled(const pic_ctx* c) {
    return c->timers != 3 || c->timed_steps % kPushSampleStride == 0;
}

// Brackets a launch sequence with events when timers are on.
struct Timed {
    pic_ctx* c;
    int stage;
    hipEvent_t a = nullptr;
    Timed(pic_ctx* c_, int st) : c(c_), stage(st) {
        if (c->timers == 1 || (c->timers >= 2 && st == ST_PUSH && push_sampled(c))) {
            a = take_event(c);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    ~Timed() {
        if (c->timers && a) {
            hipEvent_t b = take_event(c);
            if (b) {
                (void)hipEventRecord(b, c->stream);
                c->ranges.push_back({a, b, stage});
            } else {
                c->ev_free.push_back(a);
            }
        }
    }
};

// After the stream has drained: fold recorded ranges into the totals.
void collect_timers(pic_ctx* c) {
    for (auto& r : c->ranges) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) c->t_ms[r.stage] += ms;
        c->ev_free.push_back(r.a);
        c->ev_free.push_back(r.b);
    }
    c->ranges.clear();
}

bool bad_ptr(const void* p, int64_t n) { return n > 0 && p == nullptr; }

int sync_and_check(pic_ctx* c, bool stepping) {
    HIPCHK(c, hipMemcpyAsync(c->h_err, c->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    collect_timers(c);
    const unsigned e = *c->h_err;
    if (e & ERR_NONFINITE)
        return fail(c, PIC_ENONFINITE, "a particle state became non-finite during a step");
    if (e & ERR_DETCAP)
        return fail(c, PIC_ECAPACITY,
                    "deterministic J: a supercell holds more than 16383 particles of one species");
    if (e & ERR_BADPOS)
        return fail(c, stepping ? PIC_ENONFINITE : PIC_EINVAL,
                    "particle positions must be finite and inside [0, n) with finite momenta");
    if (e & ERR_SORT)
        return fail(c, PIC_EDEVICE, "internal error: inconsistent counts in the re-sort");
    return PIC_OK;
}

// FP64 positions and momenta of a species in stored order: the particle
// arrays themselves, or (mixed precision) their conversion into the staging
// arrays, valid until the next use of the staging arrays.
hipError_t fp64_view(pic_ctx* c, const SpeciesState& s, Parts& v) {
    if (c->precision == PIC_FP64) {
        v = s.buf[s.cur];
        return hipSuccess;
    }
    v = Parts{c->stage[0], c->stage[1], c->stage[2], c->stage[3], c->stage[4], c->stage[5],
              s.bufm[s.cur].id};
    return launch_to_double(s.n, s.bufm[s.cur], c->stage, c->stream);
}

int compute_refs(pic_ctx* c) {
    const int64_t nc = c->g.ncell;
    HIPCHK(c, launch_zero(c->rho, nc, c->stream));
    const double dv = c->g.dx[0] * c->g.dx[1] * c->g.dx[2];
    for (auto& s : c->sp) {
        if (s.n == 0) continue;
        Parts p;
        HIPCHK(c, fp64_view(c, s, p));
        HIPCHK(c, launch_rho(c->g, (s.c.q * s.c.w) / dv, p.x, p.y, p.z, s.n, c->rho, c->stream));
    }
    Fields f{{c->E[0], c->E[1], c->E[2]}, {c->B[0], c->B[1], c->B[2]}};
    HIPCHK(c, launch_gauss(c->g, f, c->rho, c->G0, c->stream));
    HIPCHK(c, launch_divb(c->g, f, c->divB0, c->stream));
    c->ref_dirty = false;
    return PIC_OK;
}

// The arrays of a species from its current buffer to the other one.
MoveArrays move_arrays(const pic_ctx* c, const SpeciesState& s) {
    MoveArrays mv;
    if (c->precision == PIC_FP64) {
        const Parts& a = s.buf[s.cur];
        const Parts& b = s.buf[1 - s.cur];
        const void* src[7] = {a.x, a.y, a.z, a.ux, a.uy, a.uz, a.id};
        void* dst[7] = {b.x, b.y, b.z, b.ux, b.uy, b.uz, b.id};
        for (int k = 0; k < 7; ++k) {
            mv.src[k] = src[k];
            mv.dst[k] = dst[k];
            mv.bytes[k] = 8;
        }
        mv.count = 7;
    } else {
        const PartsM& a = s.bufm[s.cur];
        const PartsM& b = s.bufm[1 - s.cur];
        const void* src[8] = {a.cell, a.ox, a.oy, a.oz, a.ux, a.uy, a.uz, a.id};
        void* dst[8] = {b.cell, b.ox, b.oy, b.oz, b.ux, b.uy, b.uz, b.id};
        for (int k = 0; k < 8; ++k) {
            mv.src[k] = src[k];
            mv.dst[k] = dst[k];
            mv.bytes[k] = k < 7 ? 4 : 8;
        }
        mv.count = 8;
    }
    return mv;
}

// Order of the next re-sort from the keys written by the last push (or from
// the positions when keys == nullptr).  after_push: keys come from the push of
// the step that ends now, and the current order is grouped by the supercells
// of sc_off, so the neighbourhood re-sort applies (unless a particle moved
// farther than the neighbouring supercells); with dense supercells it also
// moves the data into the new order.  Otherwise (a load, or the global sort)
// the data move later: with the next push, or by the staged permutation.
int do_sort(pic_ctx* c, SpeciesState& s, const unsigned* keys, bool after_push) {
    HIPCHK(c, launch_resort_prep(c->g, s.n, s.sc_off, s.sc_prev, c->scratch, c->stream));
    bool done = false;
    const bool local = after_push && keys && !c->g.absorb_x;
    const bool move = local && s.n >= (int64_t)kStagedPermuteMin * c->g.nsc;
    const MoveArrays mv = move_arrays(c, s);
    if (local)
        HIPCHK(c, launch_sort_local(c->g, s.n, keys, s.sc_prev, s.perm, s.sc_off, c->scratch,
                                    c->d_err, move ? &mv : nullptr, c->h_far, c->d_far, c->ev_sort,
                                    c->stream, &done));
    if (done && move) {
        s.cur = 1 - s.cur;
        s.pending = false;
        s.moved = true;
        return PIC_OK;
    }
    if (!done)
        HIPCHK(c, launch_sort(c->g, s.n, keys, s.buf[s.cur], s.perm, s.sc_off, c->scratch,
                              c->d_err, c->stream));
    s.pending = true;
    if (c->g.absorb_x && s.n > 0) {
        // removed particles were sorted after every supercell: the species
        // keeps the first sc_off[nsc]
        int kept = 0;
        HIPCHK(c, hipMemcpyAsync(&kept, s.sc_off + c->g.nsc, sizeof(int), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        s.n = kept;
    }
    return PIC_OK;
}

// Apply a pending re-sort order to the particle data (outside pic_step).
int resolve_pending(pic_ctx* c, SpeciesState& s) {
    if (!s.pending) return PIC_OK;
    if (c->precision == PIC_FP64)
        HIPCHK(c, launch_permute(s.n, s.perm, s.buf[s.cur], s.buf[1 - s.cur], c->stream));
    else
        HIPCHK(c, launch_permute_mixed(s.n, s.perm, s.bufm[s.cur], s.bufm[1 - s.cur], c->stream));
    s.cur = 1 - s.cur;
    s.pending = false;
    return PIC_OK;
}

// One step of every species and the Yee update, queued on the stream
// (no synchronisation); the re-sort order follows every R-th step.
int step_once(pic_ctx* c) {
    for (auto& s : c->sp) s.moved = false;
    const Fields f{{c->E[0], c->E[1], c->E[2]}, {c->B[0], c->B[1], c->B[2]}};
    const Fields fo{{c->Eo[0], c->Eo[1], c->Eo[2]}, {c->Bo[0], c->Bo[1], c->Bo[2]}};
    double* const* Jd = c->J[c->jdep];
    const bool sort_after = (c->steps_since_sort + 1 == c->R);
    // two species over one tile load per supercell
    const bool pair = c->sp.size() == 2 && c->precision == PIC_FP64 && c->sp[0].n > 0 &&
                      c->sp[1].n > 0 && c->sp[0].pending == c->sp[1].pending &&
                      push_deposit_pair_supported(c->g.S, c->g.h, c->det.hi[0] != nullptr);
    if (pair) {
        SpeciesC spc[2];
        Parts src[2], dst[2];
        const unsigned* perm[2];
        unsigned* keys[2];
        const int* off[2];
        int* fq[2];
        unsigned* fn[2];
        unsigned* fnn[2];
        for (int k = 0; k < 2; ++k) {
            SpeciesState& s = c->sp[k];
            spc[k] = s.c;
            src[k] = s.buf[s.cur];
            dst[k] = s.pending ? s.buf[1 - s.cur] : s.buf[s.cur];
            perm[k] = s.pending ? s.perm : nullptr;
            keys[k] = sort_after ? s.keys : nullptr;
            off[k] = s.sc_off;
            fq[k] = c->far_q + (k == 0 ? 0 : c->sp[0].capacity);
            fn[k] = c->far_n + 4 + 2 * k + c->pair_phase;
            fnn[k] = c->far_n + 4 + 2 * k + (1 - c->pair_phase);
        }
        const bool pend = c->sp[0].pending;
        {
            Timed t(c, pend ? ST_PUSH_PERM : ST_PUSH);
            HIPCHK(c, launch_push_deposit_pair(c->g, spc, src, dst, perm, keys, off, f, Jd,
                                               c->d_err, c->d_nfar, fq, fn, fnn, c->det,
                                               c->stream));
        }
        {
            Timed t(c, ST_FAR);
            for (int k = 0; k < 2; ++k)
                HIPCHK(c, launch_far_movers(c->g, spc[k], src[k], dst[k], perm[k], keys[k], f,
                                            Jd, c->d_err, c->d_nfar, fq[k], fn[k], fnn[k],
                                            c->det, c->stream));
        }
        c->pair_phase = 1 - c->pair_phase;
        if (c->timers && (pend || push_sampled(c))) (pend ? c->push_perm_launches : c->push_launches)++;
        if (pend) {
            Timed t(c, ST_SORT);
            for (int k = 0; k < 2; ++k) {
                SpeciesState& s = c->sp[k];
                HIPCHK(c, launch_permute_ids(s.n, s.perm, src[k].id, dst[k].id, c->stream));
                s.cur = 1 - s.cur;
                s.pending = false;
            }
        }
    }
    for (auto& s : c->sp) {
        if (pair) break;
        if (s.n == 0) continue;
        const bool mixed = c->precision == PIC_FP32_MIXED;
        if (s.pending && !c->g.absorb_x && s.n >= (int64_t)kStagedPermuteMin * c->g.nsc) {
            // dense supercells after the global sort: the re-sort order is
            // applied by a permutation staged through LDS, and the push reads
            // in stored order (reading through the order instead touches
            // about twelve times the cache lines per load when a supercell
            // holds thousands of particles)
            Timed t(c, ST_SORT);
            HIPCHK(c, launch_staged_permute(c->g, s.n, s.perm, s.sc_prev, s.sc_off,
                                            move_arrays(c, s), c->stream));
            s.cur = 1 - s.cur;
            s.pending = false;
        }
        const Parts& src = s.buf[s.cur];
        const Parts& dst = s.pending ? s.buf[1 - s.cur] : s.buf[s.cur];
        const PartsM& srcm = s.bufm[s.cur];
        const PartsM& dstm = s.pending ? s.bufm[1 - s.cur] : s.bufm[s.cur];
        const unsigned* perm = s.pending ? s.perm : nullptr;
        unsigned* keys = sort_after ? s.keys : nullptr;
        unsigned* fn = c->far_n + c->far_phase;
        unsigned* fn_next = c->far_n + (1 - c->far_phase);
        {
            Timed t(c, s.pending ? ST_PUSH_PERM : ST_PUSH);
            if (mixed)
                HIPCHK(c, launch_push_mixed(c->g, s.cm, srcm, dstm, perm, keys, s.sc_off,
                                            f, Jd, c->d_err, c->d_nfar, c->far_q, fn,
                                            fn_next, c->det, c->stream));
            else
                HIPCHK(c, launch_push_deposit(c->g, s.c, src, dst, perm, keys, s.sc_off,
                                              f, Jd, c->d_err, c->d_nfar, c->far_q, fn,
                                              fn_next, c->det, c->stream));
        }
        {
            Timed t(c, ST_FAR);
            if (mixed)
                HIPCHK(c, launch_far_mixed(c->g, s.cm, srcm, dstm, perm, keys, f, Jd,
                                           c->d_err, c->d_nfar, c->far_q, fn, fn_next,
                                           c->det, c->stream));
            else
                HIPCHK(c, launch_far_movers(c->g, s.c, src, dst, perm, keys, f, Jd,
                                            c->d_err, c->d_nfar, c->far_q, fn, fn_next,
                                            c->det, c->stream));
        }
        c->far_phase = 1 - c->far_phase;
        if (c->timers && (s.pending || push_sampled(c)))
            (s.pending ? c->push_perm_launches : c->push_launches)++;
        if (s.pending) {
            Timed t(c, ST_SORT);
            HIPCHK(c, launch_permute_ids(s.n, s.perm, mixed ? srcm.id : src.id,
                                         mixed ? dstm.id : dst.id, c->stream));
            s.cur = 1 - s.cur;
            s.pending = false;
        }
    }
    {
        Timed t(c, ST_FDTD);
        if (c->det.hi[0]) HIPCHK(c, launch_j_from_fixed(c->g.ncell, c->det, Jd, c->stream));
        if (c->g.absorb_x) {
            // the laser sheet's current at t = (step + 1/2) dt
            double lj = 0.0;
            if (c->laser_plane >= 0) {
                const double t = ((double)c->steps + 0.5) * c->g.dt;
                double el = 0.0;
                if (t >= 0.0 && t <= c->laser_T) {
                    const double pi = 3.14159265358979323846;
                    const double env = std::sin(pi * t / c->laser_T);
                    el = c->laser_amp * (env * env) * std::sin(c->laser_omega * t);
                }
                lj = (-2.0 * el) / c->g.dx[0];
            }
            HIPCHK(c, launch_fdtd_absorbing(c->g, f, fo, Jd, c->J[c->jcur], c->laser_plane, lj,
                                            c->stream));
        } else {
            HIPCHK(c, launch_fdtd(c->g, f, fo, Jd, c->J[c->jcur], c->stream));
        }
    }
    for (int d = 0; d < 3; ++d) {
        std::swap(c->E[d], c->Eo[d]);
        std::swap(c->B[d], c->Bo[d]);
    }
    c->jcur = c->jdep;
    c->jdep = 1 - c->jdep;
    c->steps++;
    if (c->timers) c->timed_steps++;
    if (sort_after) {
        Timed t(c, ST_SORT);
        for (auto& s : c->sp) {
            if (s.n == 0) continue;
            int r = do_sort(c, s, s.keys, true);
            if (r != PIC_OK) return r;
        }
        c->steps_since_sort = 0;
        c->rebins++;
    } else {
        c->steps_since_sort++;
    }
    return PIC_OK;
}

hipError_t ck_alloc(std::vector<void*>& mem, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) mem.push_back(*p);
    return e;
}

// Save the current state into k (allocating k's memory on first use).  A
// pending re-sort is applied first, so the checkpoint holds the particles in
// the order the next push reads them.
int save_checkpoint(pic_ctx* c, Checkpoint& k) {
    const size_t fb = (size_t)c->g.ncell * sizeof(double);
    const size_t ob = (size_t)(c->g.nsc + 1) * sizeof(int);
    const size_t ns = c->sp.size();
    for (auto& s : c->sp) {
        int r = resolve_pending(c, s);
        if (r != PIC_OK) return r;
    }
    if (k.mem.empty()) {
        k.n.assign(ns, 0);
        k.parts.assign(ns, Parts{});
        k.sc_off.assign(ns, nullptr);
        for (int i = 0; i < 9; ++i) HIPCHK(c, ck_alloc(k.mem, (void**)&k.EBJ[i], fb));
        for (size_t si = 0; si < ns; ++si) {
            const size_t pb = (size_t)c->sp[si].n * sizeof(double);
            Parts& P = k.parts[si];
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.x, pb));
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.y, pb));
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.z, pb));
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.ux, pb));
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.uy, pb));
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.uz, pb));
            HIPCHK(c, ck_alloc(k.mem, (void**)&P.id, (size_t)c->sp[si].n * sizeof(int64_t)));
            HIPCHK(c, ck_alloc(k.mem, (void**)&k.sc_off[si], ob));
        }
    }
    const double* src[9] = {c->E[0], c->E[1], c->E[2], c->B[0], c->B[1], c->B[2],
                            c->J[c->jcur][0], c->J[c->jcur][1], c->J[c->jcur][2]};
    for (int i = 0; i < 9; ++i)
        HIPCHK(c, hipMemcpyAsync(k.EBJ[i], src[i], fb, hipMemcpyDeviceToDevice, c->stream));
    for (size_t si = 0; si < ns; ++si) {
        const SpeciesState& s = c->sp[si];
        const Parts& S = s.buf[s.cur];
        const Parts& P = k.parts[si];
        k.n[si] = s.n;
        const size_t pb = (size_t)s.n * sizeof(double);
        if (s.n > 0) {
            HIPCHK(c, hipMemcpyAsync(P.x, S.x, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(P.y, S.y, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(P.z, S.z, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(P.ux, S.ux, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(P.uy, S.uy, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(P.uz, S.uz, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(P.id, S.id, (size_t)s.n * sizeof(int64_t),
                                     hipMemcpyDeviceToDevice, c->stream));
        }
        HIPCHK(c, hipMemcpyAsync(k.sc_off[si], s.sc_off, ob, hipMemcpyDeviceToDevice, c->stream));
    }
    k.steps = c->steps;
    k.rebins = c->rebins;
    k.since_sort = c->steps_since_sort;
    return PIC_OK;
}

int restore_checkpoint(pic_ctx* c, const Checkpoint& k) {
    const size_t fb = (size_t)c->g.ncell * sizeof(double);
    const size_t ob = (size_t)(c->g.nsc + 1) * sizeof(int);
    double* dst[9] = {c->E[0], c->E[1], c->E[2], c->B[0], c->B[1], c->B[2],
                      c->J[c->jcur][0], c->J[c->jcur][1], c->J[c->jcur][2]};
    for (int i = 0; i < 9; ++i)
        HIPCHK(c, hipMemcpyAsync(dst[i], k.EBJ[i], fb, hipMemcpyDeviceToDevice, c->stream));
    for (size_t si = 0; si < c->sp.size(); ++si) {
        SpeciesState& s = c->sp[si];
        s.pending = false;
        s.n = k.n[si];
        const Parts& D = s.buf[s.cur];
        const Parts& P = k.parts[si];
        const size_t pb = (size_t)s.n * sizeof(double);
        if (s.n > 0) {
            HIPCHK(c, hipMemcpyAsync(D.x, P.x, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(D.y, P.y, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(D.z, P.z, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(D.ux, P.ux, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(D.uy, P.uy, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(D.uz, P.uz, pb, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(D.id, P.id, (size_t)s.n * sizeof(int64_t),
                                     hipMemcpyDeviceToDevice, c->stream));
        }
        HIPCHK(c, hipMemcpyAsync(s.sc_off, k.sc_off[si], ob, hipMemcpyDeviceToDevice, c->stream));
    }
    c->steps = k.steps;
    c->rebins = k.rebins;
    c->steps_since_sort = k.since_sort;
    return PIC_OK;
}

// Reverse sweep over the recorded run (see pic_backward).  lEB and lam are
// the adjoint of the current state on entry and of the recorded start on
// return; the context's state is left at some recomputed step (the caller
// restores it).
int backward_sweep(pic_ctx* c, double* const lEB[6], std::vector<std::array<double*, 6>>& lam,
                   std::vector<std::array<double*, 6>>& lam2, std::vector<void*>& mem) {
    const size_t fb = (size_t)c->g.ncell * sizeof(double);
    const size_t ns = c->sp.size();
    const int64_t K = c->steps - c->rec_start;
    const int every = c->rec_every;
    const int seg_len = (int)std::min<int64_t>(every, K);
    double* lJ[3];
    for (int d = 0; d < 3; ++d) HIPCHK(c, ck_alloc(mem, (void**)&lJ[d], fb));
    // forward state of every step of one segment
    std::vector<std::array<double*, 6>> stEB(seg_len);
    std::vector<std::vector<std::array<double*, 6>>> stP(seg_len,
                                                         std::vector<std::array<double*, 6>>(ns));
    std::vector<std::vector<unsigned*>> stPerm(seg_len, std::vector<unsigned*>(ns, nullptr));
    std::vector<std::vector<char>> sorted(seg_len, std::vector<char>(ns, 0));
    for (int j = 0; j < seg_len; ++j) {
        for (int k = 0; k < 6; ++k) HIPCHK(c, ck_alloc(mem, (void**)&stEB[j][k], fb));
        for (size_t si = 0; si < ns; ++si) {
            const int64_t n = c->sp[si].n;
            for (int k = 0; k < 6; ++k)
                HIPCHK(c, ck_alloc(mem, (void**)&stP[j][si][k], (size_t)n * sizeof(double)));
            HIPCHK(c, ck_alloc(mem, (void**)&stPerm[j][si], (size_t)n * sizeof(unsigned)));
        }
    }
    for (int seg = (int)c->ckpts.size() - 1; seg >= 0; --seg) {
        const int64_t s0 = c->ckpts[seg].steps - c->rec_start;
        const int64_t s1 = std::min<int64_t>(s0 + every, K);
        if (s1 <= s0) continue;
        int r = restore_checkpoint(c, c->ckpts[seg]);
        if (r != PIC_OK) return r;
        const int len = (int)(s1 - s0);
        for (int j = 0; j < len; ++j) {
            const double* F[6] = {c->E[0], c->E[1], c->E[2], c->B[0], c->B[1], c->B[2]};
            for (int k = 0; k < 6; ++k)
                HIPCHK(c, hipMemcpyAsync(stEB[j][k], F[k], fb, hipMemcpyDeviceToDevice, c->stream));
            for (size_t si = 0; si < ns; ++si) {
                const SpeciesState& s = c->sp[si];
                if (s.n == 0) continue;
                const Parts& P = s.buf[s.cur];
                const double* src[6] = {P.x, P.y, P.z, P.ux, P.uy, P.uz};
                for (int k = 0; k < 6; ++k)
                    HIPCHK(c, hipMemcpyAsync(stP[j][si][k], src[k], (size_t)s.n * sizeof(double),
                                             hipMemcpyDeviceToDevice, c->stream));
            }
            r = step_once(c);
            if (r != PIC_OK) return r;
            for (size_t si = 0; si < ns; ++si) {
                SpeciesState& s = c->sp[si];
                sorted[j][si] = (s.pending || s.moved) ? 1 : 0;
                if (!sorted[j][si]) continue;
                HIPCHK(c, hipMemcpyAsync(stPerm[j][si], s.perm, (size_t)s.n * sizeof(unsigned),
                                         hipMemcpyDeviceToDevice, c->stream));
                r = resolve_pending(c, s);
                if (r != PIC_OK) return r;
            }
        }
        for (int j = len - 1; j >= 0; --j) {
            for (size_t si = 0; si < ns; ++si) {
                const int64_t n = c->sp[si].n;
                if (n == 0 || !sorted[j][si]) continue;
                HIPCHK(c, launch_unpermute(n, stPerm[j][si], lam[si].data(), lam2[si].data(),
                                           c->stream));
                std::swap(lam[si], lam2[si]);
            }
            double* lE[3] = {lEB[0], lEB[1], lEB[2]};
            double* lB[3] = {lEB[3], lEB[4], lEB[5]};
            HIPCHK(c, launch_fdtd_adjoint(c->g, lE, lB, lJ, c->stream));
            for (size_t si = 0; si < ns; ++si) {
                const SpeciesState& s = c->sp[si];
                if (s.n == 0) continue;
                const double* st[6] = {stP[j][si][0], stP[j][si][1], stP[j][si][2],
                                       stP[j][si][3], stP[j][si][4], stP[j][si][5]};
                const double* F[6] = {stEB[j][0], stEB[j][1], stEB[j][2],
                                      stEB[j][3], stEB[j][4], stEB[j][5]};
                const double* lJc[3] = {lJ[0], lJ[1], lJ[2]};
                HIPCHK(c, launch_particle_adjoint(c->g, s.c, s.n, st, F, lJc, lam[si].data(), lEB,
                                                  c->stream));
            }
        }
    }
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_eval_sqrt_div(int64_t n, const double* x, const double* a, const double* b, double* sq,
                      double* dv) {
    g_create_error.clear();
    const bool want_sq = x != nullptr || sq != nullptr;
    const bool want_dv = a != nullptr || b != nullptr || dv != nullptr;
    if (n < 0 || (want_sq && (!x || !sq)) || (want_dv && (!a || !b || !dv))) {
        g_create_error = "pic_eval_sqrt_div: n must be >= 0 and x/sq, a/b/dv given together";
        return PIC_EINVAL;
    }
    if (n == 0 || (!want_sq && !want_dv)) return PIC_OK;
    const size_t bytes = (size_t)n * sizeof(double);
    double* d[5] = {};
    auto release = [&]() {
        for (double* p : d)
            if (p) (void)hipFree(p);
    };
    auto hfail = [&](hipError_t e, const char* what) {
        g_create_error = std::string("pic_eval_sqrt_div: ") + what + ": " + hipGetErrorString(e);
        release();
        return e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE;
    };
    const double* in[3] = {x, a, b};
    const bool use[5] = {want_sq, want_dv, want_dv, want_sq, want_dv};
    for (int k = 0; k < 5; ++k) {
        if (!use[k]) continue;
        hipError_t e = hipMalloc((void**)&d[k], bytes);
        if (e != hipSuccess) return hfail(e, "hipMalloc");
        if (k < 3) {
            e = hipMemcpy(d[k], in[k], bytes, hipMemcpyDefault);
            if (e != hipSuccess) return hfail(e, "hipMemcpy");
        }
    }
    hipError_t e = launch_sqrt_div(n, d[0], d[1], d[2], d[3], d[4], nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hfail(e, "kernel");
    if (want_sq && (e = hipMemcpy(sq, d[3], bytes, hipMemcpyDefault)) != hipSuccess)
        return hfail(e, "hipMemcpy");
    if (want_dv && (e = hipMemcpy(dv, d[4], bytes, hipMemcpyDefault)) != hipSuccess)
        return hfail(e, "hipMemcpy");
    release();
    return PIC_OK;
}

int pic_eval_sqrt_div_f32(int64_t n, const float* x, const float* a, const float* b, float* sq,
                          float* dv) {
    g_create_error.clear();
    const bool want_sq = x != nullptr || sq != nullptr;
    const bool want_dv = a != nullptr || b != nullptr || dv != nullptr;
    if (n < 0 || (want_sq && (!x || !sq)) || (want_dv && (!a || !b || !dv))) {
        g_create_error = "pic_eval_sqrt_div_f32: n must be >= 0 and x/sq, a/b/dv given together";
        return PIC_EINVAL;
    }
    if (n == 0 || (!want_sq && !want_dv)) return PIC_OK;
    const size_t bytes = (size_t)n * sizeof(float);
    float* d[5] = {};
    auto release = [&]() {
        for (float* p : d)
            if (p) (void)hipFree(p);
    };
    auto hfail = [&](hipError_t e, const char* what) {
        g_create_error = std::string("pic_eval_sqrt_div_f32: ") + what + ": " +
                         hipGetErrorString(e);
        release();
        return e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE;
    };
    const float* in[3] = {x, a, b};
    const bool use[5] = {want_sq, want_dv, want_dv, want_sq, want_dv};
    for (int k = 0; k < 5; ++k) {
        if (!use[k]) continue;
        hipError_t e = hipMalloc((void**)&d[k], bytes);
        if (e != hipSuccess) return hfail(e, "hipMalloc");
        if (k < 3) {
            e = hipMemcpy(d[k], in[k], bytes, hipMemcpyDefault);
            if (e != hipSuccess) return hfail(e, "hipMemcpy");
        }
    }
    hipError_t e = launch_sqrt_div_f32(n, d[0], d[1], d[2], d[3], d[4], nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hfail(e, "kernel");
    if (want_sq && (e = hipMemcpy(sq, d[3], bytes, hipMemcpyDefault)) != hipSuccess)
        return hfail(e, "hipMemcpy");
    if (want_dv && (e = hipMemcpy(dv, d[4], bytes, hipMemcpyDefault)) != hipSuccess)
        return hfail(e, "hipMemcpy");
    release();
    return PIC_OK;
}

}  // extern "C"

namespace {

// Staging of pic_eval_sqrt_div_noalloc: one array per device, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress (per device, on the first call made
// with that device current) and only that address is used.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

}  // namespace

extern "C" {

int pic_eval_sqrt_div_noalloc(int64_t n, const double* x, const double* a, const double* b,
                              double* sq, double* dv) {
    g_create_error.clear();
    const bool want_sq = x != nullptr || sq != nullptr;
    const bool want_dv = a != nullptr || b != nullptr || dv != nullptr;
    if (n < 0 || (want_sq && (!x || !sq)) || (want_dv && (!a || !b || !dv))) {
        g_create_error = "pic_eval_sqrt_div_noalloc: n must be >= 0 and x/sq, a/b/dv given together";
        return PIC_EINVAL;
    }
    // five arrays of n doubles, each starting on a 256-byte boundary
    const size_t slot_max = (kNoAllocScratchBytes / 5) & ~(size_t)255;
    const int64_t n_max = (int64_t)(slot_max / sizeof(double));
    const size_t slot = (((size_t)(n > 0 ? n : 0) * sizeof(double)) + 255) & ~(size_t)255;
    if (n > n_max) {
        g_create_error = "pic_eval_sqrt_div_noalloc: n exceeds " + std::to_string(n_max) +
                         " (the staging holds five arrays in " +
                         std::to_string(kNoAllocScratchBytes >> 20) + " MiB)";
        return PIC_EINVAL;
    }
    if (n == 0 || (!want_sq && !want_dv)) return PIC_OK;
    auto hfail = [&](hipError_t e, const char* what) {
        g_create_error = std::string("pic_eval_sqrt_div_noalloc: ") + what + ": " +
                         hipGetErrorString(e);
        return PIC_EDEVICE;
    };
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hfail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return hfail(hipErrorInvalidDevice, "device index");
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) return hfail(e, "hipGetSymbolAddress");
            g_scratch_ptr[dev] = ptr;
        }
        base = (unsigned char*)g_scratch_ptr[dev];
    }
    double* d[5];
    for (int k = 0; k < 5; ++k) d[k] = (double*)(base + (size_t)k * slot);
    const size_t bytes = (size_t)n * sizeof(double);
    const double* in[3] = {x, a, b};
    const bool use_in[3] = {want_sq, want_dv, want_dv};
    for (int k = 0; k < 3; ++k)
        if (use_in[k] && (e = hipMemcpy(d[k], in[k], bytes, hipMemcpyDefault)) != hipSuccess)
            return hfail(e, "hipMemcpy");
    e = launch_sqrt_div(n, want_sq ? d[0] : nullptr, want_dv ? d[1] : nullptr,
                        want_dv ? d[2] : nullptr, want_sq ? d[3] : nullptr,
                        want_dv ? d[4] : nullptr, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hfail(e, "kernel");
    if (want_sq && (e = hipMemcpy(sq, d[3], bytes, hipMemcpyDefault)) != hipSuccess)
        return hfail(e, "hipMemcpy");
    if (want_dv && (e = hipMemcpy(dv, d[4], bytes, hipMemcpyDefault)) != hipSuccess)
        return hfail(e, "hipMemcpy");
    return PIC_OK;
}

int pic_create(const pic_grid_t* grid, const double dx[3], double dt,
               const pic_species_t* species, int32_t n_species, pic_ctx** out) {
    g_create_error.clear();
    auto bad = [](const std::string& m) {
        g_create_error = m;
        return PIC_EINVAL;
    };
    if (!out) return bad("out must not be NULL");
    *out = nullptr;
    if (!grid || !dx) return bad("grid and dx must not be NULL");
    if (n_species < 1 || n_species > 64 || !species)
        return bad("n_species must be in [1, 64] with a species array");
    if (grid->reserved != 0) return bad("the reserved grid field must be zero");
    if (grid->bc_x != PIC_BC_PERIODIC && grid->bc_x != PIC_BC_ABSORBING)
        return bad("bc_x must be PIC_BC_PERIODIC or PIC_BC_ABSORBING");
    if (grid->deterministic_j != 0 && grid->deterministic_j != 1)
        return bad("deterministic_j must be 0 or 1");
    if (grid->precision != PIC_FP64 && grid->precision != PIC_FP32_MIXED)
        return bad("precision must be PIC_FP64 or PIC_FP32_MIXED");
    if (grid->precision == PIC_FP32_MIXED &&
        (grid->n[0] > 1024 || grid->n[1] > 1024 || grid->n[2] > 1024))
        return bad("PIC_FP32_MIXED supports at most 1024 cells per dimension");
    const int S = grid->supercell;
    if (S < 1) return bad("supercell must be >= 1");
    if (grid->rebin_every < 1) return bad("rebin_every must be >= 1");
    const int h = grid->halo == 0 ? 1 : grid->halo;
    if (!push_deposit_supported(S, h))
        return bad("unsupported (supercell, halo) pair: the LDS tiles would not fit");
    if (grid->bc_x == PIC_BC_ABSORBING) {
        if (grid->precision != PIC_FP64 || grid->deterministic_j)
            return bad("PIC_BC_ABSORBING needs PIC_FP64 without deterministic_j");
        if (!((S == 2 || S == 4) && (h == 1 || h == 2)))
            return bad("PIC_BC_ABSORBING needs supercell 2 or 4 with halo 1 or 2");
        if (grid->n[0] < 3) return bad("PIC_BC_ABSORBING needs n[0] >= 3");
    }
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (grid->n[d] < 1) return bad("grid dimensions must be >= 1");
        if (grid->n[d] % S != 0) return bad("every grid dimension must be a multiple of supercell");
        ncell *= grid->n[d];
        if (!(dx[d] > 0.0) || !std::isfinite(dx[d])) return bad("dx must be finite and > 0");
    }
    if (ncell >= (int64_t(1) << 31)) return bad("grid too large (>= 2^31 cells)");
    if (!(dt > 0.0) || !std::isfinite(dt)) return bad("dt must be finite and > 0");
    const double lim = 1.0 / std::sqrt(1.0 / (dx[0] * dx[0]) + 1.0 / (dx[1] * dx[1]) +
                                       1.0 / (dx[2] * dx[2]));
    if (dt > lim * (1.0 + 1e-12)) return bad("dt exceeds the Yee (Courant) stability limit");
    for (int s = 0; s < n_species; ++s) {
        const pic_species_t& q = species[s];
        if (!std::isfinite(q.charge) || !(q.mass > 0.0) || !std::isfinite(q.mass) ||
            !(q.weight > 0.0) || !std::isfinite(q.weight))
            return bad("species charge must be finite, mass and weight finite and > 0");
        if (q.capacity < 0 || q.capacity >= (int64_t(1) << 29))
            return bad("species capacity must be in [0, 2^29)");
        // the Boris kick h = q dt / (2 m) enters a division whose operand
        // ranges the push kernel relies on
        const double hq = std::fabs((q.charge * dt) / (2.0 * q.mass));
        if (hq != 0.0 && !(hq > 0x1p-900 && hq < 0x1p900))
            return bad("|charge dt / (2 mass)| must be 0 or within (2^-900, 2^900)");
        // the FP32 push divides (float) h by values >= 1
        const double hf = std::fabs((double)(float)((q.charge * dt) / (2.0 * q.mass)));
        if (grid->precision == PIC_FP32_MIXED && hf != 0.0 && !(hf > 0x1p-60 && hf < 0x1p60))
            return bad("mixed precision: |charge dt / (2 mass)| must be 0 or within "
                       "(2^-60, 2^60) in FP32");
    }

    pic_ctx* c = new (std::nothrow) pic_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return PIC_ENOMEM;
    }
    auto cfail = [&](int code) {
        g_create_error = c->err;
        release(c);
        delete c;
        return code;
    };
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return cfail(hip_fail(c, e, "hipGetDevice"));
    if (grid->stream) {
        c->stream = (hipStream_t)grid->stream;
    } else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return cfail(hip_fail(c, e, "hipStreamCreateWithFlags"));
        c->own_stream = true;
    }
    Geom& g = c->g;
    for (int d = 0; d < 3; ++d) {
        g.n[d] = grid->n[d];
        g.ns[d] = grid->n[d] / S;
        g.dx[d] = dx[d];
        g.cdt[d] = dt / dx[d];
    }
    g.ncell = (int)ncell;
    g.S = S;
    g.nsc = g.ns[0] * g.ns[1] * g.ns[2];
    g.h = h;
    g.dt = dt;
    g.absorb_x = grid->bc_x == PIC_BC_ABSORBING ? 1 : 0;
    c->R = grid->rebin_every;
    c->precision = grid->precision;

    const size_t fb = (size_t)ncell * sizeof(double);
    for (int d = 0; d < 3; ++d) {
        if ((e = dalloc(c, (void**)&c->E[d], fb)) != hipSuccess) return cfail(hip_fail(c, e, "hipMalloc E"));
        if ((e = dalloc(c, (void**)&c->B[d], fb)) != hipSuccess) return cfail(hip_fail(c, e, "hipMalloc B"));
        if ((e = dalloc(c, (void**)&c->Eo[d], fb)) != hipSuccess) return cfail(hip_fail(c, e, "hipMalloc E"));
        if ((e = dalloc(c, (void**)&c->Bo[d], fb)) != hipSuccess) return cfail(hip_fail(c, e, "hipMalloc B"));
        for (int b = 0; b < 2; ++b)
            if ((e = dalloc(c, (void**)&c->J[b][d], fb)) != hipSuccess)
                return cfail(hip_fail(c, e, "hipMalloc J"));
    }
    if ((e = dalloc(c, (void**)&c->rho, fb)) != hipSuccess ||
        (e = dalloc(c, (void**)&c->tmp, fb)) != hipSuccess ||
        (e = dalloc(c, (void**)&c->G0, fb)) != hipSuccess ||
        (e = dalloc(c, (void**)&c->divB0, fb)) != hipSuccess ||
        (e = dalloc(c, (void**)&c->d_acc, (2 + 64) * sizeof(double))) != hipSuccess ||
        (e = dalloc(c, (void**)&c->d_live, 64 * sizeof(double))) != hipSuccess ||
        (e = dalloc(c, (void**)&c->d_max, 2 * sizeof(unsigned long long))) != hipSuccess ||
        (e = dalloc(c, (void**)&c->d_err, 256)) != hipSuccess ||
        (e = dalloc(c, (void**)&c->d_nfar, 256)) != hipSuccess ||
        (e = dalloc(c, (void**)&c->far_n, 256)) != hipSuccess)
        return cfail(hip_fail(c, e, "hipMalloc"));
    if ((e = hipHostMalloc((void**)&c->h_err, 256, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void**)&c->h_far, 64, hipHostMallocMapped | hipHostMallocCoherent)) !=
            hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&c->d_far, c->h_far, 0)) != hipSuccess)
        return cfail(hip_fail(c, e, "hipHostMalloc"));
    if ((e = hipEventCreateWithFlags(&c->ev_sort, hipEventDisableTiming)) != hipSuccess)
        return cfail(hip_fail(c, e, "hipEventCreate"));
    int64_t maxcap = 0;
    c->sp.resize(n_species);
    for (int s = 0; s < n_species; ++s) {
        SpeciesState& st = c->sp[s];
        const pic_species_t& q = species[s];
        st.c.q = q.charge;
        st.c.m = q.mass;
        st.c.w = q.weight;
        st.c.hq = (q.charge * dt) / (2.0 * q.mass);
        const double qw = q.charge * q.weight;
        for (int d = 0; d < 3; ++d) {
            const double area = dx[(d + 1) % 3] * dx[(d + 2) % 3];
            st.c.jc[d] = qw / (dt * area);
        }
        st.cm.h = (float)st.c.hq;
        for (int d = 0; d < 3; ++d) {
            st.cm.jc[d] = (float)st.c.jc[d];
            st.cm.cdt[d] = (float)(dt / dx[d]);
        }
        st.capacity = q.capacity;
        if (q.capacity > maxcap) maxcap = q.capacity;
        // one spare slot past the end of every state array (see Parts::spare)
        const size_t pb = (size_t)(q.capacity + 1) * sizeof(double);
        const size_t fb4 = (size_t)(q.capacity + 1) * sizeof(float);
        for (int b = 0; b < 2 && c->precision == PIC_FP32_MIXED; ++b) {
            PartsM& P = st.bufm[b];
            if ((e = dalloc(c, (void**)&P.cell, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.ox, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.oy, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.oz, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.ux, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.uy, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.uz, fb4)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.id, (size_t)q.capacity * sizeof(int64_t))) != hipSuccess)
                return cfail(hip_fail(c, e, "hipMalloc particles"));
            P.spare = (unsigned)q.capacity;
        }
        for (int b = 0; b < 2 && c->precision == PIC_FP64; ++b) {
            Parts& P = st.buf[b];
            if ((e = dalloc(c, (void**)&P.x, pb)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.y, pb)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.z, pb)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.ux, pb)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.uy, pb)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.uz, pb)) != hipSuccess ||
                (e = dalloc(c, (void**)&P.id, (size_t)q.capacity * sizeof(int64_t))) != hipSuccess)
                return cfail(hip_fail(c, e, "hipMalloc particles"));
            P.spare = (unsigned)q.capacity;
        }
        if ((e = dalloc(c, (void**)&st.sc_off, (size_t)(g.nsc + 1) * sizeof(int))) != hipSuccess ||
            (e = dalloc(c, (void**)&st.sc_prev, (size_t)(g.nsc + 1) * sizeof(int))) != hipSuccess ||
            (e = dalloc(c, (void**)&st.keys, (size_t)q.capacity * sizeof(unsigned))) != hipSuccess ||
            (e = dalloc(c, (void**)&st.perm, (size_t)q.capacity * sizeof(unsigned))) != hipSuccess)
            return cfail(hip_fail(c, e, "hipMalloc sc_off / keys / perm"));
    }
    // far-mover queue: one slot per particle of the largest species, or of
    // the first two species together (their two-species launch fills two
    // queues at once)
    int64_t qcap = maxcap;
    if (n_species == 2) qcap = species[0].capacity + species[1].capacity;
    if ((e = dalloc(c, (void**)&c->far_q, (size_t)(qcap > 0 ? qcap : 1) * sizeof(int))) !=
        hipSuccess)
        return cfail(hip_fail(c, e, "hipMalloc far queue"));
    if (grid->deterministic_j) {
        // scale 2^k with 4 * (sum of capacities) * max |q w / (dt area)| * 2^k <= 2^62:
        // no sum of hi parts can overflow
        double bound = 0.0;
        for (auto& st : c->sp) {
            double jm = 0.0;
            for (int d = 0; d < 3; ++d) jm = std::fmax(jm, std::fabs(st.c.jc[d]));
            bound += 4.0 * (double)(st.capacity > 0 ? st.capacity : 1) * jm;
        }
        int k = 0;
        if (bound > 0.0) {
            (void)std::frexp(bound, &k);       // bound < 2^k
            k = 62 - k;
        }
        if (k > 900) k = 900;
        if (k < -900) k = -900;
        c->det.scale = std::ldexp(1.0, k);
        for (int d = 0; d < 3; ++d)
            if ((e = dalloc(c, (void**)&c->det.hi[d], fb)) != hipSuccess ||
                (e = dalloc(c, (void**)&c->det.lo[d], fb)) != hipSuccess ||
                (e = hipMemsetAsync(c->det.hi[d], 0, fb, c->stream)) != hipSuccess ||
                (e = hipMemsetAsync(c->det.lo[d], 0, fb, c->stream)) != hipSuccess)
                return cfail(hip_fail(c, e, "hipMalloc deterministic J"));
    }
    if (c->precision == PIC_FP32_MIXED)
        for (int k = 0; k < 6; ++k)
            if ((e = dalloc(c, (void**)&c->stage[k], (size_t)(maxcap > 0 ? maxcap : 1) *
                                                         sizeof(double))) != hipSuccess)
                return cfail(hip_fail(c, e, "hipMalloc staging"));
    c->scratch_bytes = rebin_scratch_bytes(maxcap, g);
    if ((e = dalloc(c, &c->scratch, c->scratch_bytes)) != hipSuccess)
        return cfail(hip_fail(c, e, "hipMalloc sort scratch"));
    // fields, both J buffers, counters to zero
    for (int d = 0; d < 3; ++d) {
        if ((e = launch_zero(c->E[d], ncell, c->stream)) != hipSuccess ||
            (e = launch_zero(c->B[d], ncell, c->stream)) != hipSuccess ||
            (e = launch_zero(c->J[0][d], ncell, c->stream)) != hipSuccess ||
            (e = launch_zero(c->J[1][d], ncell, c->stream)) != hipSuccess)
            return cfail(hip_fail(c, e, "zero fields"));
    }
    if ((e = hipMemsetAsync(c->d_err, 0, 256, c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->d_nfar, 0, 256, c->stream)) != hipSuccess ||
        (e = hipMemsetAsync(c->far_n, 0, 256, c->stream)) != hipSuccess)
        return cfail(hip_fail(c, e, "hipMemsetAsync"));
    for (auto& st : c->sp) {
        // no particles yet: every supercell empty
        if ((e = launch_sort(g, 0, nullptr, st.buf[0], st.perm, st.sc_off, c->scratch, c->d_err,
                             c->stream)) != hipSuccess)
            return cfail(hip_fail(c, e, "init offsets"));
    }
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return cfail(hip_fail(c, e, "hipStreamSynchronize"));
    *out = c;
    return PIC_OK;
}

int pic_load_particles(pic_ctx* c, int32_t species, int64_t n, const double* x, const double* y,
                       const double* z, const double* ux, const double* uy, const double* uz,
                       const int64_t* id) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (species < 0 || species >= (int)c->sp.size()) return fail(c, PIC_EINVAL, "bad species index");
    SpeciesState& s = c->sp[species];
    if (n < 0) return fail(c, PIC_EINVAL, "n must be >= 0");
    if (c->recording) end_recording(c);
    if (n > s.capacity) return fail(c, PIC_ECAPACITY, "n exceeds the species capacity");
    if (bad_ptr(x, n) || bad_ptr(y, n) || bad_ptr(z, n) || bad_ptr(ux, n) || bad_ptr(uy, n) ||
        bad_ptr(uz, n))
        return fail(c, PIC_EINVAL, "particle arrays must not be NULL");
    HIPCHK(c, hipSetDevice(c->device));
    const bool mixed = c->precision == PIC_FP32_MIXED;
    Parts& P = s.buf[0];
    int64_t* const idp = mixed ? s.bufm[0].id : P.id;
    double* const dst[6] = {mixed ? c->stage[0] : P.x, mixed ? c->stage[1] : P.y,
                            mixed ? c->stage[2] : P.z, mixed ? c->stage[3] : P.ux,
                            mixed ? c->stage[4] : P.uy, mixed ? c->stage[5] : P.uz};
    const double* const src[6] = {x, y, z, ux, uy, uz};
    const size_t b = (size_t)n * sizeof(double);
    HIPCHK(c, hipMemsetAsync(c->d_err, 0, sizeof(unsigned), c->stream));
    if (n > 0) {
        for (int k = 0; k < 6; ++k)
            HIPCHK(c, hipMemcpyAsync(dst[k], src[k], b, hipMemcpyDefault, c->stream));
        if (id) {
            HIPCHK(c, hipMemcpyAsync(idp, id, (size_t)n * sizeof(int64_t), hipMemcpyDefault,
                                     c->stream));
        } else {
            int nb = (int)((n + 255) / 256);
            if (nb > 65536) nb = 65536;
            hipLaunchKernelGGL(iota_kernel, dim3(nb), dim3(256), 0, c->stream, idp, n);
            HIPCHK(c, hipGetLastError());
        }
        if (mixed)
            HIPCHK(c, launch_to_mixed(c->g, n, c->stage, s.bufm[0], s.keys, c->d_err, c->stream));
    }
    s.n = n;
    s.cur = 0;
    s.pending = false;
    {
        Timed t(c, ST_SORT);
        int r = do_sort(c, s, mixed ? s.keys : nullptr, false);
        if (r == PIC_OK) r = resolve_pending(c, s);
        if (r != PIC_OK) return r;
    }
    int r = sync_and_check(c, false);
    if (r != PIC_OK) {
        s.n = 0;
        s.pending = false;
        (void)launch_sort(c->g, 0, nullptr, s.buf[0], s.perm, s.sc_off, c->scratch, c->d_err,
                          c->stream);
        (void)hipStreamSynchronize(c->stream);
        return r;
    }
    s.loaded = true;
    c->any_loaded = true;
    c->steps_since_sort = 0;
    c->ref_dirty = true;
    return PIC_OK;
}

int pic_set_fields(pic_ctx* c, const double* const EB[6]) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!EB) return fail(c, PIC_EINVAL, "EB must not be NULL");
    for (int k = 0; k < 6; ++k)
        if (!EB[k]) return fail(c, PIC_EINVAL, "EB entries must not be NULL");
    HIPCHK(c, hipSetDevice(c->device));
    if (c->recording) end_recording(c);
    const size_t fb = (size_t)c->g.ncell * sizeof(double);
    for (int d = 0; d < 3; ++d) {
        HIPCHK(c, hipMemcpyAsync(c->E[d], EB[d], fb, hipMemcpyDefault, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->B[d], EB[3 + d], fb, hipMemcpyDefault, c->stream));
        HIPCHK(c, launch_zero(c->J[0][d], c->g.ncell, c->stream));
        HIPCHK(c, launch_zero(c->J[1][d], c->g.ncell, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->ref_dirty = true;
    return PIC_OK;
}

int pic_set_laser(pic_ctx* c, double amplitude, double omega, double duration,
                  int32_t plane) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!c->g.absorb_x) return fail(c, PIC_EINVAL, "the laser source needs PIC_BC_ABSORBING");
    if (!std::isfinite(amplitude) || !std::isfinite(omega) || !(omega >= 0.0) ||
        !std::isfinite(duration) || !(duration > 0.0))
        return fail(c, PIC_EINVAL, "laser: finite amplitude, omega >= 0 and duration > 0 needed");
    if (plane < 1 || plane > c->g.n[0] - 2)
        return fail(c, PIC_EINVAL, "laser plane must lie in [1, n0 - 2]");
    c->laser_amp = amplitude;
    c->laser_omega = omega;
    c->laser_T = duration;
    c->laser_plane = amplitude == 0.0 ? -1 : plane;
    return PIC_OK;
}

int pic_step(pic_ctx* c, int32_t n_steps) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (n_steps < 0) return fail(c, PIC_EINVAL, "n_steps must be >= 0");
    if (!c->any_loaded) return fail(c, PIC_ESTATE, "pic_step before any pic_load_particles");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemsetAsync(c->d_err, 0, sizeof(unsigned), c->stream));
    if (c->ref_dirty) {
        int r = compute_refs(c);
        if (r != PIC_OK) return r;
    }
    {
        Timed total(c, ST_TOTAL);
        for (int it = 0; it < n_steps; ++it) {
            int r = step_once(c);
            if (r != PIC_OK) return r;
            if (c->recording && (c->steps - c->rec_start) % c->rec_every == 0) {
                c->ckpts.emplace_back();
                r = save_checkpoint(c, c->ckpts.back());
                if (r != PIC_OK) return r;
            }
        }
    }
    return sync_and_check(c, true);
}

int pic_get_fields(pic_ctx* c, double* const EBJ[9]) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!EBJ) return fail(c, PIC_EINVAL, "EBJ must not be NULL");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t fb = (size_t)c->g.ncell * sizeof(double);
    const double* src[9] = {c->E[0], c->E[1], c->E[2], c->B[0], c->B[1], c->B[2],
                            c->J[c->jcur][0], c->J[c->jcur][1], c->J[c->jcur][2]};
    for (int k = 0; k < 9; ++k)
        if (EBJ[k]) HIPCHK(c, hipMemcpyAsync(EBJ[k], src[k], fb, hipMemcpyDefault, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

int pic_get_particles(pic_ctx* c, int32_t species, int64_t capacity, int64_t* n_out, double* x,
                      double* y, double* z, double* ux, double* uy, double* uz, int64_t* id) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (species < 0 || species >= (int)c->sp.size()) return fail(c, PIC_EINVAL, "bad species index");
    if (!n_out) return fail(c, PIC_EINVAL, "n_out must not be NULL");
    SpeciesState& s = c->sp[species];
    *n_out = s.n;
    if (capacity < s.n) return fail(c, PIC_ECAPACITY, "caller capacity is smaller than n");
    HIPCHK(c, hipSetDevice(c->device));
    {
        int r = resolve_pending(c, s);
        if (r != PIC_OK) return r;
    }
    Parts P;
    HIPCHK(c, fp64_view(c, s, P));
    const size_t b = (size_t)s.n * sizeof(double);
    double* dst[6] = {x, y, z, ux, uy, uz};
    const double* src[6] = {P.x, P.y, P.z, P.ux, P.uy, P.uz};
    if (s.n > 0) {
        for (int k = 0; k < 6; ++k)
            if (dst[k]) HIPCHK(c, hipMemcpyAsync(dst[k], src[k], b, hipMemcpyDefault, c->stream));
        if (id)
            HIPCHK(c, hipMemcpyAsync(id, P.id, (size_t)s.n * sizeof(int64_t), hipMemcpyDefault,
                                     c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

int pic_diagnostics(pic_ctx* c, double out[8]) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!out) return fail(c, PIC_EINVAL, "out must not be NULL");
    HIPCHK(c, hipSetDevice(c->device));
    if (c->ref_dirty) {
        int r = compute_refs(c);
        if (r != PIC_OK) return r;
    }
    HIPCHK(c, hipMemsetAsync(c->d_acc, 0, (2 + 64) * sizeof(double), c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_max, 0, 2 * sizeof(unsigned long long), c->stream));
    const int64_t nc = c->g.ncell;
    const double* Ep[3] = {c->E[0], c->E[1], c->E[2]};
    const double* Bp[3] = {c->B[0], c->B[1], c->B[2]};
    HIPCHK(c, launch_sum_squares(Ep, nc, c->d_acc + 0, c->stream));
    HIPCHK(c, launch_sum_squares(Bp, nc, c->d_acc + 1, c->stream));
    const double dv = c->g.dx[0] * c->g.dx[1] * c->g.dx[2];
    double qtot = 0.0;
    std::vector<double> live(c->sp.size(), 0.0);
    double* d_live = c->d_live;
    if (c->g.absorb_x) HIPCHK(c, launch_zero(d_live, (int64_t)c->sp.size(), c->stream));
    for (size_t k = 0; k < c->sp.size(); ++k) {
        const SpeciesState& s = c->sp[k];
        if (!c->g.absorb_x) qtot += s.c.q * s.c.w * (double)s.n;
        if (s.n == 0) continue;
        Parts P;
        HIPCHK(c, fp64_view(c, s, P));
        if (c->g.absorb_x)
            HIPCHK(c, launch_kinetic(P.ux, P.uy, P.uz, s.n, c->d_acc + 2 + k, c->stream, P.x,
                                     d_live + k));
        else
            HIPCHK(c, launch_kinetic(P.ux, P.uy, P.uz, s.n, c->d_acc + 2 + k, c->stream));
    }
    if (c->g.absorb_x) {
        HIPCHK(c, hipMemcpyAsync(live.data(), d_live, live.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < c->sp.size(); ++k) qtot += c->sp[k].c.q * c->sp[k].c.w * live[k];
    }
    // rho, Gauss residual and div B against the references
    HIPCHK(c, launch_zero(c->rho, nc, c->stream));
    for (auto& s : c->sp) {
        if (s.n == 0) continue;
        Parts P;
        HIPCHK(c, fp64_view(c, s, P));
        HIPCHK(c, launch_rho(c->g, (s.c.q * s.c.w) / dv, P.x, P.y, P.z, s.n, c->rho, c->stream));
    }
    Fields f{{c->E[0], c->E[1], c->E[2]}, {c->B[0], c->B[1], c->B[2]}};
    HIPCHK(c, launch_gauss(c->g, f, c->rho, c->tmp, c->stream));
    HIPCHK(c, launch_maxabs_diff(c->tmp, c->G0, nc, c->d_max + 0, c->stream));
    HIPCHK(c, launch_divb(c->g, f, c->tmp, c->stream));
    HIPCHK(c, launch_maxabs_diff(c->tmp, c->divB0, nc, c->d_max + 1, c->stream));
    double acc[2 + 64];
    unsigned long long mx[2];
    HIPCHK(c, hipMemcpyAsync(acc, c->d_acc, sizeof(acc), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(mx, c->d_max, sizeof(mx), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double K = 0.0;
    for (size_t k = 0; k < c->sp.size(); ++k) K += c->sp[k].c.w * c->sp[k].c.m * acc[2 + k];
    out[0] = 0.5 * acc[0] * dv;
    out[1] = 0.5 * acc[1] * dv;
    out[2] = K;
    out[3] = qtot;
    double g0, g1;
    std::memcpy(&g0, &mx[0], sizeof(double));
    std::memcpy(&g1, &mx[1], sizeof(double));
    out[4] = g0;
    out[5] = g1;
    out[6] = (double)c->steps * c->g.dt;
    out[7] = (double)c->steps;
    return PIC_OK;
}

int pic_enable_timers(pic_ctx* c, int32_t on) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    (void)hipStreamSynchronize(c->stream);
    collect_timers(c);
    if (on < 0 || on > 3) return fail(c, PIC_EINVAL, "timer mode must be 0, 1, 2 or 3");
    c->timers = on;
    for (int k = 0; k < ST_N; ++k) c->t_ms[k] = 0.0;
    c->push_launches = 0;
    c->push_perm_launches = 0;
    c->timed_steps = 0;
    return PIC_OK;
}

int pic_get_timers(pic_ctx* c, double ms[10]) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!ms) return fail(c, PIC_EINVAL, "ms must not be NULL");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    collect_timers(c);
    ms[0] = c->t_ms[ST_PUSH];
    ms[1] = (double)c->push_launches;
    ms[2] = c->t_ms[ST_PUSH_PERM];
    ms[3] = (double)c->push_perm_launches;
    ms[4] = c->t_ms[ST_FAR];
    ms[5] = c->t_ms[ST_FDTD];
    ms[6] = c->t_ms[ST_SORT];
    ms[7] = c->t_ms[ST_TOTAL];
    ms[8] = (double)c->timed_steps;
    ms[9] = 0.0;
    return PIC_OK;
}

int pic_get_counters(pic_ctx* c, int64_t out[4]) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!out) return fail(c, PIC_EINVAL, "out must not be NULL");
    unsigned long long nfar = 0;
    HIPCHK(c, hipMemcpyAsync(&nfar, c->d_nfar, sizeof(nfar), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = (int64_t)nfar;
    out[1] = c->rebins;
    out[2] = c->steps;
    const bool det = c->det.hi[0] != nullptr;
    out[3] = c->precision == PIC_FP64 ? push_deposit_lds_bytes(c->g, det)
                                      : push_mixed_lds_bytes(c->g, det);
    return PIC_OK;
}

int pic_record(pic_ctx* c, int32_t checkpoint_every) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (checkpoint_every < 1) return fail(c, PIC_EINVAL, "checkpoint_every must be >= 1");
    if (c->precision != PIC_FP64)
        return fail(c, PIC_EINVAL, "the adjoint supports PIC_FP64 contexts only");
    if (c->g.absorb_x)
        return fail(c, PIC_EINVAL, "the adjoint supports periodic boundaries only");
    if (!c->any_loaded) return fail(c, PIC_ESTATE, "pic_record before any pic_load_particles");
    HIPCHK(c, hipSetDevice(c->device));
    end_recording(c);
    c->rec_every = checkpoint_every;
    c->rec_start = c->steps;
    c->recording = true;
    c->ckpts.emplace_back();
    int r = save_checkpoint(c, c->ckpts.back());
    if (r == PIC_OK) r = sync_and_check(c, false);
    if (r != PIC_OK) end_recording(c);
    return r;
}

int pic_backward(pic_ctx* c, const double* const seed_fields[6],
                 const double* const* seed_particles, double* const grad_fields[6],
                 double* const* grad_particles) {
    if (!c) return PIC_EINVAL;
    c->err.clear();
    if (!c->recording) return fail(c, PIC_ESTATE, "pic_backward without pic_record");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemsetAsync(c->d_err, 0, sizeof(unsigned), c->stream));
    const size_t ns = c->sp.size();
    const int64_t nc = c->g.ncell;
    const size_t fb = (size_t)nc * sizeof(double);
    std::vector<void*> mem;
    Checkpoint fin;
    unsigned long long nfar = 0;
    const int timers = c->timers;
    int r = PIC_OK;
    auto run = [&]() -> int {
        HIPCHK(c, hipMemcpyAsync(&nfar, c->d_nfar, sizeof(nfar), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        int rr = save_checkpoint(c, fin);     // the current state; seeds are in its order
        if (rr != PIC_OK) return rr;
        double* lEB[6];
        for (int k = 0; k < 6; ++k) {
            HIPCHK(c, ck_alloc(mem, (void**)&lEB[k], fb));
            if (seed_fields && seed_fields[k])
                HIPCHK(c, hipMemcpyAsync(lEB[k], seed_fields[k], fb, hipMemcpyDefault, c->stream));
            else
                HIPCHK(c, launch_zero(lEB[k], nc, c->stream));
        }
        std::vector<std::array<double*, 6>> lam(ns), lam2(ns);
        for (size_t si = 0; si < ns; ++si) {
            const int64_t n = c->sp[si].n;
            for (int k = 0; k < 6; ++k) {
                HIPCHK(c, ck_alloc(mem, (void**)&lam[si][k], (size_t)n * sizeof(double)));
                HIPCHK(c, ck_alloc(mem, (void**)&lam2[si][k], (size_t)n * sizeof(double)));
                const double* sd = seed_particles ? seed_particles[6 * si + k] : nullptr;
                if (sd && n > 0)
                    HIPCHK(c, hipMemcpyAsync(lam[si][k], sd, (size_t)n * sizeof(double),
                                             hipMemcpyDefault, c->stream));
                else
                    HIPCHK(c, launch_zero(lam[si][k], n, c->stream));
            }
        }
        c->timers = 0;
        rr = backward_sweep(c, lEB, lam, lam2, mem);
        if (rr != PIC_OK) return rr;
        for (int k = 0; k < 6; ++k)
            if (grad_fields && grad_fields[k])
                HIPCHK(c, hipMemcpyAsync(grad_fields[k], lEB[k], fb, hipMemcpyDefault, c->stream));
        for (size_t si = 0; si < ns && grad_particles; ++si) {
            const int64_t n = c->sp[si].n;
            for (int k = 0; k < 6; ++k) {
                double* gd = grad_particles[6 * si + k];
                if (gd && n > 0)
                    HIPCHK(c, hipMemcpyAsync(gd, lam[si][k], (size_t)n * sizeof(double),
                                             hipMemcpyDefault, c->stream));
            }
        }
        return PIC_OK;
    };
    r = run();
    // back to the state of the call, whatever happened
    c->timers = timers;
    if (!fin.mem.empty()) {
        int r2 = restore_checkpoint(c, fin);
        if (r == PIC_OK) r = r2;
        if (hipMemcpyAsync(c->d_nfar, &nfar, sizeof(nfar), hipMemcpyHostToDevice, c->stream) !=
                hipSuccess && r == PIC_OK)
            r = fail(c, PIC_EDEVICE, "restoring the far-mover counter");
    }
    int r3 = sync_and_check(c, true);
    if (r == PIC_OK) r = r3;
    free_checkpoint(fin);
    for (void* p : mem) (void)hipFree(p);
    end_recording(c);
    return r;
}

const char* pic_last_error(const pic_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

void pic_destroy(pic_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    release(c);
    delete c;
}

}  // extern "C"
