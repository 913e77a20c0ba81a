// rewl_internal.h -- device data layout shared by the host plan (rewl_host.cpp)
// and the kernels (rewl_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

// One (walker, e, m) cell of a window table: ln g in units of 2^-K, and the
// visit count H of stage `stamp` packed as (H << 6) | stamp.  A count written
// in an earlier stage reads as zero, so resetting H at a stage change costs
// nothing.  ln g > 0 marks a bin the walker has visited (ln g only grows).
struct Bin {
    int64_t lng;
    uint64_t hs;
};
static_assert(sizeof(Bin) == 16, "bin layout");
constexpr int STAMP_BITS = 6;
constexpr uint64_t STAMP_MASK = (1u << STAMP_BITS) - 1;

// Static description of one walker.
struct WDesc {
    uint64_t table_off;  // first bin of its (hi-lo+1) x (N+1) table
    uint32_t spin_off;   // first word of its L x row_words packed spins
    int32_t prob;        // problem index
    int32_t lo, hi;      // energy-bin window
    int32_t win;         // window index within the problem
    int32_t gid;         // walker id within the problem: win * W + a
};

// Static description of one problem.
struct PDesc {
    int32_t L, N, K, nwin, W, flat_num, flat_den, row_words;
    int64_t X;
    uint64_t seed;
    int32_t walker_off;  // first global walker index
    int32_t init;
};

// A window pair (w, w+1) of one problem that may exchange configurations.
struct PairDesc {
    int32_t prob, w;
};

// Device pointers into the three caller buffers.
struct DevState {
    const WDesc* wd;
    const PDesc* pd;
    const PairDesc* pairs;
    Bin* tables;
    uint32_t* spins;
    // per walker
    int32_t* e;
    int32_t* m;
    int64_t* t;       // WL trials made
    int64_t* te;      // entry trials made
    uint32_t* nseen;  // bins with ln g > 0
    uint32_t* flag;   // flat in the current stage (latched)
    uint32_t* scan;   // chunk where the last flatness scan failed (a hint)
    // per problem
    int32_t* stage;
    int32_t* done;
    int64_t* rnd;     // boundaries passed
    int64_t* tstage;  // trial count at the start of the stage
    int64_t* xr;      // exchange round of the boundary just closed
    int32_t* xon;     // that boundary exchanges
    int64_t* lngb;    // upper bound of any ln g entry (units), for the int64 headroom guard
    int64_t* tseen;   // trial count at the last boundary
    // misc
    int32_t* counters;  // [0] walkers outside their window (entry), [1] error bits
    int64_t n_walk;
    int32_t n_prob;
    int32_t n_pairs;
};

enum : int32_t { ERR_OVERFLOW = 1 };

// Launchers (rewl_kernels.hip).  All enqueue on `st` and return the launch status.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_init(const DevState& S, hipStream_t st);
hipError_t launch_entry(const DevState& S, int64_t cap, hipStream_t st);
hipError_t launch_sweep(const DevState& S, int64_t g_begin, int64_t g_count, int64_t n_trials,
                        int l_max, int wg, hipStream_t st);
hipError_t sweep_setup();
hipError_t launch_flat(const DevState& S, hipStream_t st);
hipError_t launch_stage(const DevState& S, hipStream_t st);
hipError_t launch_exchange(const DevState& S, hipStream_t st);

// Reweighting.
hipError_t launch_lnz_forward(const double* lng, int N, int e0, int nE, int m0, int nM,
                              const double* beta, const double* h, int64_t G, double* lnz,
                              hipStream_t st);
hipError_t launch_lnz_moments(const double* lng, int N, int e0, int nE, int m0, int nM,
                              const double* beta, const double* h, int64_t G, const double* lnz,
                              const double* gout, double* mom, double* gbeta, double* gh,
                              hipStream_t st);
hipError_t launch_lnz_grad_lng(const double* lng, int N, int e0, int nE, int m0, int nM,
                               const double* beta, const double* h, int64_t G, const double* lnz,
                               const double* grad_out, double* grad_lng, hipStream_t st);

}  // namespace rewl
