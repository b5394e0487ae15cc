// Internal declarations shared by the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gtls.h"

namespace gtls {

// Per-(period, duration) best window, written by the slide kernel and read
// by the per-period reduction.
// Items with every T0 offset are split into tiles of windows, one slot per
// tile; strided items fill slot 0 only.  Slot 0 records how many are used.
struct ItemBest {
    double dchi2;    // best chi2 improvement; -inf when the duration is invalid
    double depth;    // depth at that window
    int32_t start;   // window start in phase order, -1 when invalid
    int32_t d;       // points in the duration
    int32_t evals;   // windows evaluated by this slot
    int32_t ntiles;  // (slot 0) number of slots holding results
};

struct SearchArgs {
    // device inputs
    const double* t;
    const double* y;
    const double* dy;
    int64_t n;
    const double* periods;
    int32_t n_periods;
    const double* durations;
    int32_t n_durations;
    const double* tmpl;
    int32_t n_tmpl;
    gtls_params prm;
    // device outputs
    double* chi2;
    int32_t* best_dur;
    int32_t* best_start;
    double* depth;
    double* t0;
    double* sr;
    double* sde_raw;
    double* sde;
    gtls_summary* summary;
    // Allocation-free calls: every scratch region is carved from this
    // device buffer of fixed_bytes instead of the context's own buffers.
    char* fixed = nullptr;
    size_t fixed_bytes = 0;
};

struct DeviceBuffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Batched survey: host CSR offsets, device data and outputs.
struct BatchArgsHost {
    const int64_t* offsets;        // host [nc + 1]
    const int64_t* poffsets;       // host [nc + 1]
    int32_t nc;
    const double* t;               // device
    const double* y;
    const double* dy;
    const double* periods;
    const double* durations;
    int32_t nd;
    const double* tmpl;
    int32_t nt;
    gtls_params prm;
    double* chi2;                  // device outputs (CSR over periods)
    int32_t* best_dur;
    int32_t* best_start;
    double* depth;
    double* t0;
    double* sr;
    double* sde_raw;
    double* sde;
    gtls_summary* summaries;       // device [nc]
};

// Cached executable graph of the batched pipeline and autotuned grid sizes.
struct BatchCache {
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
    std::vector<std::pair<std::vector<uint64_t>, int>> tuned;   // shape key -> workgroups per CU
};

}  // namespace gtls

struct gtls_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    // grow-only device scratch
    gtls::DeviceBuffer curve;    // per-point arrays and scalars
    gtls::DeviceBuffer batch;    // per-period-batch arrays
    gtls::DeviceBuffer io;       // device copies for host-pointer calls
    gtls::DeviceBuffer sde_tmp;  // SDE scratch
    gtls::DeviceBuffer table;    // template rows per point count D and per-D sums
    gtls::DeviceBuffer bcurve;   // batched: per-point arrays, per-curve scalars, queue
    gtls::DeviceBuffer bscratch; // batched: per-workgroup sort/padding scratch
    gtls::BatchCache bcache;
    int num_cus = 0;
    // Device address of the library's static scratch array on this context's
    // device (resolved once per device at context creation).
    char* static_scratch = nullptr;
    // per-stage timing (gtls_profile_enable / gtls_profile_read)
    bool profiling = false;
    double prof_ms[8] = {0};
    int64_t prof_launches[8] = {0};
    struct Pending {
        int stage;
        hipEvent_t start, stop;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
};

namespace gtls {

// Launchers (kernels.hip).  Return hipSuccess or the first HIP error.
hipError_t run_search(gtls_ctx* ctx, const SearchArgs& a);
hipError_t run_fold_sort(gtls_ctx* ctx, const double* t_dev, int64_t n, const double* periods_dev,
                         int32_t n_periods, int32_t* perm_dev);
hipError_t run_transit_stats(gtls_ctx* ctx, const double* t, const double* y, const double* dy, int64_t n,
                             const double* period_dev, int64_t d, int64_t start, const double* tm, int32_t nt,
                             int64_t nep_max, int64_t max_transits, gtls_transit_stats* st_dev, int64_t* epoch,
                             double* t_mid, double* depth, double* sigma, int64_t* count);
hipError_t run_sde(gtls_ctx* ctx, const double* chi2_dev, int32_t n, int32_t window, double* sr_dev,
                   double* raw_dev, double* sde_dev, gtls_summary* summary_dev);
hipError_t ensure(gtls_ctx* ctx, DeviceBuffer& b, size_t bytes);
hipError_t run_search_batch(gtls_ctx* ctx, const BatchArgsHost& a);
// Address of the static scratch array on `device` (which must be current),
// resolved with hipGetSymbolAddress on the first call for that device.
hipError_t static_scratch_address(int device, char** ptr);
extern const size_t kStaticScratchBytes;
hipError_t profile_collect(gtls_ctx* ctx);

enum Stage { kStagePrep = 0, kStageSort = 1, kStageSlide = 2, kStageReduce = 3, kStageSde = 4, kStageStrided = 5 };

// Brackets one kernel launch with events on the context's stream when
// profiling is on.
class StageTimer {
  public:
    StageTimer(gtls_ctx* ctx, int stage);
    ~StageTimer();

  private:
    gtls_ctx* ctx_;
    int stage_;
    hipEvent_t stop_ = nullptr, start_ = nullptr;
};

}  // namespace gtls
