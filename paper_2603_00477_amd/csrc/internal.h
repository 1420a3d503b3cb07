// Internal declarations of the stencil library (host side and kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/stencil.h"
#include "mfma_layout.h"

namespace stl {

constexpr int kMaxD = 3;
constexpr int kMaxK = 512;  // single-step points handled by the kernels' weight arrays

// Record a message for stencil_last_error() and return `code`.
int fail(int code, const std::string &msg);

// Bytes per stored element of a dtype (bf16x3 stores float32).
int dtype_bytes(int dtype);

// Canonical offsets of the pattern; returns K (or -1).
int pattern_offsets(int shape, int d, int r, std::vector<int> *offs);

// Dense composite kernel of T steps, (2rT+1)^d values indexed by offset+rT.
void compose_dense(int shape, int d, int r, const double *w, int T, std::vector<double> *out);

// Arguments of one pass of one job, as the launchers take them.
struct PassArgs {
    const void *src;
    void *dst;
    int64_t dims[kMaxD];
    int d;
    int region_lo[kMaxD];    // output box [lo, hi) written by this launch
    int region_hi[kMaxD];
    int boundary;
    double halo;
    int steps;               // steps fused in this pass (1..T)
    const double *w;         // K single-step weights, canonical order (host memory)
    const int *offs;         // K x d offsets, canonical order (host memory)
    int K;
    int tile_rows;           // VALU rows per workgroup (0 = auto)
    const void *afrag;       // MFMA operand fragments (device memory)
    const void *afrag_lo;    // compensated mode: lo parts
    int R;                   // MFMA composite radius (r * steps)
    int num_cu;
    int slots_per_cu;        // resident workgroups per CU of the launched kernel (0 = unknown)
};

// Device copies of small host tables (job lists of batched launches).  put()
// copies `bytes` into a pinned host region and enqueues its upload on
// `stream`.  Each begin() .. end() bracket (one batch call) fills one slot of
// a ring; its regions stay valid until the slot comes round again (also when
// the slot had to grow in between), and begin() waits only if the batch that
// last used that slot is still queued.
class BatchStaging {
public:
    hipError_t begin(hipStream_t stream);
    hipError_t put(const void *host, size_t bytes, void **dev, hipStream_t stream);
    hipError_t end(hipStream_t stream);
    ~BatchStaging();

private:
    // A ring of pinned-host / device buffer pairs: one batch call fills one
    // slot, so up to kSlots batches can be queued on the device before a new
    // call has to wait for the oldest to finish with its slot.
    static constexpr int kSlots = 4;
    struct Slot {
        uint8_t *host = nullptr;
        uint8_t *dev = nullptr;
        size_t cap = 0, used = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
        // buffers replaced by grow() during the current batch (host, device)
        std::vector<std::pair<uint8_t *, uint8_t *>> retired;
    };
    hipError_t grow(Slot &s, size_t need);
    Slot slots_[kSlots];
    int cur_ = kSlots - 1;
};

// Stage a batched launch's job table (`job_bytes` bytes) and the tile-start
// prefix of its jobs as one block; *djobs and *dstart receive the device
// addresses of the two parts.
hipError_t stage_job_table(BatchStaging *stage, const void *jobs, size_t job_bytes,
                           const std::vector<int> &start, void **djobs, void **dstart, hipStream_t stream);

// One launchable kernel variant.
struct KernelEntry {
    int path;    // STENCIL_PATH_VALU or one of the MFMA paths
    int dtype;
    int shape;   // -1 = any
    int d;
    int r;       // -1 = any
    int t;       // steps per pass, -1 = any
    hipError_t (*launch)(const PassArgs &, hipStream_t);
    // n passes of this variant (different grids) in one persistent launch; may be null
    hipError_t (*launch_batch)(const PassArgs *, int, BatchStaging *, hipStream_t) = nullptr;
};

// Kernel registries, one per source file; all_kernel_tables() lists them.
const std::vector<KernelEntry> &valu2d_table_f64();
const std::vector<KernelEntry> &valu2d_table_f32();
const std::vector<KernelEntry> &valu2d_table_bf16();
const std::vector<KernelEntry> &valu2d_table_f16();
const std::vector<KernelEntry> &valu2d_table_x3();  // float storage, FP64 arithmetic
const std::vector<KernelEntry> &valu3d_kernels();
const std::vector<KernelEntry> &valu3d_fused_kernels();
const std::vector<KernelEntry> &valu3d_box_kernels();  // boxes r >= 2, one step per pass
const std::vector<KernelEntry> &valu2d_table_cases();  // r = 7, and r = 1 with T = 5..8
const std::vector<KernelEntry> &mfma2d_table_cases();  // composite radius 7
const std::vector<KernelEntry> &mfma3d_table_cases();  // composite radius 7, periodic
const std::vector<KernelEntry> &generic_kernels();
const std::vector<KernelEntry> &mfma2d_table_f64();
const std::vector<KernelEntry> &mfma2d_table_f32();
const std::vector<KernelEntry> &mfma2d_table_bf16();
const std::vector<KernelEntry> &mfma2d_table_f16();
const std::vector<KernelEntry> &mfma2d_table_x3();
const std::vector<KernelEntry> &mfma2d_table_sparse();  // 2:4 structured-sparse instructions
const std::vector<KernelEntry> &mfma2d_table_seq();     // sequential-step fusion
const std::vector<KernelEntry> &mfma3d_table_f64();
const std::vector<KernelEntry> &mfma3d_table_f32();
std::vector<const std::vector<KernelEntry> *> all_kernel_tables();

const KernelEntry *find_kernel(int path, int dtype, int shape, int d, int r, int t);

// MFMA operand fragments for the composite of `steps` steps.
struct MfmaLayout {
    int R;       // composite radius
    int kdim;    // k of the MFMA instruction
    int Kp;      // padded band length (multiple of kdim)
    int nblk;    // Kp / kdim
    double S;    // useful / executed MACs of this layout
};
MfmaLayout mfma_layout(int shape, int d, int r, int steps, int dtype);

// MFMA-family paths (operand fragments on the device).
inline bool is_mfma_path(int path)
{
    return path == STENCIL_PATH_MFMA || path == STENCIL_PATH_MFMA_SPARSE || path == STENCIL_PATH_MFMA_SEQ;
}
// Paths that apply the T-step composite kernel (exact on Dirichlet grids only
// at distance >= r (T - 1) from the boundary: the band is redone by VALU steps).
inline bool is_kernel_fused_path(int path) { return path == STENCIL_PATH_MFMA || path == STENCIL_PATH_MFMA_SPARSE; }

// Operands of the 2:4 sparse layout (d = 2, 16-bit): per column pair, 64
// lanes x 8 compressed weights, then 64 lanes x one int32 of positions.
void mfma_build_sparse_fragments(int shape, int r, const double *w, int steps, int dtype,
                                 std::vector<uint8_t> *out);

// Operands of the 16-bit row layout (d = 2; see mfma_layout.h): per
// non-empty k-block of each composite row, 64 lanes x 8 weights.
void mfma_build_row_fragments(int shape, int r, const double *w, int steps, int dtype,
                              std::vector<uint8_t> *out);
// Whether a dense MFMA pass of t steps uses the row layout: 16-bit operands,
// d = 2, and an operand table that fits LDS (24 fragments; larger composites
// keep the column layout, whose table is read per column).
inline bool mfma_row_layout(int dtype, int d, int shape, int r, int t)
{
    return d == 2 && (dtype == STENCIL_BF16 || dtype == STENCIL_F16) && rows_total_frags(shape, r, t) <= 24;
}

// Build the lane-ordered operand fragments of the composite on the host.
// `hi`/`lo` receive raw element bytes in the MFMA operand type.
void mfma_build_fragments(int shape, int d, int r, const double *w, int steps, int dtype,
                          std::vector<uint8_t> *hi, std::vector<uint8_t> *lo);

int device_cu_count();

// stencil_run with a caller-provided intermediate grid (`scratch`, capacity
// `scratch_cap` bytes): no device memory is allocated.  MFMA plans must
// already hold their operand fragments on the current device.
int run_without_allocation(struct ::stencil_plan_s *p, const void *in, void *out, int64_t steps,
                           hipStream_t stream, void *scratch, size_t scratch_cap);

}  // namespace stl

struct stencil_plan_s {
    int shape, d, r, T, dtype, boundary;
    int path_req;   // requested (may be AUTO)
    int path;       // resolved
    int64_t dims[stl::kMaxD];
    int64_t npts;
    int K;
    std::vector<int> offs;
    std::vector<double> w;      // canonical single-step weights
    double halo;
    int tile_rows;
    // model results
    int K_T;
    double alpha, S, gamma;
    double pred_valu, pred_mfma;
    int pred_winner, scenario;
    // device resources
    int device;
    void *scratch;
    size_t scratch_bytes;
    // MFMA fragments per pass depth (index = steps in pass, 1..T)
    std::vector<void *> afrag;
    std::vector<void *> afrag_lo;
    size_t afrag_bytes;
};
