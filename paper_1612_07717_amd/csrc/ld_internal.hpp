// ld_internal.hpp -- structures shared by the host runtime and the kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/ldmlmc.h"

namespace ldm {

enum { KINTEG_SE = 0, KINTEG_GL = 1, KINTEG_BAOAB = 2,
       KINTEG_SE_ADAPT = 3,       // kernel variants: symplectic Euler with adaptive steps (Sec. 7),
       KINTEG_SE_ADAPT_WIDE = 4 };  // 32-bit tick counters, or 64-bit where T in ticks needs them
enum { KPROFILE_HOMOGENEOUS = 0, KPROFILE_NEUTRAL = 1 };
enum { KRELEASE_FIXED_W = 0, KRELEASE_GAUSSIAN_W = 1, KRELEASE_WELL_MIXED = 2 };
enum { KQOI_MEAN_Z = 0, KQOI_P_ABOVE = 1, KQOI_P_BOX = 2, KQOI_VELOCITY = 3, KQOI_VELOCITY_SQ = 4 };

constexpr int kFoldMax = 16;      // reflections allowed in one fold before a path is declared runaway
constexpr int kAdaptTickBits = 20;    // adaptive steps: ticks of h_l / 2^20
constexpr int kBlock = 256;       // threads per block of the level kernel (4 wave64)
constexpr int kMaxItems = 40;     // (level, range) items per launch
constexpr int kMaxCoef = 10;      // smoothing polynomial p_r, r <= 8

// Block modes. STREAM: each lane runs whole coupled samples (throughput). PIPE: a block
// serves 64 samples with its four waves specialised - two draw normals, one advances
// the fine paths, one the coarse paths - handing data through LDS, so the per-sample
// instruction stream of the critical (fine) wave is short (latency of long paths).
enum { KMODE_STREAM = 0, KMODE_PIPE = 1 };
constexpr int kPipeChunk = 8;                     // coarse steps per LDS hand-off (FP64; FP32 twice that)
constexpr uint64_t kPipeMaxSamples = 64u * 2048u; // larger ranges fill the GPU in STREAM mode
constexpr uint32_t kPipeMinSteps = 256;           // shorter paths are not latency-critical

// Problem parameters in FP64, prepared on the host (kernel argument).
struct KProblem {
    double H, eps_reg, ks, kappa_tau, sigma_u, tau, T;
    double z0, w0, su_z0;          // release; su_z0 = regularised sigma_U(z0)
    double lam_max;                // max of lambda = 1/tau over [0, H]
    double ksH, kl;                // kappa_sigma u_* H^(-3/4) and ksH / kappa_tau
    double x_adapt;                // adaptive symplectic Euler: reference height (0: uniform)
    double qa, qb, inv_delta;
    double coef[kMaxCoef];
    int32_t integ, profile, release, qoi_kind, r, ncoef, M0, adaptive;
    uint32_t stream_id;
    uint64_t seed;
};

// One (level, sample range) of a launch. Blocks [block_begin, block_begin + n_blocks)
// cover it; each lane of a block handles `spl` samples.
struct KItem {
    int32_t level;
    uint32_t spl;           // samples per lane (STREAM mode)
    uint32_t block_begin;
    uint32_t n_blocks;
    uint64_t sample_begin;
    uint64_t n_samples;
    uint32_t out_slot;
    uint16_t mode;          // KMODE_*
    uint16_t prio;          // wave priority 0..3 (longest paths highest)
};

struct KArgs {
    KProblem prob;
    int32_t n_items;
    int32_t precision;
    KItem items[kMaxItems];
};

// Host-side launch of the level kernels (kernels.hip). partials must hold
// total_blocks ld_level_sums; out holds one per item (indexed by out_slot).
int launch_levels(const KArgs& args, uint32_t total_blocks, ld_level_sums* d_partials,
                  ld_level_sums* d_out, double* d_dump, void* stream);

// Block partials of the allocation-free level sums: a device array the library owns,
// one per device for the life of the process. No launch plan of one (level, range) uses
// more blocks than this (STREAM ranges are cut into at most 32768 blocks, PIPE ranges
// into at most 2048, adaptive ones into at most 1280).
constexpr uint32_t kScratchPartials = 32768;
// Device address of that array on the current device (looked up once per device).
// LD_ENODEVICE without a device, LD_EDEVICE if the runtime refuses the lookup.
int scratch_partials(ld_level_sums** out);

// ---- multi-estimator engine ------------------------------------------------------
// A tile is one block's work: block `local_block` of the range (slot, level,
// sample_begin, n_samples) in the given mode.
struct KTile {
    uint32_t slot;          // query slot: index into the problem table and running sums
    int32_t level;
    uint64_t sample_begin;  // first sample of the range
    uint64_t n_samples;     // samples in the range
    uint32_t local_block;
    uint32_t spl;
    uint16_t mode;
    uint16_t prio;
    uint32_t pad;
};

struct KQueue {
    uint32_t first;         // first tile of this queue in the tile table
    uint32_t n_tiles;
    uint32_t counter;       // index of its counter in the counter array
    uint32_t pad;
};

// Tile queues of an engine iteration: one per profile kind, and one for adaptive
// symplectic Euler (neutral profile), whose tiles run in a kernel of their own.
enum { KQUEUE_ADAPT = 2, kNumQueues = 3 };

struct KHeader {
    KQueue queue[kNumQueues];   // [KPROFILE_*], [KQUEUE_ADAPT]
    uint32_t n_ranges;
    uint32_t pad[3];
};

// A range of an engine iteration: samples [sample_begin, sample_begin + n_samples) of
// (slot, level), cut into n_tiles tiles of one mode (spl samples per lane in STREAM
// tiles) at tiles [tile_begin, tile_begin + n_tiles) of the tile table, whose partials
// are contiguous alike; the device writes the tiles from the range. fresh: the first
// range of this (slot, level) since the slot was taken, so its running sums start from
// zero (whatever an earlier query left there).
struct KRange {
    uint32_t slot;
    int32_t level;
    uint32_t tile_begin;
    uint32_t n_tiles;
    uint64_t sample_begin;
    uint64_t n_samples;
    uint32_t spl;
    uint16_t mode;
    uint16_t prio;
    uint32_t fresh;
    uint32_t pad;
};

constexpr int kMergeGrid = 256;   // blocks of the range-merge kernel (grid-stride)

// A small iteration's tables as one kernel argument (under 4 KB): the header, the ranges
// and the problems of newly admitted queries (slots new_lo .. new_lo + n_new - 1). The
// expand kernel stores them where the larger iterations' uploads go, so no copy is queued.
constexpr int kInlineRanges = 24;
constexpr int kInlineProblems = 4;
struct KInline {
    KHeader hdr;
    uint32_t new_lo, n_new, pad[2];
    KRange ranges[kInlineRanges];
    KProblem problems[kInlineProblems];
};
static_assert(sizeof(KInline) <= 3584, "an inline iteration must fit the kernel argument space");

// Enqueues one engine iteration: the tile table written from the ranges, then for each
// queue whose bit (1 << KPROFILE_*,
// 1 << KQUEUE_ADAPT) is set in queue_mask, its tiles in grid_blocks[queue] blocks, either
// persistent ones that take tiles from the queue's counter (a fixed grid, for captured
// graphs) or one block per tile (grid_blocks[queue] = its tile count); then the range
// merge into the running sums, which also sets the queue counters back to zero (they
// must be zero when an iteration starts). inl (not NULL): the tables come as the expand
// kernel's argument and it stores the header, ranges and new problems first.
int launch_engine_iteration(int precision, bool persistent, const uint32_t* grid_blocks, uint32_t queue_mask,
                            const KHeader* d_hdr, const KTile* d_tiles, const KProblem* d_problems,
                            ld_level_sums* d_partials, uint32_t* d_counters,
                            const KRange* d_ranges, ld_level_sums* d_running,
                            ld_level_sums* d_range_out, ld_level_sums* h_running, void* stream,
                            const KInline* inl = nullptr);
// Binned concentration: bins [a0 + i width, a0 + (i+1) width], i < n_bins (<= 64),
// over a dump of n (X_f, X_c) pairs of `level`.
struct KBins {
    double a0, width;
    int32_t n_bins, level;
    uint64_t n;
};
constexpr uint32_t kPdfChunk = 2048;                // dumped samples per bins block
constexpr int kMaxBins = 64;
inline uint32_t pdf_blocks(uint64_t n) { return (uint32_t)((n + kPdfChunk - 1) / kPdfChunk); }
// pdf_bins_kernel over the dump, then the per-bin merge into d_out[0 .. n_bins).
// d_partials holds pdf_blocks(n) * n_bins sums. kp: the problem with the box QoI (r,
// delta, smoothing coefficients).
int launch_pdf_bins(const KBins& bins, const KProblem& kp, const double* d_dump,
                    ld_level_sums* d_partials, ld_level_sums* d_out, void* stream);

int launch_clear_sums(ld_level_sums* d_sums, uint32_t n, void* stream);
// Sets the engine's queue counters to zero (once, when the engine is made).
int launch_reset_counters(uint32_t* d_counters, void* stream);

}  // namespace ldm
