// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sng_device.hpp"

namespace sng {

// Launch shape of the sampled-distance pass (resolved from sng_config).
struct PassAShape {
    int lanes;            // lanes per pair (G)
    int chunks_per_wave;  // 64-call chunks per wavefront
    int stage_lds;        // source row staged in LDS
    int waves_per_block;
    int owners_per_batch; // Philox calls of a group whose partners are fetched together
};

// Fills the binary32 band [lo, hi] around eps2 for dimension d.
void band_fp32(double eps2, int d, float *lo, float *hi, double *rel);

// Extra inputs of the mixed-precision pass.
struct LowpArgs {
    const uint16_t *Xlp;   // 16-bit copy, row stride ld_lp (multiple of 8), 16-byte aligned
    int64_t ld_lp;
    float scale;           // X ~= scale * X_lp
    double scale2;         // scale^2
    double *stats;         // [n][4]: ||v||^2, ||v||, r, pad (rounded up)
    uint64_t *queue;       // undecided slots i*m + t
    uint64_t qcap;
    double eps2_lo, eps2_hi;  // S <= eps2_lo forces acceptance, S > eps2_hi rejection
    double gamma_acc;      // relative error of the FP32 MFMA accumulation
    double gamma_norm;     // relative error of the binary64 norms and their combination
    double tiny;           // absolute slack for flushed subnormals
};

// waves: wavefronts per block of the MFMA pass (0: as many of 4, 2, 1 as
// the LDS allows); ksteps: 32-wide K-steps of partner fragments loaded
// together (0: 8). Shapes whose LDS does not fit return hipErrorInvalidValue.
hipError_t launch_lowp(const Inst &I, const LowpArgs &L, int prec, hipStream_t st,
                       int waves = 0, int ksteps = 0);

// Sweep over a grid of eps (ascending) and MinPts values. The per-level
// thresholds travel by value in the kernel arguments.
constexpr int kSweepMaxK = 64;
constexpr int kSweepMaxP = 16;
struct SweepConst {
    float lo[kSweepMaxK];   // binary32 band of each eps_k^2
    float hi[kSweepMaxK];
    double e2[kSweepMaxK];  // fl64(eps_k^2)
    int32_t min_pts[kSweepMaxP];
};
struct SweepArgs {
    SweepConst c;
    int K, P;
    uint32_t *hist;      // [n][K] accepted slots per point and level
    uint32_t *codes;     // per Philox call: four level codes (K = none)
    uint8_t *kc;         // [P][n] first core level (K = never)
    int32_t *link;       // [P][n] level links set aside between two levels
    int32_t *labels;     // [P][K][n]
    uint32_t *degrees;   // [K][n] or null
};

hipError_t launch_sweep(const Inst &I, const SweepArgs &S, const PassAShape &sh,
                        const struct BucketGeom *B, hipStream_t st);

// Geometry of a batch (device tables are exclusive prefixes, count+1 long).
constexpr uint32_t kPointsPerBlock = 2048;  // points of one instance per block
constexpr uint32_t kWordsPerBlock = 4096;   // accept words of one instance per block
struct BatchGeom {
    int count;
    const uint64_t *pblk;          // point blocks per instance (at least one each)
    const uint64_t *wblk;          // accept-word blocks per instance
    const uint64_t *chunk_starts;  // 64-call chunks per instance
    uint64_t total_pblocks, total_wblocks, total_chunks;
};

hipError_t launch_batch(const Inst *T, const BatchGeom &G, int d, bool vec_ok,
                        const PassAShape &sh, hipStream_t st);

// L2-reuse schedule of the sampled-distance pass (sng_bucket.hip).
constexpr int kXcds = 8;                    // workgroup b runs on XCD b mod 8
constexpr uint64_t kRangeCalls = 8192;      // Philox calls per generator range (one workgroup)
constexpr uint32_t kMaxPartnerBlocks = 1024;
// Rows of at most kLdsMaxD floats get partner blocks of at most
// kLdsBlockBytes, which the evaluate kernel stages in LDS whole.
constexpr int kLdsMaxD = 8;
constexpr uint32_t kLdsBlockBytes = 128u << 10;
struct BucketGeom {
    uint32_t bshift;     // partner block = 2^bshift rows
    uint32_t NJ;         // partner blocks
    uint32_t lds;        // 1: blocks sized for LDS (rows of at most kLdsMaxD floats); records
                         // then hold [partner offset: bshift bits][word: 2][call within
                         // the point: tc_bits][source offset within the range: the rest]
    uint32_t tc_bits;    // LDS records: bits of the call-within-point field
    uint64_t ranges;     // generator ranges
    uint64_t region;     // records per generator range (capacity)
    uint32_t *rec;       // [ranges][region] 4-byte slot records
    uint32_t *seg;       // [ranges][NJ][2] segment offset and count
    uint32_t *start;     // [ranges][2] source and call of each range's first call
    unsigned long long *queue;  // [kXcds] next ticket of each XCD's queue
    unsigned long long *hdr;    // [2] tag of the sample held in rec, and its self-pair count
    uint64_t tag;               // tag of the sample these arguments describe (never 0)
    DivMagic cdiv;              // division by ceil(m/4), the calls per point
    uint32_t x_bytes;           // bytes of X addressed through the buffer descriptor
};
// u64 index of BucketGeom::hdr inside an instance's counter header
constexpr int kSampleHdr = 32;
// u64 index of the simple-graph table's chosen log2 size in the header
constexpr int kSimpleHdr = 40;
// Workspace layouts whose record areas differ: a sample is valid only for
// the layout that drew it.
constexpr uint32_t kLayoutPlain = 1;
constexpr uint32_t kLayoutSweep = 2;
constexpr uint32_t kLayoutSimilarity = 3;
constexpr uint32_t kLayoutSimpleTable = 0x10;  // or-ed in: a simple-graph table precedes the records
uint64_t sample_tag(int64_t n, int64_t m, uint64_t seed, uint32_t bshift, uint32_t layout);
bool bucket_geometry(int64_t n, int d, int64_t m, bool force, BucketGeom *g);
size_t bucket_bytes(const BucketGeom &g);
// Draws and sorts the sample into B (B.hdr gets its tag once complete).
hipError_t launch_bucket_generate(const Inst &I, const BucketGeom &B, hipStream_t st);
// Evaluates the sample held in B, drawing it first unless `reuse`.
hipError_t launch_bucket_plain(const Inst &I, const BucketGeom &B, const PassAShape &sh,
                               bool reuse, hipStream_t st);
hipError_t launch_bucket_sweep(const Inst &I, const SweepArgs &S, const BucketGeom &B,
                               const PassAShape &sh, hipStream_t st);

// Resolves the launch shape for an instance (d, row alignment, user config).
PassAShape resolve_shape(int d, bool vec_ok, int lanes_req, int cpw_req, int lds_req,
                         int prefetch_req);

// Sampled-distance pass over `chunks` 64-call chunks of one instance.
hipError_t launch_pass_a(const Inst &I, const PassAShape &sh, hipStream_t st);

// Sampled-distance pass over every instance of a batch table (device).
hipError_t launch_pass_a_batch(const Inst *table, int count, const uint64_t *chunk_starts,
                               uint64_t total_chunks, int d, bool vec_ok, const PassAShape &sh,
                               hipStream_t st);

// Similarity queries: set_similarity fills I.sim (and for the cosine the
// band and the row pointer of the unit copy) for kind (kSimDot, kSimCos) and
// tau; launch_similarity_rows then writes the unit copy [n][unit_copy_ld(d)]
// that the cosine's pass reads (carved by the caller; nothing for the dot
// product).
int64_t unit_copy_ld(int32_t d);
void set_similarity(Inst &I, int32_t kind, double tau, float *unit);
hipError_t launch_similarity_rows(const Inst &I, float *unit, hipStream_t st);

// Simple-graph degrees (distinct accepted neighbours) from the accept bits
// of the pass: table has 2^max_log2 u64 entries (simple_table_log2), the
// size used is chosen on the device and kept in *log2_word.
uint32_t simple_table_log2(int64_t n, int64_t m);
hipError_t launch_simple_degrees(const Inst &I, unsigned long long *table, uint32_t max_log2,
                                 uint32_t *log2_word, hipStream_t st);

// Post-processing kernels (core mask, hooks, finalize).
hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t v, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t count, unsigned long long v,
                           hipStream_t st);
hipError_t launch_core_init(const Inst &I, hipStream_t st);
hipError_t launch_compact(const int32_t *labels, uint32_t n, int32_t *out, int32_t *n_clusters,
                          hipStream_t st);
// blocks: the grid of the hook launch (0: the default).
hipError_t launch_hook_mask(const Inst &I, hipStream_t st, unsigned blocks = 0);
hipError_t launch_finalize(const Inst &I, hipStream_t st);
hipError_t launch_edge_degrees(const int32_t *edges, int64_t n_edges, uint32_t *deg,
                               hipStream_t st);
hipError_t launch_hook_edges(const Inst &I, const int32_t *edges, int64_t n_edges,
                             hipStream_t st);

}  // namespace sng
