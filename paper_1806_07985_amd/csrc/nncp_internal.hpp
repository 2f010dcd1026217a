// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "nncp.h"

namespace nncpk {

constexpr int kMaxModes = NNCP_MAX_MODES;
constexpr int kMaxRank = NNCP_MAX_RANK;
// Rank handled by one partial-MTTKRP launch (four 16-wide MFMA column blocks);
// larger ranks are processed in column chunks of this size.
constexpr int kPmMaxCols = 64;
// Dynamic LDS one partial-MTTKRP work-group may request: all of a CU's 160 KiB
// (the kernels declare no static LDS).
constexpr size_t kPmMaxLds = 160 * 1024;

// Khatri-Rao operand description: rows are indexed by a mixed-radix index over
// `nm` modes, the first listed mode fastest; row q of the operand is the
// elementwise product of row d_j(q) of each factor (Section II-A).
//
// The factors are stored unnormalised during the iteration; `lam` (device, N x R,
// row stride lam_ld) holds each mode's column norms and every operand column is
// multiplied by prod_j 1/lam[mode_j][r] (0 where a norm is 0). lam == nullptr
// means the factors are used as they are.
struct KrpDesc {
  const float* f[kMaxModes];   // factor base pointers (column-major, ld = dim)
  int dim[kMaxModes];
  int mode[kMaxModes];
  int nm;
  const double* lam;
  int lam_ld;
};

// The reduction index k of a partial MTTKRP runs over the contracted modes
// (krp.dim[0] fastest); it is split as k = i1 + I1*j with i1 the first contracted
// mode's index and j the index over the remaining contracted modes. The operand
// row is K(k, :) = H_1(i1, :) * Krest(j, :): the kernels keep the H_1 rows of
// their i1 block in LDS and apply Krest(j, :) (times the column scales) as a
// per-output-column factor when the FP32 MFMA partial sums are added into FP64.
struct PmArgs {
  const void* X;
  int64_t IL, IR;        // X viewed as column-major IL x IR
  KrpDesc krp;           // contracted modes (first = fastest)
  int I1, I1pad;         // extent of the first contracted mode, padded to the k-step
  int i1blk, n_i1blk;    // i1 rows per split block, number of i1 blocks
  int64_t J;             // product of the remaining contracted extents
  int jblk, n_jblk;      // j per split block, number of j blocks
  int fold;              // k-steps summed in FP32 before folding into FP64 (divides i1blk/k-step)
  int R;                 // columns handled by this launch (<= kPmMaxCols)
  int col0;              // first column (offset into factor columns)
  void* T;               // output, column-major, ld = Mtot: column c at T + Mtot*c
  int t_f64;             // T is double (else float)
  double* partial;       // split-K partials (FP64)
  const void* zeros;     // >= 64 bytes of zeros in device memory (read by out-of-range lanes)
  unsigned* counters;    // one per M tile; zero on entry, left zero on exit
  int nsplit;            // (n_i1blk / istages) * n_jblk
  int wm;                // waves along M in a work-group (1 or 4); the other 4 / wm split K
  int mtiles;            // M tiles of the output
  int mper;              // M tiles one work-group streams in turn (> 1 only with wm == 4, istages == 1)
  // the number of i1 blocks one work-group walks in turn (restaging LDS between
  // them) instead of splitting K over work-groups
  int istages;
  // 16-bit tensors only: the first contracted factor split into pm16_terms values
  // of the tensor's 16-bit type, scaled per column by a power of two (hscale
  // holds the inverse), laid out [term 0 rows RP][term 1 rows RP]... x I1pad
  unsigned short* hpack;
  float* hscale;
  // Optional: the per-(j, column) Khatri-Rao scales of the whole launch in FP64,
  // sctab[j * RP + r] (RP = 16 * nb), written by a pre-kernel before the partial
  // MTTKRP (the launchers run it); the work-groups then copy their j block
  // instead of each computing it. nullptr: every group computes its own block.
  double* sctab;
};

// 16-bit tensors: the first contracted factor enters the MFMA as a sum of this
// many values of the tensor's type (FP16: hi + lo, 22 bits; BF16: hi + mid + lo,
// 24 bits), so the factor operand is as exact as FP32.
__host__ __device__ constexpr int pm16_terms(int dtype) { return dtype == NNCP_BF16 ? 3 : 2; }

// Plan of one partial-MTTKRP launch (tile shape and split count).
struct PmLaunch {
  int side;      // 0 left (m contiguous), 1 right (k contiguous)
  int dtype;
  int nb;        // 16-wide column blocks
  int mtile;     // output rows per M tile
  int mtiles;
  int mper;      // M tiles per work-group
  int mgroups;   // work-groups along M: ceil(mtiles / mper)
  int nsplit;
  int I1, I1pad, i1blk, n_i1blk, jblk, n_jblk, fold, istages;
  int j1;        // 16-bit right node with J == 1: the specialised kernel (column scale at the end)
  int wm;        // waves along M per work-group (1 or 4)
  int wide;      // FP32 only: the group takes a whole CU's LDS (one i1 block of a long first mode)
  int xs;        // FP32 right node only: X staged through LDS in 256-byte column runs
  int64_t J;
  size_t lds_bytes;
  size_t partial_doubles;
  size_t pack_bytes;     // 16-bit tensors: bytes of the packed factor terms + scales
  int ncounters;
};

// I1 = extent of the first contracted mode (mode s+1 for the left node, mode 1
// for the right node).
// wg_kib: aim for at least this many KiB of X per work-group (<= 0: 256).
PmLaunch pm_plan(int side, int dtype, int64_t IL, int64_t IR, int I1, int R, int wg_kib = 0);
void pm_fill_args(const PmLaunch& L, PmArgs& a);
hipError_t pm_launch(const PmLaunch& L, const PmArgs& a, hipStream_t st);
struct Sink;
struct ReduceArgs;
hipError_t pm_launch(const PmLaunch& L, const PmArgs& a, const Sink& sk);
// per-dtype kernels (pm_kernels.hip, pm16_kernels.hip + pm16_{bf16,f16}{,_mt}.hip)
int pm_f32_wave_rows(int side, int nb, bool xs = false);
int pm_f32_kstep(int side, bool xs = false);
// LDS of the four waves' staging tiles of the xs form
size_t pm_f32_xs_tile_lds(int nb);
// doubles of the scale table of a launch plan (J x 16 nb), and the pre-kernel
// that writes it (a.sctab, a.krp, a.R, a.col0)
size_t pm_sctab_doubles(const PmLaunch& L);
hipError_t pm_scale_table_launch(const PmLaunch& L, const PmArgs& a, hipStream_t st);
// the same pre-kernel recorded into a batch (slot 0, before the partial MTTKRP)
hipError_t pm_scale_table_record(const PmLaunch& L, const PmArgs& a, const Sink& sk);
const void* pm_sctab_batch_kernel();
bool pm_f32_xs_ok(int64_t Ktot, int nb);
size_t pm_f32_reduce_lds(int side, int nb, int wm);
hipError_t pm_launch_f32(const PmLaunch& L, const PmArgs& a, const Sink& sk);
int pm_16_wave_rows(int side, int nb, int j1 = 0);
int pm_16_kstep(int side);
size_t pm_16_reduce_lds(int side, int nb, int wm);
hipError_t pm_launch_16(const PmLaunch& L, const PmArgs& a, const Sink& sk);
template <int DT, bool MT>
const void* pm16_kernel_form(int side, int nb, int j1, int fast, bool batch);
// Every vector load of every k-step lies inside the tensor for this shape (no
// padded i1, and on the left side no row group straddling a column end): the
// kernels then skip the per-step check.
bool pm_f32_fast(int side, int64_t IL, int I1, int nb, bool xs = false);
bool pm16_fast(int side, int64_t IL, int I1, int nb);
template <int DT>
const void* pm16_pack_kernel(bool batch);
// Batched (work-list) forms of the partial-MTTKRP kernels, by recorded variant.
const void* pm_f32_batch_kernel(int variant);
const void* pm16_batch_kernel(int variant);
const void* pm16_pack_batch_kernel(int variant);
// Largest dynamic LDS any launch of this partial-MTTKRP variant uses.
size_t pm_variant_max_lds(int kind, int variant);
// Lets kernel k use `bytes` of dynamic LDS (once per kernel; thread safe).
void pm_allow_lds(const void* k, size_t bytes);

// Multi-TTV kernels ---------------------------------------------------------
struct MttvArgs {
  const void* T;        // node temporary: I_a x J x R (column-major)
  int t_f64;            // T is double (else float)
  int64_t Ia, J;
  int R;
  KrpDesc krp;          // trail: the contracted last modes; lead: the contracted first modes (first fastest)
  void* out;
  int out_f64;          // out is double (else float)
};
hipError_t mttv_trail_launch(const MttvArgs& a, hipStream_t st);
hipError_t mttv_lead_launch(const MttvArgs& a, hipStream_t st);
hipError_t mttv_trail_launch(const MttvArgs& a, const Sink& sk);
hipError_t mttv_lead_launch(const MttvArgs& a, const Sink& sk);

// Factor update, Gram, lambda, fit -----------------------------------------
struct UpdateArgs {
  const void* M;          // I x R MTTKRP result (others normalised)
  int m_f64;              // M is double (else float)
  float* W;               // in: stored factor of this mode (scaled by lam_self), out: new W_hat
  int64_t I;
  int R;
  const double* S;        // R x R (device)
  const double* lam_model;  // current model weights
  const double* lam_self;   // column norms of W as stored
  int update;             // NNCP_HALS / NNCP_MU
  int sweeps;             // update sweeps (>= 1; 0 is taken as 1): at most this many
  double tol;             // > 0: a row stops once a sweep changes none of its entries by more
                          // than tol x the row's largest entry
  double* W64;            // optional: the new W_hat also in FP64 (I x R, column-major)
};
hipError_t update_launch(const UpdateArgs& a, hipStream_t st);
hipError_t update_launch(const UpdateArgs& a, const Sink& sk);

struct FinalizeArgs {
  const float* W;         // I x R new factor (unnormalised)
  const void* M;          // I x R (for beta) or nullptr
  int m_f64;
  int64_t I;
  int R;
  int N, mode;
  double* G;              // N x R x R: normalised Grams (this mode written)
  double* lam;            // N x R: per-mode column norms (this mode written)
  double* lam_model;      // R (written when set_model)
  double* S;              // N x R x R: S^(next) written for next_mode >= 0
  int next_mode;
  int set_model;
  // fit
  int do_fit;
  const double* alpha;
  double* fit_out;        // indexed by *iter_counter
  int* iter_counter;
  int fit_capacity;
  // scratch
  double* gram_raw;       // optional: W^T W (unnormalised) written here
  double* partial;        // nchunks x (R*R + 1)
  int nchunks;
  int rows_per_chunk;
};
int finalize_chunks(int64_t I, int R, int* rows_per_chunk);
hipError_t finalize_launch(const FinalizeArgs& a, hipStream_t st);
hipError_t finalize_launch(const FinalizeArgs& a, const Sink& sk);

hipError_t pm_reduce_launch(const ReduceArgs& r, const Sink& sk);

// lam_model = lam_in * prod_k lam[k]; S[0] = prod_{k != 0} G[k]
hipError_t init_model_launch(const double* lam_in, double* lam, double* lam_model, const double* G,
                             double* S, int N, int R, hipStream_t st);
// H[k] <- H[k] / lam[k] for all columns; lam[k] <- (lam>0 ? 1 : 0); lam_out_dev <- lam_model
hipError_t normalize_out_launch(float* W, int64_t I, int R, double* lam_self, hipStream_t st);

// ||X||^2 in FP64: norm_sq_blocks(n) <= kNormSqMaxBlocks groups, each writing one
// FP64 partial; counter must be zero on entry (the last group resets it).
constexpr int kNormSqMaxBlocks = 1024;
hipError_t norm_sq_launch(const void* X, int dtype, int64_t n, double* out, double* partial,
                          unsigned* counter, int nblocks, hipStream_t st);
int norm_sq_blocks(int64_t n);
hipError_t quantize_launch(const float* src, void* dst, int dtype, int64_t n, hipStream_t st);
hipError_t fill_u32_launch(unsigned* p, int64_t n, unsigned v, hipStream_t st);
hipError_t fill_f64_launch(double* p, int64_t n, double v, hipStream_t st);
hipError_t copy_f64_launch(double* dst, const double* src, int64_t n, hipStream_t st);
hipError_t widen_f32_launch(double* dst, const float* src, int64_t n, hipStream_t st);
// lam[k] <- (lam[k] > 0 ? 1 : 0), n entries (after normalize_out)
hipError_t unit_lambda_launch(double* lam, int64_t n, hipStream_t st);

// ---------------------------------------------------------------------------
// Launch records. Every kernel launch of the iteration goes through a Sink: it
// is either launched on the sink's stream at once, or appended to the sink's
// record as data (kernel kind + template variant + stand-alone grid + args).
// The batched executor records one outer iteration per job and replays the
// records of many jobs through persistent work-list kernels, one launch per
// step and kernel family, so each job's arithmetic (tiling, split order) is
// exactly that of its stand-alone launches.
// ---------------------------------------------------------------------------
struct ReduceArgs {      // split-K sum of partial-MTTKRP partials
  const double* part;
  void* T;
  int t_f64;
  int64_t Mtot, Mpad;
  int RP, R, col0, nsplit;
};
struct PackArgs {        // term pack of the first contracted factor (16-bit tensors)
  const float* H1;
  int I1, I1pad, R, col0, RP;
  unsigned short* pack;
  float* hscale;
};

enum KKind : int {
  K_PM_F32 = 1,     // variant: xs*100000 + wide*10000 + side*1000 + nb*100 + mt*10 + fast
  K_PM_16 = 2,      // variant: j1*100000 + (dtype == BF16)*10000 + side*1000 + nb*100 + mt*10 + fast
  K_PACK16 = 3,     // variant: dtype == BF16
  K_PM_REDUCE = 4,  // variant: t_f64
  K_MTTV_TRAIL = 5, // variant: t_f64
  K_MTTV_LEAD = 6,  // variant: group size * 10 + t_f64
  K_UPDATE = 7,     // variant: R > 64: values per lane (1, 2); R <= 64: register columns (16, 32, 64)
  K_FIN_FUSED = 9,  // R > 64: one row chunk
  K_GRAM_CHUNKS = 10,
  K_FIN_TAIL = 11,
  K_FIN1K = 12,     // R <= 64, one row chunk, 1024 threads; variant: R x R entries per thread
  K_GRAM1K = 13,    // R <= 64, one row chunk's Gram partial, 1024 threads; variant as K_FIN1K
  K_TAIL1K = 14,    // R <= 64, sum of the chunk partials and the finish, 1024 threads
  K_SCTAB = 15      // a partial MTTKRP's scale table (u.pm); variant: 16 * column blocks
};
struct KOp {
  int kind;
  int variant;
  int stage;         // batching order: 64 * mode + 4 * step + slot (see kslot)
  unsigned gx, gy;   // work-groups of the stand-alone launch (x, y)
  unsigned lds;      // dynamic LDS bytes
  unsigned coarse;   // batched small ops: stand-alone work-groups (along x) one batch item runs in turn
  union {
    PmArgs pm;
    MttvArgs mt;
    UpdateArgs up;
    FinalizeArgs fin;
    ReduceArgs red;
    PackArgs pk;
  } u;
};

// One work-group's share of a recorded launch: op index and its (x, y) tile
// (for a small op, x counts runs of `coarse` stand-alone work-groups).
struct BItem {
  int op;
  int bx, by;
};

struct Sink {
  hipStream_t st = nullptr;
  void* rec = nullptr;  // std::vector<KOp>* when recording
  int mode = 0;         // mode whose steps are being recorded
  int step = 0;         // position of the recorded op in the mode's sequence (see kslot)
  Sink() = default;
  Sink(hipStream_t s) : st(s) {}  // launch on s (implicit: a stream is a launching sink)
};
// Batching order of a recorded op: stage = 64 * mode + 4 * step + kslot(kind).
// The driver numbers a mode's tree ops 0, 1, ... (a partial MTTKRP is its pack
// (slot 0), the kernel (slot 1) and its split-K reduction (slot 2); a
// multi-TTV is slot 1), the update is step kStepUpdate and the Gram/finalize
// step kStepFinal (chunk partials slot 0, the finish slot 1).
constexpr int kStepUpdate = 13, kStepFinal = 14;
inline int kslot(int kind) {
  switch (kind) {
    case K_PACK16: case K_SCTAB: return 0;
    case K_PM_F32: case K_PM_16: case K_MTTV_LEAD: case K_MTTV_TRAIL: case K_UPDATE: return 1;
    case K_PM_REDUCE: return 2;
    case K_GRAM_CHUNKS: case K_GRAM1K: return 0;
    default: return 1;
  }
}
// Append a record (host), stamping its stage; returns hipSuccess.
hipError_t sink_record(const Sink& s, const KOp& op);

// Persistent batched kernels: each has the signature
//   (const BItem* items, const int* grp, const KOp* ops)
// and its work-group b walks items grp[0] + b, grp[0] + b + gridDim.x, ...
// below grp[0] + grp[1] (device arrays), each naming an op in `ops`. Partial
// MTTKRPs have one such kernel per recorded variant (the stand-alone kernel's
// body in a loop); the other kinds share a kernel per family (a switch over
// the kind): the 256-thread small kernels and the 1024-thread Gram/finalize.
struct BatchKernel {
  const void* fn = nullptr;
  int threads = 0;    // block size
  size_t lds = 0;     // dynamic LDS the kernel is launched with (the most any of its ops uses)
  int per_cu = 1;     // work-groups kept resident per CU (the persistent grid is per_cu x CUs)
};
// Ops of equal id run in the same launch of one stage.
int batch_kernel_id(int kind, int variant);
BatchKernel batch_kernel_for(int kind, int variant);
// Batched form of a small op's kernel (nullptr for a kind without one).
const void* small_batch_kernel_ptr(int kind, int variant);
const void* fin_batch_kernel_ptr();
size_t fin_batch_max_lds();

// Column scale of a Khatri-Rao operand, prod_j 1/lam[mode_j][r] (device code).
__device__ __forceinline__ double krp_colscale(const KrpDesc& k, int r) {
  double s = 1.0;
  if (k.lam) {
    for (int j = 0; j < k.nm; ++j) {
      double l = k.lam[(int64_t)k.mode[j] * k.lam_ld + r];
      s = (l > 0.0) ? s / l : 0.0;
    }
  }
  return s;
}

// Process-wide record of the most recent failed HIP runtime call (any thread):
// its hipError_t and a source location (line in the driver; 200000 + line in
// the serving loop). Read back through nncp_last_device_error.
void note_device_error(int hip_error, int where);
uint64_t last_device_error();

}  // namespace nncpk
