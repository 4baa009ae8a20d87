// Internal declarations shared by the library's translation units.
// gfx950 only: wave64, MFMA, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct nnp_model;
struct nnp_nlist;

namespace nnp {

// Sets the calling thread's error message (nnp_last_error) and returns code.
int fail(int code, const char *fmt, ...);

// Model internals used by the serving layer.
size_t model_workspace_bytes(nnp_model *m, int64_t max_atoms, int max_systems, bool pooled);
int model_reserve_pooled(nnp_model *m, int64_t max_atoms, int max_systems);
const int *model_status_word(const nnp_model *m);
int model_device(const nnp_model *m);
int model_precision(const nnp_model *m);
int model_species(const nnp_model *m);
// Per-slot neighbour counts of a pool (kept past the capacity on overflow).
const int *nlist_counts(const nnp_nlist *nl);

struct CallSizes;
// Graph replay of calls on persistent lists (serving).  A call's launches
// are recorded once per capacity bucket (its atom and system counts rounded
// up to the bucket, which sizes every grid) into a HIP graph together with
// the caller's own kernels before and after them, and replayed for every
// later call in the bucket: the kernels read the call's own sizes from its
// descriptors (uploaded before the replay).  pre/post get the launch sizes
// and the device address of the live sizes (null when launched directly).
struct GraphCache;
GraphCache *graph_cache_create();
void graph_cache_destroy(GraphCache *gc);
struct GraphRun {
  void (*pre)(void *ctx, hipStream_t st, int n_launch, int s_launch, const CallSizes *live) = nullptr;
  void (*post)(void *ctx, hipStream_t st, int n_launch, int s_launch, const CallSizes *live) = nullptr;
  void *ctx = nullptr;
  GraphCache *cache = nullptr;
  hipStream_t capture_stream = nullptr;  // a stream of the caller's own (capture is not allowed on the null stream)
  bool use_graph = true;                 // false: the same launches, issued directly with the exact sizes
  long long captures = 0, replays = 0;   // counted here
};
// The capacity bucket of a size (what recorded launches are sized for).
int64_t launch_bucket(int64_t v);
int run_nlist(nnp_model *m, nnp_nlist *nl, int n_systems, const int64_t *offs, const int64_t *slots,
              const int32_t *rebuild, const float *coords, const int32_t *species, const float *box,
              double *energy, float *forces, double *virial, float *atom_energy, hipStream_t st,
              GraphRun *gr);

// A launch size: the value itself or, for launches recorded once and
// replayed for calls of other sizes (a graph per capacity bucket, its grids
// sized for the bucket), the device address where every call leaves its own
// value.  Kernels read it once on entry; blocks past the live size leave.
struct Live {
  int v;
  const int *p;
  __host__ __device__ Live(int v_ = 0, const int *p_ = nullptr) : v(v_), p(p_) {}
  __device__ __forceinline__ int get() const { return p ? *p : v; }
};

// Sizes of a call, the first bytes of its device descriptors.
struct CallSizes {
  int N, n_sys, n_cells, n_chunks, n_groups, pad[3];
};

constexpr int kWave = 64;
constexpr int kMaxSpecies = 7;
constexpr int kNShfRad = 16;
constexpr int kNShfAng = 4;
constexpr int kNShfZ = 8;
constexpr int kAngBlock = kNShfAng * kNShfZ;  // 32 features per species pair
constexpr int kTileM = 128;                   // MLP row tile; buckets pad to it

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): block b runs on XCD b % 8.  Logical block of dispatch slot bid when
// chunks of C consecutive logical blocks go to the XCDs in turn: the blocks
// of one chunk (those that share an operand tile) run on one XCD and hit the
// same L2, and any prefix of the logical blocks (the part of a grid sized
// for more rows than a call has) is spread evenly over all eight XCDs.  The
// grid must be a multiple of 8 C (xcd_grid); logical blocks past the real
// count exit at once.
__device__ inline int xcd_chunked(int bid, int C) {
  const int x = bid % 8, k = bid / 8;
  return ((k / C) * 8 + x) * C + (k % C);
}
__host__ inline unsigned xcd_grid(unsigned blocks, int C) {
  const unsigned g = 8u * (unsigned)C;
  return (blocks + g - 1) / g * g;
}

// Device status word bits.
enum : int { kStatOverflow = 1, kStatBadSpecies = 2, kStatBadPairs = 4 };

// One system of a batch, as the kernels see it.  Filled on the host except
// the non-periodic cell grid (origin/edge/nc), which a kernel derives from
// the system's bounding box.
struct SysDesc {
  float L[3];        // box lengths (periodic) or 0
  int periodic;
  int atom_off, n;   // atoms [atom_off, atom_off + n)
  int cell_off;      // first cell of this system in the global cell arrays
  int cell_cap;      // cells reserved for this system
  float origin[3];
  float edge[3];
  int nc[3];
  int rebuild;       // nonzero: build this system's neighbour list in this call
  int order_off;     // first wave of this system's centres in the AEV kernels'
                     // launch order (systems by decreasing size)
  long long list_off;   // first neighbour row of the system in the list pool
  long long state_off;  // first per-atom state slot (reference position, wrap)
};

// Offset from atom index to its slot in the fixed-point force accumulators
// (the launch order of the systems: slot = order_off + local index).
__host__ __device__ inline int fix_shift(const SysDesc &d) { return d.order_off - d.atom_off; }

// Persistent per-atom state of a neighbour list: the caller's coordinates at
// the last build (w unused) and the periodic wrap applied then (in box units).
struct AtomState {
  float4 ref;
  float4 wrap;
};

// Neighbour row of atom i (cap entries): entries hold (j - atom_off, image).
__host__ __device__ inline size_t nbr_row(const SysDesc &d, int i, int cap) {
  return (size_t)d.list_off + (size_t)(i - d.atom_off) * (size_t)cap;
}

// AEV hyper-parameters, passed by value to the AEV kernels.
struct AevConst {
  float rc_r, eta_r, rc_a, eta_a, zeta, scale;
  float shf_r[kNShfRad];
  float shf_a[kNShfAng];
  float hcz[kNShfZ], hsz[kNShfZ];  // halved cos / sin of the angle shifts
  int S;        // species
  int D;        // AEV length
  int rad_len;  // S * 16
};

// DeepPot-style descriptor parameters, passed by value to its kernels.
constexpr int kDpMaxSlots = 256;   // neighbours kept per centre, all species together
struct DpConst {
  double rc2;                  // cutoff squared, float64 (neighbour order and cutoff test)
  int S;                       // species
  int n_slots;                 // sum of sel
  int D;                       // 4 * n_slots
  int ldm;                     // slot records per centre: n_slots + 2 (frame neighbours a, b first)
  int sel[kMaxSpecies];        // neighbours kept per species
  int soff[kMaxSpecies];       // first slot of each species block
};

// Neighbour entry: j and a packed lattice image (10 bits per axis, +512).
__host__ __device__ inline int pack_image(int x, int y, int z) {
  return (x + 512) | ((y + 512) << 10) | ((z + 512) << 20);
}
__host__ __device__ inline void unpack_image(int c, int &x, int &y, int &z) {
  x = (c & 1023) - 512;
  y = ((c >> 10) & 1023) - 512;
  z = ((c >> 20) & 1023) - 512;
}

// ---- dense layers
constexpr int kMaxMembers = 8;  // ensemble members

struct GemmGroup {
  const void *B;      // [n_out][ldb] row-major, float or bf16; segment q at column q * K
  const float *bias;  // [n_out] (forward only)
  int n_out, K;       // K per segment
  int ldb;            // row stride of B in elements (0: n_seg * K)
  int pad;
};

struct GemmLaunch {
  const void *A; int lda;      // [rows][...] activations (operand type)
  int a_member_stride;         // column offset of member m's input
  int a_seg_stride;            // column offset of K segment q
  void *C; int ldc;            // output
  int c_member_stride;
  const void *H; int ldh;      // backward: layer input activations for CELU'
  int h_member_stride;
  const int *bucket_off;       // [n_groups + 1] padded row offsets (device)
  // Nullable: per row, bit h set when columns [16 h, 16 h + 16) of the AEV
  // row may be non-zero (the AEV forward's record of the real rows, the
  // first bucket_cnt rows of each bucket).  With it the direct-to-LDS kernel
  // skips the zero work of its row tile: first layer (A = the AEVs, one K
  // segment): K halves no row has; dE/dG output: column halves no row has,
  // not stored (their readers read a row's own halves only), and no MFMAs
  // for a wave whose columns are all such.
  const unsigned long long *row_mask;
  const int *bucket_cnt;       // [n_groups] real rows per bucket (with row_mask)
  int n_groups;                // species
  int n_members;               // grid dimension over ensemble members
  int n_seg;                   // K segments summed into one output
  int col_tiles;               // set by the launcher
  int k32;                     // every K and stride allows 32-wide K chunks (direct-to-LDS kernel)
  int span;                    // set by the launcher: members' columns side by side
  int n_blocks;                // set by the launcher: real blocks (the grid is padded)
  int xcd_chunk;               // set by the launcher: logical blocks per XCD chunk
  GemmGroup g[kMaxMembers * kMaxSpecies];  // [member][species]
  float alpha;                 // CELU alpha
  float scale;
};

enum { kEpiFwd = 0, kEpiBwd = 1, kEpiOut = 2 };

// Fused hidden-layer chain (bfloat16 models): layers 1 .. L-2 and the output
// layer of one (member, species) network, forward and input gradient.
constexpr int kChainRows = 32;   // rows per workgroup
constexpr int kChainMax = 3;     // hidden layers after the first, at most
struct ChainNet {
  const uint16_t *W[kChainMax];   // layer l: bfloat16 [width[l]][width[l-1]]
  const uint16_t *Wt[kChainMax];  // its transpose [width[l-1]][width[l]]
  const float *b[kChainMax];      // [width[l]]
  const float *w_out;             // output layer weights [width[NL]]
  float b_out;                    // output layer bias
  int width[kChainMax + 1];       // width of h_0 .. h_NL
};
struct ChainLaunch {
  const uint16_t *H0; int ldh; int h_member_stride;  // h_0 (first layer output)
  uint16_t *D0; int ldd; int d_member_stride;        // d_0 = dE/dz_0 out
  const ChainNet *nets;                               // device [member][species]
  const int *bucket_off; int n_groups; int n_members;
  int lds_off[kChainMax + 1];                         // byte offset of the h_l tile
  int lds_ld[kChainMax + 1];                          // its row stride (elements)
  float alpha, inv_m;
  float *e_mem;                                       // [rows][members] energies
  int n_blocks, xcd_chunk;                            // set by the launcher
  const int *perm; float *e_atom;
};

struct EnergyLaunch {
  const void *Hin; int ldh; int h_member_stride;  // input of the last layer
  void *Gout; int ldg; int g_member_stride;       // dE/d(input), scaled by inv_m
  const float *w[kMaxMembers * kMaxSpecies];
  const float *b[kMaxMembers * kMaxSpecies];
  int K[kMaxSpecies];
  const int *perm;            // row -> atom (-1 padding)
  const int *bucket_off;
  int n_groups, n_members;
  float *e_atom;
  float inv_m, alpha;
  int hidden, want_grad;
};

// ---- launchers (stream-ordered, no host sync)
void launch_skin_check(const float *coords, SysDesc *sys, Live n_sys, const AtomState *state,
                       float half_skin, int *stats, hipStream_t st);
// zero_forces (nullable): the force output, cleared here for the backward
// zero_fix (nullable): the fixed-point force accumulators, cleared here
// wave_atom (nullable): gets, at order_off + k, the k-th atom of each system.
void launch_ingest(const float *coords, const int *species, const unsigned char *mask,
                   const SysDesc *sys, Live n_sys, Live N, int S, float4 *pos, int *sys_of,
                   AtomState *state, int *status, float *zero_forces, unsigned long long *zero_fix,
                   int *wave_atom, hipStream_t st);
constexpr int kSmallSystem = 512;   // largest non-periodic system of the small-system search
void launch_nbr_small(const float4 *pos, const int *sys_of, const SysDesc *sys, Live N, float rc_list,
                      int cap, int2 *nbr, int *nbr_cnt, int *status, hipStream_t st);
void launch_pairs_to_rows(const int *pairs, const int *shifts, long long n_pairs, int half,
                          const unsigned char *mask, const float4 *pos, int N, const float L[3],
                          float rc, int cap, int2 *nbr, int *nbr_cnt, int *status, hipStream_t st);
void launch_grid(SysDesc *sys, Live n_sys, const float4 *pos, int *cell_count, float rc_list,
                 hipStream_t st);
void launch_cell_count(const float4 *pos, const int *sys_of, const SysDesc *sys, Live N,
                       int *cell_count, int *atom_cell, int *atom_slot, hipStream_t st);
void launch_scan(const int *in, int *out, Live n, hipStream_t st);
void launch_cell_scatter(const int *atom_cell, const int *atom_slot, const int *cell_start,
                         Live N, int *cell_atoms, hipStream_t st);
void launch_cell_sort(const int *cell_start, Live n_cells, int *cell_atoms, hipStream_t st);
void launch_nbr_build(const float4 *pos, const int *sys_of, const SysDesc *sys, Live n_sys, int n_cells,
                      const int *cell_start, const int *cell_atoms, Live N, float rc_list, int cap,
                      int2 *nbr, int *nbr_cnt, int *status, hipStream_t st);
// Rows of each species bucket follow the atoms in wave_atom's order (the AEV
// kernels' launch order: centres running together read neighbouring rows),
// or the atom order without it.
void launch_species_bucket(const float4 *pos, const int *wave_atom, Live N, int S, int *block_counts,
                           int n_blocks, int *bucket_off, int *bucket_cnt, int *perm, int *row_of_atom,
                           int rows_cap, hipStream_t st);
// DeepPot-style descriptor: forward into G rows (and the per-centre slot
// records {d, j} for the backward, nullable), backward from dE/dG and the
// records to forces and virial.
void launch_dp_fwd(const float4 *pos, const float *coords, const AtomState *state, const int *sys_of,
                   const SysDesc *sys, const int2 *nbr, const int *nbr_cnt, int cap,
                   const int *row_of_atom, void *G, bool g_bf16, int ldg, int N, const DpConst &c,
                   float4 *rec, int wpb_pref, hipStream_t st);
void launch_dp_bwd(const SysDesc *sys, int n_sys, bool small_systems, const int *cell_start,
                   const int *cell_atoms, int n_cells, const int *row_of_atom, const float *dG, int ldg, int N,
                   const DpConst &c, const float4 *rec, float *F, float *W_atom, int wpb_pref, hipStream_t st);
// row_mask (nullable): per G row, the 16-column halves that may be non-zero
// (radial species s: half s; angular species pair p: halves S + 2 p and
// S + 2 p + 1); every other half of the row is written as zeros.
// wave_atom (nullable): the centre of wave w (the ingest's launch order, the
// costliest systems first, so that no long centre starts last); else w.
// nbr null: no neighbour list; each centre takes the atoms of its system
// (small non-periodic systems of at most cap + 1 atoms) and records its
// neighbour count as the list build would, largest in status[1] (nullable).
void launch_aev_fwd(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                    const int *nbr_cnt, int cap, const int *row_of_atom, void *G, bool g_bf16,
                    int ldg, Live N, const AevConst &c, unsigned long long *row_mask, const int *wave_atom,
                    int *status, int wpb_pref, hipStream_t st);
// How the AEV backward groups its centres (at most one of the two forms):
// groups[n_groups] = {first centre, count} of consecutive centres of one
// small non-periodic system (max_sys_atoms: the largest such system), or the
// cell grid of the call.  Neither: one wave per centre.  Launches sized for
// more groups or cells than a call has read the live counts from live_*
// (nullable).
struct AevBwdGroups {
  const int2 *groups = nullptr;
  int n_groups = 0, max_sys_atoms = 0;
  const int *cell_start = nullptr, *cell_atoms = nullptr;
  int n_cells = 0;
  const int *live_groups = nullptr, *live_cells = nullptr;
  const int *wave_atom = nullptr;  // one wave per centre: the centre of wave w (nullable: w)
};
// Forces go into Ffix [N][3] (64-bit fixed point, cleared by the caller).
// nbr null: no neighbour list (as for launch_aev_fwd).
void launch_aev_bwd(const float4 *pos, const int *sys_of, const SysDesc *sys, const int2 *nbr,
                    const int *nbr_cnt, int cap, const int *row_of_atom, const float *dG,
                    int ldg, Live N, const AevConst &c, unsigned long long *Ffix, float *W_atom,
                    const AevBwdGroups &gp, int wpb_pref, size_t max_lds, hipStream_t st);
// tn_pref: column-tile width 64, 128 or 256 (anything else: the width heuristic).
void launch_gemm(int epi, bool bf16, GemmLaunch gl, int row_tiles, int max_n_out, int tn_pref, hipStream_t st);
void launch_energy(const EnergyLaunch &el, bool bf16, int rows, hipStream_t st);
// waves per workgroup 4 or 8; rt = 2: 64 rows per workgroup (2 lds_bytes of
// LDS), else 32
void launch_chain(ChainLaunch cl, int n_hidden, bool grad, int rows, size_t lds_bytes, int waves, int rt,
                  hipStream_t st);
// src: host memory the device reads directly (coherent pinned); bytes are
// rounded up to 16 on both sides
void launch_copy_from_host(const void *src, void *dst, size_t bytes, hipStream_t st);
void launch_fill(float *p, size_t n, float v, hipStream_t st);
void launch_fill_i32(int *p, size_t n, int v, hipStream_t st);
// Ffix (nullable): fixed-point forces, converted into F [N][3] float32 here.
// direct: chunk s is system s for every system (one pass, no partials).
void launch_reduce(const float *e_atom, const float *W_atom, const SysDesc *sys, Live n_sys,
                   const int *chunk_sys, const int *chunk_begin, Live n_chunks,
                   const int *sys_chunk_off, bool direct, double *partial, double *energy, double *virial,
                   const unsigned long long *Ffix, float *F, hipStream_t st);
void launch_gather_rows(const float *src, int ld, const int *row_of_atom, int N, int D,
                        float *dst, hipStream_t st);
void launch_export_nbr(const int2 *nbr, const int *nbr_cnt, int cap, const SysDesc *sys,
                       const int *sys_of, int N, int *counts, int *entries, int out_cap,
                       hipStream_t st);
void launch_f32_to_bf16(const float *src, uint16_t *dst, size_t n, hipStream_t st);

}  // namespace nnp
