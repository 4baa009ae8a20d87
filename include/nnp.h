/*
 * nnp.h - C ABI of the MI355X (gfx950) neural-network-potential library.
 *
 * The library evaluates an ANI-style high-dimensional neural network
 * potential (Deep-HP paper, arXiv 2207.14276): the total energy is the sum
 * of atomic energies, each produced by the network of the atom's element from
 * its atomic environment vector (AEV) (section "Neural Network Potentials",
 * energy-decomposition equation); the AEV is built from radial and angular
 * symmetry functions with a cosine cutoff (section "ANI models", cutoff,
 * radial and angular equations) over a cell-list neighbour search
 * (section "Massive Parallelism within Tinker-HP"); forces are the analytic
 * negative gradient of the energy.  Device data crosses this boundary as raw
 * addresses with no copies (section "A General Machine Learning Platform").
 *
 * Conventions for every call:
 *   - All functions return NNP_OK (0) on success and a negative NNP_E* code on
 *     failure; none throws.  nnp_last_error() then holds a message for the
 *     calling thread.
 *   - "DEVICE" pointers are HIP device allocations on the model's device
 *     (e.g. torch tensors' data_ptr()); "HOST" pointers are host memory that
 *     the call reads before it returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and
 *     the call returns without waiting for it; outputs are valid once the
 *     stream reaches that point.  The caller keeps every device buffer alive
 *     until then.
 *   - A model is used by one host thread at a time.
 */
#ifndef NNP_H
#define NNP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NNP_OK = 0,
  NNP_EINVAL = -1,       /* bad argument (null pointer, bad offsets, ...) */
  NNP_ENOMEM = -2,       /* device or pinned host allocation failed */
  NNP_ECAPACITY = -3,    /* a neighbour list overflowed its capacity */
  NNP_EDEVICE = -4,      /* a HIP runtime error; message carries its text */
  NNP_ESPECIES = -5,     /* an atom's species index is outside the model */
  NNP_EUNSUPPORTED = -6  /* a valid description this build does not run */
};

enum { NNP_FP32 = 0, NNP_BF16 = 1 };

typedef struct nnp_model nnp_model; /* opaque, library-owned */

/* AEV hyper-parameters (section "ANI models").  The radial term of
 * neighbour j at distance R is radial_scale * exp(-eta_rad (R - Rs)^2) fc(R)
 * with fc(R) = 0.5 cos(pi R / rc) + 0.5 for R < rc, else 0.  The angular term
 * of an unordered neighbour pair {j, k} inside rc_ang is
 * 2^(1-zeta) (1 + cos(theta_ijk - theta_s))^zeta
 *   * exp(-eta_ang ((R_ij + R_ik)/2 - Rs)^2) fc(R_ij) fc(R_ik).
 * Feature layout: radial block of neighbour species s at s*n_shf_rad + m;
 * angular block of the species pair (a <= b), numbered row by row through the
 * upper triangle, at n_species*n_shf_rad + pair*(n_shf_ang*n_shf_z)
 * + r*n_shf_z + z.  Host arrays, copied at creation.
 * This build runs n_shf_rad = 16, n_shf_ang = 4, n_shf_z = 8, n_species <= 7
 * and rc_ang <= rc_rad; other values give NNP_EUNSUPPORTED. */
typedef struct {
  int n_species;
  float rc_rad, eta_rad;
  int n_shf_rad;
  const float *shf_rad;
  float rc_ang, eta_ang, zeta;
  int n_shf_ang;
  const float *shf_ang;
  int n_shf_z;
  const float *shf_z; /* angle shifts theta_s, radians */
  float radial_scale;
} nnp_aev_params;

/* A set of element networks (section "Neural Network Potentials").  Each
 * species s has n_layers[s] fully connected layers; hidden layers apply
 * CELU(z) = max(0, z) + min(0, alpha (exp(z / alpha) - 1)); the last layer
 * has one output, the atomic energy.  With n_ensemble > 1 the atomic energy
 * is the mean over the ensemble members.
 *   widths:  per species, n_layers[s] + 1 widths, concatenated; the first is
 *            the AEV length, the last is 1.  All species must have the same
 *            number of layers in this build.
 *   weights: float32, concatenated over (member, species, layer), each layer
 *            as W[out][in] row-major followed by b[out].
 * All arrays are HOST memory, copied by nnp_create (the caller may free them
 * afterwards).  precision = NNP_FP32 runs the dense layers in float32;
 * NNP_BF16 rounds their operands to bfloat16 and accumulates in float32; AEV,
 * forces and per-atom energies stay float32 and the per-system energy and
 * virial sums are float64 in both. */
typedef struct {
  nnp_aev_params aev;
  int n_ensemble;
  const int *n_layers;
  const int *widths;
  const float *weights;
  float celu_alpha;
  int precision;
} nnp_model_desc;

/* Builds a model on device hip_device (< 0: the calling thread's current
 * HIP device); the caller's current device is left as it was.  *out receives
 * the handle.  Every later call on the model runs on that device.  The
 * weights are copied (section "A General Machine Learning Platform": the
 * model is set up once, then fed positions every step). */
int nnp_create(const nnp_model_desc *desc, int hip_device, nnp_model **out);
void nnp_destroy(nnp_model *model);

/* DeepPot-style local-frame descriptor (section "DeePMD Models"), a second
 * model family behind the same entry points.  The neighbours of a centre
 * within rc are grouped by species (ascending slot) and ordered nearest
 * first; at most sel[s] of species s are kept, in slots
 * sel[0] + ... + sel[s-1] + rank, and each kept neighbour fills four features
 * {1/R, x/R, y/R, z/R}: (x, y, z) = (d . e_x, d . e_y, d . e_z) in the
 * centre's local frame, e_x along the nearest neighbour a, e_y along the part
 * of the second nearest b orthogonal to e_x, e_z = e_x x e_y (e_y = e_z = 0
 * with a single neighbour or when b is collinear with a, |u|^2 <= 1e-12
 * |d_b|^2).  Empty slots are zero; the descriptor length is 4 * sum(sel).
 * The neighbour order and the cutoff test are decided in float64 from the
 * caller's float32 coordinates: d = (r_j - r_i) + n L (n the lattice image
 * relative to those coordinates), R^2 = (dx dx + dy dy) + dz dz, R^2 < rc^2,
 * each operation rounded on its own; exact ties go to the smaller neighbour
 * index within the system, then the smaller image (x, y, z).  No smoothing
 * at the cutoff.  Neighbour lists reach rc + 1e-3 A (plus a pool's skin).
 * This build runs n_species <= 7 and sum(sel) <= 256. */
typedef struct {
  int n_species;
  float rc;        /* cutoff, Angstrom */
  const int *sel;  /* HOST int[n_species], copied at creation */
} nnp_dp_params;

/* A DeepPot-style model: the descriptor and the same element networks as
 * nnp_model_desc (widths[s][0] must be 4 * sum(sel)). */
typedef struct {
  nnp_dp_params dp;
  int n_ensemble;
  const int *n_layers;
  const int *widths;
  const float *weights;
  float celu_alpha;
  int precision;
} nnp_dp_model_desc;

/* Builds a DeepPot-style model on device hip_device (< 0: the current one;
 * as nnp_create); the handle works with every entry point below (energies,
 * forces, virials, pair lists, persistent lists, descriptor export,
 * serving). */
int nnp_create_dp(const nnp_dp_model_desc *desc, int hip_device, nnp_model **out);

/* Pre-sizes the library workspace (the paper's bounded up-front buffer,
 * section "Massive Parallelism within Tinker-HP") for calls of up to
 * max_atoms atoms and max_systems systems, and sets the per-atom neighbour
 * list capacity (0 keeps the current one; default 256).  Without it the
 * workspace grows on demand, which synchronizes the device. */
int nnp_reserve(nnp_model *model, int64_t max_atoms, int max_systems, int nbr_capacity);

/* Energy and forces of a batch of independent systems: per system the sum
 * of the atomic energies of its atoms (section "Neural Network Potentials",
 * energy-decomposition equation; with an ensemble, the mean over members,
 * section "Neural Network Potentials"), each from the element network of its
 * AEV (section "ANI models", radial and angular equations) over the atoms and
 * periodic images within the cutoff (neighbour search: section "Massive
 * Parallelism within Tinker-HP"), and the forces as the analytic negative
 * gradient.  Positions go in and energies and forces come out as device
 * addresses (section "A General Machine Learning Platform").
 * The call only enqueues: it does not wait for the device, except when the
 * workspace must grow (see nnp_reserve) or when the descriptors of 32
 * earlier calls are still being copied (a ring of pinned staging slots).
 * Calls on one model share its workspace: they must be on one stream, or
 * ordered by the caller.
 *   n_systems      >= 1
 *   batch_offsets  HOST int64[n_systems + 1]; offsets[0] = 0, non-decreasing;
 *                  system s owns atoms [offsets[s], offsets[s+1]).
 *   coords         DEVICE float32[N][3], Angstrom, N = offsets[n_systems].
 *   species        DEVICE int32[N], slot index < n_species.  An index outside
 *                  the model sets a device flag that nnp_status reports as
 *                  NNP_ESPECIES; that call's outputs are then undefined.
 *   box            HOST float32[n_systems][3]: orthorhombic box lengths of a
 *                  periodic system, or 0,0,0 for a non-periodic one.  Every
 *                  periodic image inside the cutoff is a neighbour, so boxes
 *                  smaller than twice the cutoff are valid.
 *   energy         DEVICE float64[n_systems] out, kcal/mol.
 *   forces         DEVICE float32[N][3] out, kcal/mol/A, or NULL for energy
 *                  only (skips the backward pass).
 *   virial         DEVICE float64[n_systems][9] out, row-major
 *                  W = -sum over neighbour terms of d (x) dE/dd (equal to
 *                  sum_i r_i (x) F_i for a non-periodic system), or NULL.
 *                  Requires forces != NULL.
 *   atom_energy    DEVICE float32[N] out (ensemble-mean atomic energies), or
 *                  NULL.
 * Neighbour-list overflow sets a device flag (nnp_status -> NNP_ECAPACITY). */
int nnp_energy_forces(nnp_model *model, int n_systems, const int64_t *batch_offsets,
                      const float *coords, const int32_t *species, const float *box,
                      double *energy, float *forces, double *virial, float *atom_energy,
                      void *stream);

/* nnp_energy_forces without any allocation, for callers that cannot
 * allocate device memory: code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * nnp_energy_forces; the call's whole workspace (atom records, cells,
 * neighbour rows, AEV and activation rows, force accumulators, descriptors)
 * comes from a fixed 64 MiB device array that the library holds on every
 * device it runs on until the process ends, and the descriptors go through
 * the model's existing pinned staging slots.  It calls no hipMalloc,
 * hipFree or other allocating routine.
 *   Limits: a call whose workspace exceeds the 64 MiB (with the ANI-2x
 *   widths and the default capacity of 256 neighbours, roughly 4,000 atoms
 *   in float32 and 6,000 in bfloat16; the message gives the bytes needed),
 *   or whose descriptors exceed a 128 KiB staging slot (about 1,400
 *   systems), is refused with NNP_EUNSUPPORTED before anything is
 *   enqueued.
 *   Sharing: every call on a device, on any model, uses that device's one
 *   array; calls that overlap on a device (other streams, other threads)
 *   race and give undefined results.  Each call clears what must start at
 *   zero; nothing of an earlier call's contents is used. */
int nnp_energy_forces_noalloc(nnp_model *model, int n_systems, const int64_t *batch_offsets,
                              const float *coords, const int32_t *species, const float *box,
                              double *energy, float *forces, double *virial, float *atom_energy,
                              void *stream);

/* Persistent neighbour lists (device-resident state for repeated calls on
 * slowly moving systems, e.g. successive MD steps).  A pool holds `slots`
 * atom slots; each system of a call occupies a caller-chosen range of slots
 * for as long as it lives, wherever its atoms sit in that call's batch.  A
 * system's list is built with cutoff rc_rad + skin and reused until one of
 * its atoms has moved more than skin / 2 from where it was at the last build
 * (checked on the device every call), so no neighbour can enter the cutoff
 * unseen.  Periodic coordinates are not re-wrapped while a list is reused.
 * nnp_nlist_create allocates device memory (slots * capacity * 8 bytes plus
 * 36 bytes per slot); capacity <= 1024. */
typedef struct nnp_nlist nnp_nlist;
int nnp_nlist_create(nnp_model *model, int64_t slots, int capacity, float skin, nnp_nlist **out);
void nnp_nlist_destroy(nnp_nlist *list);

/* As nnp_energy_forces, with the neighbour lists kept in `list`:
 *   slots    HOST int64[n_systems]: first pool slot of each system; the ranges
 *            [slots[s], slots[s] + n_s) lie inside the pool and do not
 *            overlap (NNP_EINVAL otherwise).
 *   rebuild  HOST int32[n_systems] or NULL: nonzero forces a fresh list for
 *            that system (set it the first time a system uses its slots, or
 *            after its atoms were renumbered).
 * The pool records, per system (by its first slot), the box, the list
 * cutoff (the model's cutoff + skin) and the atom count its rows were built
 * for; a call that differs in any of them rebuilds that system's rows, so a
 * pool can be shared by models of different cutoffs and by systems whose box
 * changes.  Renumbered atoms are not detected: use rebuild. */
int nnp_energy_forces_nlist(nnp_model *model, nnp_nlist *list, int n_systems,
                            const int64_t *batch_offsets, const int64_t *slots,
                            const int32_t *rebuild, const float *coords, const int32_t *species,
                            const float *box, double *energy, float *forces, double *virial,
                            float *atom_energy, void *stream);

/* Energy and forces of one system from the caller's own pair list, over an
 * ML region (section "A General Machine Learning Platform": the host MD code
 * keeps the neighbour list and passes positions and pairs; section "Hybrid
 * Model: Neural Network Solutes in AMOEBA Polarizable Solvent/Protein": the
 * network sees only the solute P, whose environments contain solute atoms
 * only, giving V_ML(P) of the hybrid potential).
 *   n_atoms   atoms of the system (N).
 *   coords    DEVICE float32[N][3], species DEVICE int32[N] (as above; the
 *             species of every atom, inside the region or not, must be a
 *             valid slot).
 *   box       HOST float32[3]: lengths that scale the lattice shifts (0 for a
 *             non-periodic system).  Coordinates are used as given (no
 *             wrapping): a shift is relative to them.
 *   pairs     DEVICE int32[n_pairs][2] (i, j): atom j moved by the lattice
 *             vector shifts[p] * box is a neighbour of atom i.  half_list = 1:
 *             each unordered pair appears once and both directions are used;
 *             half_list = 0: each direction appears.  Pairs at a distance
 *             >= rc_rad are ignored, so a list built with a larger cutoff
 *             (and skin) may be passed.  A pair inside the cutoff listed
 *             twice, an index outside [0, N), i == j with a zero shift, or a
 *             shift component beyond +-511 sets a device flag (nnp_status ->
 *             NNP_EINVAL).
 *   shifts    DEVICE int32[n_pairs][3] or NULL (all zero).
 *   ml_mask   DEVICE uint8[N] or NULL (every atom): atoms with a zero entry
 *             are outside the ML region; pairs touching them are ignored,
 *             they contribute no energy and receive zero force.
 *   energy    DEVICE float64[1]: E_ML = sum of the atomic energies of the
 *             region.  forces / virial / atom_energy as in nnp_energy_forces
 *             (virial: -sum over pairs d (x) dE/dd with the image vectors).
 * More than `capacity` neighbours of one atom inside the cutoff set the
 * overflow flag (nnp_status -> NNP_ECAPACITY, with the largest count); the
 * capacity is the model's (nnp_reserve).  Enqueues on `stream`; no host
 * synchronization. */
int nnp_energy_forces_pairs(nnp_model *model, int64_t n_atoms, const float *coords,
                            const int32_t *species, const float *box, int64_t n_pairs,
                            const int32_t *pairs, const int32_t *shifts, int half_list,
                            const uint8_t *ml_mask, double *energy, float *forces, double *virial,
                            float *atom_energy, void *stream);

/* Waits for `stream`; *builds = number of system lists built in the pool so
 * far (forced and skin-triggered). */
int nnp_nlist_builds(nnp_nlist *list, void *stream, int64_t *builds);

/* Same inputs; writes the descriptor (AEV, or the DeepPot-style
 * environment) of every atom, DEVICE float32[N][nnp_aev_dim], atom order.
 * For tests and inspection. */
int nnp_debug_aev(nnp_model *model, int n_systems, const int64_t *batch_offsets,
                  const float *coords, const int32_t *species, const float *box,
                  float *aev_out, void *stream);

/* Same inputs; writes the neighbour lists the last build produced:
 * DEVICE int32[N] counts and DEVICE int32[N][capacity][4] entries
 * (j, image x, image y, image z), up to `capacity` per atom.  For tests. */
int nnp_debug_neighbors(nnp_model *model, int n_systems, const int64_t *batch_offsets,
                        const float *coords, const int32_t *species, const float *box,
                        int32_t *counts, int32_t *entries, int capacity, void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of energy/force requests (a request is one
 * system and a number of successive evaluations, as an MD client or a
 * free-energy window produces them).
 *
 * Every admitted request keeps its coordinates, species and persistent
 * neighbour list (cutoff rc_rad + skin, rebuilt when an atom has moved more
 * than skin / 2) on the device.  Each nnp_server_step admits queued requests
 * first-come first-served (a contiguous range of `slots` of the request's
 * size must be free, the atoms of one iteration stay within the batch budget
 * and the requests in flight within max_active) and enqueues one iteration:
 * the next step of every request in flight in one batched evaluation,
 * followed by the built-in client's move of each continuing request, a random
 * walk x += sigma * z per coordinate with z ~ N(0, 1) drawn from Philox4x32-10
 * (Salmon et al., SC 2011; counter = (atom index in the request, step + 1,
 * 0, 0), key = seed) and the Box-Muller transform, so a request's trajectory
 * and results do not depend on what it is batched with.  Two iterations are
 * kept in flight; results are filed when an iteration's work has completed.
 *
 * Memory: the server allocates its coordinate store and list pool for
 * `slots` atoms, batch buffers, and grows the model's workspace once, for the
 * largest per-iteration atom count that fits `hbm_budget` bytes (0 = 90% of
 * the device memory free at creation) and max_batch_atoms (0 = no limit
 * beyond the budget and the slots).  Requests that do not fit wait in the
 * queue; a request larger than the pool or the batch budget is refused.
 * The server uses the model exclusively while it lives (same host thread).
 *
 * Graphs (use_graphs = 1): an iteration's kernels (gather, list update,
 * descriptor, dense layers, backward, reductions, client move) are recorded
 * once per capacity bucket into a HIP graph on a stream of the server's own
 * and replayed on the caller's stream for every later iteration whose atom
 * and request counts round up to the same bucket (the next of 2^k, 1.25,
 * 1.5 and 1.75 times 2^k): grids are sized for the bucket and the kernels
 * read the iteration's own sizes from its descriptors, uploaded before the
 * replay.  Graphs hold no memset or allocation nodes.  The workspace is
 * reserved for the bucket of the batch budget; the 48 most recently used
 * graphs are kept.  Models of the DeepPot-style descriptor launch directly.
 * ---------------------------------------------------------------------- */
typedef struct nnp_server nnp_server;

typedef struct {
  int64_t slots;            /* atom slots (coordinate store and list pool) */
  int nbr_capacity;         /* neighbour entries per atom in the pool, <= 1024 */
  float skin;               /* list skin, Angstrom */
  int64_t max_batch_atoms;  /* atoms per iteration at most, 0 = memory-bound */
  int max_active;           /* requests in flight at most, >= 1 */
  uint64_t hbm_budget;      /* device bytes granted to the server, 0 = 90% of free */
  int use_graphs;           /* 1: each iteration's kernels are recorded once per
                             * capacity bucket as a HIP graph and replayed (see
                             * below); 0: launched one by one */
} nnp_server_opts;

typedef struct {
  int n_atoms;
  const float *coords;     /* HOST float32[n_atoms][3], copied by the call */
  const int32_t *species;  /* HOST int32[n_atoms], copied by the call */
  float box[3];            /* orthorhombic box lengths or 0,0,0 */
  int n_steps;             /* evaluations requested, >= 1 */
  float sigma;             /* random-walk step per coordinate, Angstrom */
  uint64_t seed;           /* random-walk key */
} nnp_request;

typedef struct {
  int64_t iterations;       /* iterations launched */
  int64_t atom_evals;       /* sum over iterations of the atoms evaluated */
  int64_t queued, active;   /* requests waiting / in flight */
  int64_t max_batch_atoms;  /* the per-iteration atom budget in force */
  int64_t max_batch_seen;   /* largest iteration so far */
  uint64_t device_bytes;    /* device memory granted at creation (estimate) */
  int64_t list_builds;      /* neighbour lists built (waits for the device) */
  int64_t graph_captures;   /* iterations recorded as a new graph */
  int64_t graph_replays;    /* iterations launched as a graph (recorded ones included) */
  double host_launch_s;     /* host time spent admitting, staging and enqueuing iterations */
} nnp_server_counters;

/* NNP_ENOMEM when the slots or a batch of one atom do not fit the budget;
 * waits for the device and fails with the flag's code if the model has a
 * device flag raised (see nnp_status). */
int nnp_server_create(nnp_model *model, const nnp_server_opts *opts, nnp_server **out);
/* Waits for the work in flight, then frees everything. */
void nnp_server_destroy(nnp_server *server);
/* Seconds on the server's monotonic clock (0 at creation). */
double nnp_server_clock(const nnp_server *server);
/* Queues a request; t_arrival on the server clock (< 0: now).  *id receives
 * its handle (ids count up from 0).  NNP_EINVAL if it can never run,
 * NNP_ESPECIES if a species index is outside the model. */
int nnp_server_submit(nnp_server *server, const nnp_request *req, double t_arrival, int64_t *id);
/* Admits, launches one iteration on `stream` if any request is in flight,
 * and files the results of completed iterations (waiting while two are in
 * flight).  *pending (nullable) = requests queued or in flight plus
 * iterations not yet filed; 0 means everything submitted is finished.
 * A request whose neighbour list overflows the pool's capacity (on any
 * build) stops alone: it is reported finished by nnp_server_poll and
 * nnp_server_result returns NNP_ECAPACITY for it (naming the count), while
 * every other request goes on unaffected (section "Massive Parallelism
 * within Tinker-HP": buffers are bounded up front, and a request that does
 * not fit must not bring the run down).  Species are checked when a request
 * is submitted (NNP_ESPECIES). */
int nnp_server_step(nnp_server *server, void *stream, int64_t *pending);
/* Waits for every launched iteration and files its results. */
int nnp_server_drain(nnp_server *server);
/* Ids of up to max finished requests not yet reported; *n = how many. */
int nnp_server_poll(nnp_server *server, int64_t *ids, int max, int *n);
/* Results of a finished request, each output nullable: energies HOST
 * float64[n_steps] (kcal/mol, one per step), coords and forces HOST
 * float32[n_atoms][3] of the last step (coordinates evaluated, kcal/mol/A),
 * times HOST float64[3] = arrival, admission, completion (server clock; the
 * completion time is when the host saw the last step's results).  Releases
 * the request's record: a second call fails with NNP_EINVAL.  For a request
 * that stopped on a neighbour overflow it fills only times (completion =
 * when the overflow was seen) and returns NNP_ECAPACITY. */
int nnp_server_result(nnp_server *server, int64_t id, double *energies, float *coords, float *forces,
                      double *times);
int nnp_server_stats(nnp_server *server, nnp_server_counters *out);

/* The server's admission logic on its own, host only (no device use): for
 * callers that drive their own evaluation, and for tests.
 *   submit   NNP_EINVAL if the request can never run or the id is in use.
 *   admit    admits from the head of the queue; ids/slots (nullable) get the
 *            admitted requests and their first slots, at most max.
 *   launch   one step of every request in flight, in admission order: ids,
 *            slots, n_atoms, steps (0-based step index), each nullable, at
 *            most max.  A request whose last step is launched leaves the
 *            flight and frees its slots.
 *   complete results of one launched step of id are back at time `now`;
 *            *finished = 1 when it was the last.
 *   fail     stops an admitted, unfinished request at time `now` (its
 *            evaluation failed): it leaves the flight, frees its slots and
 *            counts as finished; NNP_EINVAL otherwise.
 *   job      times[3] = arrival, admission, completion (-1 = not yet), first
 *            slot and steps completed of a known request.
 *   info     info[6] = queued, in flight, atoms in flight, free slots,
 *            iterations, atom-evals. */
typedef struct nnp_sched nnp_sched;
int nnp_sched_create(int64_t slots, int64_t max_batch_atoms, int max_active, nnp_sched **out);
void nnp_sched_destroy(nnp_sched *sched);
int nnp_sched_submit(nnp_sched *sched, int64_t id, int n_atoms, int n_steps, double t_arrival);
int nnp_sched_admit(nnp_sched *sched, double now, int64_t *ids, int64_t *slots, int max, int *n);
int nnp_sched_launch(nnp_sched *sched, int64_t *ids, int64_t *slots, int32_t *n_atoms, int32_t *steps,
                     int max, int *n);
int nnp_sched_complete(nnp_sched *sched, int64_t id, double now, int *finished);
int nnp_sched_fail(nnp_sched *sched, int64_t id, double now);
int nnp_sched_job(nnp_sched *sched, int64_t id, double *times, int64_t *slot, int32_t *steps_done);
int nnp_sched_info(nnp_sched *sched, int64_t *info);

/* Tile-shape tuning for a representative batch (section "Massive Parallelism
 * within Tinker-HP" reports the kernel time split that makes these choices
 * matter).  Runs the batch (inputs as for nnp_energy_forces, energies and
 * forces computed into the call's own scratch) with each candidate round's
 * shapes, the rounds taking turns six times (the first untimed), and keeps,
 * for every tunable launch ("site"), the candidate with the fastest of its
 * times measured with HIP events on `stream`:
 *   site 0           AEV forward: waves per workgroup 1, 2 or 4 (candidates
 *                    whose LDS does not fit are skipped);
 *   site 1           AEV backward: 1 wave per centre (forces by device
 *                    atomics), or 4, 5 or 8 waves per workgroup summing the
 *                    forces of a system (batches of small non-periodic
 *                    systems) or of a cell (cell grids) in LDS first;
 *   site 2 + l       dense layer l forward GEMM: column-tile width 64, 128
 *                    or 256 (256: for a layer whose members share the input,
 *                    the members' columns side by side in one tile space);
 *   site 10 + l      dense layer l input-gradient GEMM: width 64, 128 or 256;
 *   site 18          the dE/dG GEMM: width 64, 128 or 256;
 *   site 19          the fused hidden-layer chain: 4 or 8 waves per workgroup on
 *                    32 rows, or 18: 8 waves on 64 rows (when twice the LDS fits).
 * The choices stay with the model for all later calls (no call changes any
 * result: tile shapes change no per-element arithmetic order); sites that did
 * not run keep their default (0).  Waits for the stream; allocates. */
int nnp_autotune(nnp_model *model, int n_systems, const int64_t *batch_offsets, const float *coords,
                 const int32_t *species, const float *box, void *stream);
/* Copies up to n tuned site values (0 = default shape) into values; returns
 * the number of sites (20). */
int nnp_tuning(const nnp_model *model, int *values, int n);

/* Bennett acceptance ratio estimate of a free-energy difference between two
 * states, host only (section "Accelerating Hybrid Simulations: an
 * Alternative Reweighting Strategy" and its supplementary section: stored
 * snapshots of a reference ensemble U are re-evaluated with the network's
 * energies (nnp_energy_forces with forces = NULL) and reweighted to the
 * hybrid potential U').  Reduced units (energies times beta):
 *   u[n0]   HOST float64: beta (U_1 - U_0) on the samples of state 0;
 *   v[n1]   HOST float64: beta (U_0 - U_1) on the samples of state 1;
 *   lw0, lw1  HOST float64 log weights of the samples, or NULL (unweighted):
 *           -beta (U'_s - U_s) to reweight samples of ensemble U to U';
 *           u and v are then differences of U'.
 *   delta   out: beta (F_1 - F_0), the root of Bennett's self-consistent
 *           equation with the variance-minimizing constant (sample sizes
 *           n1/n0, or Kish effective sizes when weighted);
 *   sigma   out (or NULL): its asymptotic standard deviation.
 * NNP_EINVAL for empty or non-finite samples, or no overlap. */
int nnp_bar(int64_t n0, const double *u, const double *lw0, int64_t n1, const double *v,
            const double *lw1, double *delta, double *sigma);

/* Waits for `stream` and returns the device flags raised since the last
 * nnp_status call (NNP_ECAPACITY, NNP_ESPECIES) or NNP_OK; clears them.
 * *max_neighbors (nullable) receives the largest neighbour count seen. */
int nnp_status(nnp_model *model, void *stream, int *max_neighbors);

/* Descriptor length of the model: the AEV length (1008 for 7 species), or
 * 4 * sum(sel) for a DeepPot-style model. */
int nnp_aev_dim(const nnp_model *model);

/* Message of the last failed call on this thread ("" if none). */
const char *nnp_last_error(void);

/* Per-stage timing with HIP events recorded on the call's stream.
 * nnp_set_timing(model, 1) turns it on and clears what was recorded; every
 * later nnp_energy_forces / nnp_energy_forces_nlist call records one set of
 * stage-boundary events (up to 4096 calls between two reads; calls beyond
 * that are not timed).  nnp_set_timing(model, 2 + s) records only the two
 * events around stage s (each event costs a few microseconds of device time,
 * so timing one stage disturbs the calls least); 0 turns timing off; other
 * values give NNP_EINVAL.  nnp_stage_timings waits for the last recorded
 * call, writes up to n stage durations in ms, each the mean over the calls
 * recorded since the previous read (-1 for stages not recorded), with the
 * stage names (static strings), clears the record and returns the number of
 * stages (0 when nothing was recorded).  The recording adds no wait to the
 * calls themselves. */
int nnp_set_timing(nnp_model *model, int enable);
int nnp_stage_timings(nnp_model *model, float *ms_out, const char **names_out, int n);

#ifdef __cplusplus
}
#endif

#endif /* NNP_H */
