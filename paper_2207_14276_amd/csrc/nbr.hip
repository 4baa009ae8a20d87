// Ingest, cell list and neighbour list (linked-cell search, section
// "Massive Parallelism within Tinker-HP"), species buckets, small utilities.
#include "internal.h"

namespace nnp {

// ------------------------------------------------------------------ ingest
// Caller AoS float32[N][3] -> packed 16-byte atom records {x, y, z, species}.
// A system whose neighbour list is (re)built in this call has its periodic
// coordinates wrapped into [0, L) and the wrap and the caller's coordinates
// recorded; a system that reuses its list applies the recorded wrap instead,
// so neighbour vectors stay consistent with the stored lattice images.
constexpr int kIngestLdsSystems = 1024;  // more systems: staging costs more than it saves

__global__ void k_ingest(const float *__restrict__ coords, const int *__restrict__ species,
                         const unsigned char *__restrict__ mask,
                         const SysDesc *__restrict__ sys, Live n_sys_, Live N_, int S,
                         float4 *__restrict__ pos, int *__restrict__ sys_of,
                         AtomState *__restrict__ state, int *__restrict__ status,
                         float *__restrict__ zero_forces, unsigned long long *__restrict__ zero_fix,
                         int *__restrict__ wave_atom) {
  const int n_sys = n_sys_.get(), N = N_.get();
  // the systems' first atoms, staged in LDS when they fit: the search below
  // then waits on LDS instead of on a chain of dependent global loads
  __shared__ int s_off[kIngestLdsSystems];
  const bool staged = n_sys <= kIngestLdsSystems;
  if (staged) {
    for (int k = threadIdx.x; k < n_sys; k += blockDim.x) s_off[k] = sys[k].atom_off;
    __syncthreads();
  }
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  // the force output starts from zero (the backward accumulates into it)
  if (zero_forces) {
    zero_forces[3 * (size_t)i] = 0.f;
    zero_forces[3 * (size_t)i + 1] = 0.f;
    zero_forces[3 * (size_t)i + 2] = 0.f;
  }
  if (zero_fix) {
    zero_fix[3 * (size_t)i] = 0ull;
    zero_fix[3 * (size_t)i + 1] = 0ull;
    zero_fix[3 * (size_t)i + 2] = 0ull;
  }
  auto first_atom = [&](int k) { return staged ? s_off[k] : sys[k].atom_off; };
  // system of atom i: last s with atom_off <= i (binary search)
  int lo = 0, hi = n_sys - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (first_atom(mid) <= i) lo = mid; else hi = mid - 1;
  }
  // skip empty systems that share the offset
  while (lo + 1 < n_sys && first_atom(lo + 1) <= i) ++lo;
  const SysDesc &d = sys[lo];
  if (wave_atom) wave_atom[d.order_off + (i - d.atom_off)] = i;
  const float cx = coords[3 * i], cy = coords[3 * i + 1], cz = coords[3 * i + 2];
  float x = cx, y = cy, z = cz;
  AtomState &a = state[d.state_off + (i - d.atom_off)];
  if (d.periodic) {
    float wx, wy, wz;
    if (d.rebuild) {
      wx = floorf(cx / d.L[0]); wy = floorf(cy / d.L[1]); wz = floorf(cz / d.L[2]);
    } else {
      const float4 w = a.wrap;
      wx = w.x; wy = w.y; wz = w.z;
    }
    x = cx - wx * d.L[0];
    y = cy - wy * d.L[1];
    z = cz - wz * d.L[2];
    if (d.rebuild) {
      // rounding can land exactly on L: fold into the cell grid's range
      if (x >= d.L[0]) { x -= d.L[0]; wx += 1.f; }
      if (y >= d.L[1]) { y -= d.L[1]; wy += 1.f; }
      if (z >= d.L[2]) { z -= d.L[2]; wz += 1.f; }
      a.wrap = make_float4(wx, wy, wz, 0.f);
    }
  }
  if (d.rebuild) a.ref = make_float4(cx, cy, cz, 0.f);
  int s = species[i];
  if (s < 0 || s >= S) {
    atomicOr(status, kStatBadSpecies);
    s = 0;
  }
  // an atom outside the caller's mask has no network (species slot -1)
  if (mask && !mask[i]) s = -1;
  pos[i] = make_float4(x, y, z, __int_as_float(s));
  sys_of[i] = lo;
}

void launch_ingest(const float *coords, const int *species, const unsigned char *mask,
                   const SysDesc *sys, Live n_sys, Live N, int S, float4 *pos, int *sys_of,
                   AtomState *state, int *status, float *zero_forces, unsigned long long *zero_fix,
                   int *wave_atom, hipStream_t st) {
  if (N.v <= 0) return;
  k_ingest<<<(N.v + 255) / 256, 256, 0, st>>>(coords, species, mask, sys, n_sys, N, S, pos, sys_of,
                                            state, status, zero_forces, zero_fix, wave_atom);
}

// One wave per system: a system that keeps its neighbour list is rebuilt
// once any atom has moved more than half the skin since the last build
// (then no pair can have entered the cutoff unseen).  stats[0] counts builds.
__global__ void k_skin_check(const float *__restrict__ coords, SysDesc *__restrict__ sys, Live n_sys,
                             const AtomState *__restrict__ state, float half_skin,
                             int *__restrict__ stats) {
  const int s = blockIdx.x;
  if (s >= n_sys.get()) return;
  const int lane = threadIdx.x;
  const SysDesc d = sys[s];
  int rebuild = d.rebuild;
  if (!rebuild) {
    float mx = 0.f;
    for (int a = lane; a < d.n; a += kWave) {
      const int i = d.atom_off + a;
      const float4 r = state[d.state_off + a].ref;
      const float dx = coords[3 * i] - r.x, dy = coords[3 * i + 1] - r.y, dz = coords[3 * i + 2] - r.z;
      mx = fmaxf(mx, dx * dx + dy * dy + dz * dz);
    }
    for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    rebuild = mx > half_skin * half_skin;
  }
  if (lane == 0) {
    sys[s].rebuild = rebuild;
    if (rebuild && d.n > 0) atomicAdd(stats, 1);
  }
}

void launch_skin_check(const float *coords, SysDesc *sys, Live n_sys, const AtomState *state,
                       float half_skin, int *stats, hipStream_t st) {
  if (n_sys.v <= 0) return;
  k_skin_check<<<n_sys.v, kWave, 0, st>>>(coords, sys, n_sys, state, half_skin, stats);
}

// -------------------------------------------------------------- cell grids
// One wave per system.  Periodic: the host already set nc/edge.  Non-periodic:
// cells of edge >= rc_list over the bounding box, at most cell_cap cells.
// Also clears the system's cell counters.
__global__ void k_grid(SysDesc *__restrict__ sys, Live n_sys, const float4 *__restrict__ pos,
                       int *__restrict__ cell_count, float rc_list) {
  int s = blockIdx.x;
  if (s >= n_sys.get()) return;
  int lane = threadIdx.x;
  SysDesc d = sys[s];
  if (!d.periodic) {
    float mn[3] = {3.4e38f, 3.4e38f, 3.4e38f}, mx[3] = {-3.4e38f, -3.4e38f, -3.4e38f};
    for (int a = lane; a < d.n; a += kWave) {
      float4 p = pos[d.atom_off + a];
      mn[0] = fminf(mn[0], p.x); mx[0] = fmaxf(mx[0], p.x);
      mn[1] = fminf(mn[1], p.y); mx[1] = fmaxf(mx[1], p.y);
      mn[2] = fminf(mn[2], p.z); mx[2] = fmaxf(mx[2], p.z);
    }
    for (int off = 32; off >= 1; off >>= 1)
      for (int k = 0; k < 3; ++k) {
        mn[k] = fminf(mn[k], __shfl_xor(mn[k], off));
        mx[k] = fmaxf(mx[k], __shfl_xor(mx[k], off));
      }
    if (lane == 0) {
      const float rc = rc_list * (1.0f + 1e-5f);
      int nc[3];
      float ext[3];
      for (int k = 0; k < 3; ++k) {
        if (d.n == 0) { mn[k] = 0.f; mx[k] = 0.f; }
        ext[k] = fmaxf(mx[k] - mn[k], 0.f);
        nc[k] = max(1, (int)floorf(ext[k] / rc));
        nc[k] = min(nc[k], 1024);
      }
      // keep the product within the reserved cells: widen the largest axis' cells
      while ((long long)nc[0] * nc[1] * nc[2] > d.cell_cap) {
        int k = (nc[0] >= nc[1] && nc[0] >= nc[2]) ? 0 : (nc[1] >= nc[2] ? 1 : 2);
        nc[k] = max(1, nc[k] - 1);
      }
      for (int k = 0; k < 3; ++k) {
        d.origin[k] = mn[k];
        d.nc[k] = nc[k];
        d.edge[k] = nc[k] > 1 ? ext[k] / nc[k] : fmaxf(ext[k], rc);
        // guard the edge so floor((x - origin) / edge) of the max lands in-grid
        d.edge[k] = fmaxf(d.edge[k], rc);
      }
      sys[s] = d;
    }
  }
  for (int c = lane; c < d.cell_cap; c += kWave) cell_count[d.cell_off + c] = 0;
}

void launch_grid(SysDesc *sys, Live n_sys, const float4 *pos, int *cell_count, float rc_list,
                 hipStream_t st) {
  if (n_sys.v <= 0) return;
  k_grid<<<n_sys.v, kWave, 0, st>>>(sys, n_sys, pos, cell_count, rc_list);
}

__device__ inline int cell_coord(float x, float o, float e, int nc) {
  int c = (int)floorf((x - o) / e);
  return min(max(c, 0), nc - 1);
}

__global__ void k_cell_count(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
                             const SysDesc *__restrict__ sys, Live N, int *__restrict__ cell_count,
                             int *__restrict__ atom_cell, int *__restrict__ atom_slot) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N.get()) return;
  const SysDesc &d = sys[sys_of[i]];
  float4 p = pos[i];
  int cx = cell_coord(p.x, d.origin[0], d.edge[0], d.nc[0]);
  int cy = cell_coord(p.y, d.origin[1], d.edge[1], d.nc[1]);
  int cz = cell_coord(p.z, d.origin[2], d.edge[2], d.nc[2]);
  int c = d.cell_off + (cx * d.nc[1] + cy) * d.nc[2] + cz;
  atom_cell[i] = c;
  atom_slot[i] = atomicAdd(&cell_count[c], 1);
}

void launch_cell_count(const float4 *pos, const int *sys_of, const SysDesc *sys, Live N,
                       int *cell_count, int *atom_cell, int *atom_slot, hipStream_t st) {
  if (N.v <= 0) return;
  k_cell_count<<<(N.v + 255) / 256, 256, 0, st>>>(pos, sys_of, sys, N, cell_count, atom_cell,
                                                atom_slot);
}

// Exclusive prefix sum, out[0..n]: one workgroup of 1024 threads walks the
// array in coalesced 1024-element steps, carrying the running total.
__global__ void __launch_bounds__(1024) k_scan(const int *__restrict__ in, int *__restrict__ out,
                                               Live n_) {
  const int n = n_.get();
  __shared__ int wsum[1024 / kWave];
  __shared__ int carry_s;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int v = base + t < n ? in[base + t] : 0;
    int x = v;
    for (int off = 1; off < kWave; off <<= 1) {
      int y = __shfl_up(x, off);
      if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int before = carry_s;
    for (int q = 0; q < w; ++q) before += wsum[q];
    if (base + t < n) out[base + t] = before + x - v;
    __syncthreads();
    if (t == 1023) carry_s = before + x;
    __syncthreads();
  }
  if (t == 0) out[n] = carry_s;
}

void launch_scan(const int *in, int *out, Live n, hipStream_t st) {
  k_scan<<<1, 1024, 0, st>>>(in, out, n);
}

__global__ void k_cell_scatter(const int *__restrict__ atom_cell, const int *__restrict__ atom_slot,
                               const int *__restrict__ cell_start, Live N,
                               int *__restrict__ cell_atoms) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N.get()) return;
  cell_atoms[cell_start[atom_cell[i]] + atom_slot[i]] = i;
}

void launch_cell_scatter(const int *atom_cell, const int *atom_slot, const int *cell_start, Live N,
                         int *cell_atoms, hipStream_t st) {
  if (N.v <= 0) return;
  k_cell_scatter<<<(N.v + 255) / 256, 256, 0, st>>>(atom_cell, atom_slot, cell_start, N,
                                                  cell_atoms);
}

// Sorts each cell's atoms by index so neighbour lists (and every sum over
// them) come out in the same order on every call.  One workgroup per cell,
// rank sort in LDS; cells above kSortMax atoms keep their arrival order.
constexpr int kSortMax = 2048;

__global__ void __launch_bounds__(256) k_cell_sort(const int *__restrict__ cell_start, Live n_cells,
                                                   int *__restrict__ cell_atoms) {
  __shared__ int buf[kSortMax];
  const int c = blockIdx.x;
  if (c >= n_cells.get()) return;
  const int b = cell_start[c], n = cell_start[c + 1] - b;
  if (n <= 1 || n > kSortMax) return;
  for (int k = threadIdx.x; k < n; k += blockDim.x) buf[k] = cell_atoms[b + k];
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int v = buf[k];
    int rank = 0;
    for (int q = 0; q < n; ++q) rank += buf[q] < v;
    cell_atoms[b + rank] = v;
  }
}

void launch_cell_sort(const int *cell_start, Live n_cells, int *cell_atoms, hipStream_t st) {
  if (n_cells.v <= 0) return;
  k_cell_sort<<<n_cells.v, 256, 0, st>>>(cell_start, n_cells, cell_atoms);
}

// ----------------------------------------------------------- neighbour list
// One wave per atom: walk the stencil of cells around the atom's cell (every
// periodic image through the wrap of the cell index), the lanes splitting each
// cell's atoms, and keep each (j, image) with |d| < rc_list except the atom
// itself in the home image.  Entries are appended in cell order and, within a
// cell, in sorted atom order (ballot prefix), so the list is deterministic.
__device__ inline void wrap_cell(int u, int nc, bool periodic, int &w, int &shift, bool &ok) {
  if (periodic) {
    shift = u >= 0 ? u / nc : -((-u + nc - 1) / nc);
    w = u - shift * nc;
    ok = true;
  } else {
    ok = u >= 0 && u < nc;
    w = u;
    shift = 0;
  }
}

__global__ void __launch_bounds__(256)
k_nbr_build(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
            const SysDesc *__restrict__ sys, const int *__restrict__ cell_start,
            const int *__restrict__ cell_atoms, Live N, float rc_list, int cap,
            int2 *__restrict__ nbr, int *__restrict__ nbr_cnt, int *__restrict__ status) {
  const int lane = threadIdx.x % kWave;
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= N.get()) return;
  const SysDesc d = sys[sys_of[i]];
  if (!d.rebuild) return;
  const float4 p = pos[i];
  const float rc2 = rc_list * rc_list;
  int c[3], k[3];
  const float pc[3] = {p.x, p.y, p.z};
  for (int a = 0; a < 3; ++a) {
    c[a] = cell_coord(pc[a], d.origin[a], d.edge[a], d.nc[a]);
    k[a] = d.periodic ? (int)ceilf(rc_list / d.edge[a]) : 1;
  }
  int cnt = 0;
  int2 *out = nbr + nbr_row(d, i, cap);
  for (int ox = -k[0]; ox <= k[0]; ++ox) {
    int wx, sx; bool okx;
    wrap_cell(c[0] + ox, d.nc[0], d.periodic, wx, sx, okx);
    if (!okx) continue;
    for (int oy = -k[1]; oy <= k[1]; ++oy) {
      int wy, sy; bool oky;
      wrap_cell(c[1] + oy, d.nc[1], d.periodic, wy, sy, oky);
      if (!oky) continue;
      for (int oz = -k[2]; oz <= k[2]; ++oz) {
        int wz, sz; bool okz;
        wrap_cell(c[2] + oz, d.nc[2], d.periodic, wz, sz, okz);
        if (!okz) continue;
        const float shx = sx * d.L[0], shy = sy * d.L[1], shz = sz * d.L[2];
        const bool home = (sx | sy | sz) == 0;
        const int code = pack_image(sx, sy, sz);
        const int cell = d.cell_off + (wx * d.nc[1] + wy) * d.nc[2] + wz;
        const int qb = cell_start[cell], qe = cell_start[cell + 1];
        for (int base = qb; base < qe; base += kWave) {
          const int q = base + lane;
          bool inside = false;
          int j = 0;
          if (q < qe) {
            j = cell_atoms[q];
            const float4 pj = pos[j];
            const float dx = (pj.x - p.x) + shx, dy = (pj.y - p.y) + shy, dz = (pj.z - p.z) + shz;
            inside = dx * dx + dy * dy + dz * dz < rc2 && !(home && j == i);
          }
          const unsigned long long m = __ballot(inside);
          const int at = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
          if (inside && at < cap) out[at] = make_int2(j - d.atom_off, code);
          cnt += __popcll(m);
        }
      }
    }
  }
  if (lane == 0) {
    nbr_cnt[d.state_off + (i - d.atom_off)] = cnt;
    if (cnt > cap) atomicOr(status, kStatOverflow);
    // most waves do not raise the maximum: read before the atomic
    if (cnt > __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(status + 1, cnt);
  }
}

// The same lists, built one cell per workgroup: the atoms of the cell's
// stencil of neighbour cells (with their lattice images) are staged in LDS,
// in chunks, once for all atoms of the cell, instead of every atom walking
// the stencil through global memory.  Candidates are taken in stencil order
// (x offset outermost) and cell order, and each atom's entries in candidate
// order, so a row is identical to k_nbr_build's; the distance test uses the
// same arithmetic, (r_j - r_i) + image * L.
constexpr int kCandChunk = 1024;  // candidates staged at a time
constexpr int kHomeChunk = 256;   // atoms of the home cell handled at a time

__global__ void __launch_bounds__(256)
k_nbr_cell(const float4 *__restrict__ pos, const SysDesc *__restrict__ sys, Live n_sys_,
           const int *__restrict__ cell_start, const int *__restrict__ cell_atoms, float rc_list,
           int cap, int2 *__restrict__ nbr, int *__restrict__ nbr_cnt, int *__restrict__ status) {
  __shared__ float4 cpos[kCandChunk];   // candidate r_j (w: j as int bits)
  __shared__ int ccode[kCandChunk];     // candidate image code
  __shared__ int st_cell[kWave], st_code[kWave], st_pre[kWave + 1];
  __shared__ float4 hpos[kHomeChunk];
  __shared__ int hidx[kHomeChunk], hcnt[kHomeChunk];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int cell = blockIdx.x;
  const int n_sys = n_sys_.get();
  // the system owning this cell: last s with cell_off <= cell (cells past the
  // last system's range leave below)
  int lo = 0, hi = n_sys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].cell_off <= cell) lo = mid; else hi = mid - 1;
  }
  const SysDesc &d = sys[lo];
  if (!d.rebuild || cell >= d.cell_off + d.cell_cap) return;
  const int hb = cell_start[cell], he = cell_start[cell + 1];
  if (hb >= he) return;
  const int local = cell - d.cell_off;
  const int hc[3] = {local / (d.nc[1] * d.nc[2]), (local / d.nc[2]) % d.nc[1], local % d.nc[2]};
  int k[3], n1[3];
  for (int a = 0; a < 3; ++a) {
    k[a] = d.periodic ? (int)ceilf(rc_list / d.edge[a]) : 1;
    n1[a] = 2 * k[a] + 1;
  }
  const int nst = n1[0] * n1[1] * n1[2];
  const float rc2 = rc_list * rc_list;
  const int home_code = pack_image(0, 0, 0);

  for (int hb0 = hb; hb0 < he; hb0 += kHomeChunk) {
    const int nh = min(kHomeChunk, he - hb0);
    for (int t = tid; t < nh; t += blockDim.x) {
      const int i = cell_atoms[hb0 + t];
      hidx[t] = i;
      hpos[t] = pos[i];
      hcnt[t] = 0;
    }
    for (int sc0 = 0; sc0 < nst; sc0 += kWave) {
      __syncthreads();
      if (wave == 0) {
        // stencil cells sc0 .. sc0 + 63: cell index, image and atom count
        const int e = sc0 + lane;
        int cnt = 0, cidx = 0, code = 0;
        if (e < nst) {
          const int o[3] = {e / (n1[1] * n1[2]) - k[0], (e / n1[2]) % n1[1] - k[1], e % n1[2] - k[2]};
          int w[3], sh[3];
          bool ok = true;
          for (int a = 0; a < 3; ++a) {
            bool oka;
            wrap_cell(hc[a] + o[a], d.nc[a], d.periodic, w[a], sh[a], oka);
            ok = ok && oka;
          }
          if (ok) {
            cidx = d.cell_off + (w[0] * d.nc[1] + w[1]) * d.nc[2] + w[2];
            code = pack_image(sh[0], sh[1], sh[2]);
            cnt = cell_start[cidx + 1] - cell_start[cidx];
          }
        }
        // inclusive scan over the wave
        int incl = cnt;
        for (int off = 1; off < kWave; off <<= 1) {
          const int v = __shfl_up(incl, off);
          if (lane >= off) incl += v;
        }
        st_cell[lane] = cidx;
        st_code[lane] = code;
        st_pre[lane + 1] = incl;
        if (lane == 0) st_pre[0] = 0;
      }
      __syncthreads();
      const int total = st_pre[kWave];
      for (int t0 = 0; t0 < total; t0 += kCandChunk) {
        const int nc = min(kCandChunk, total - t0);
        if (t0 > 0) __syncthreads();   // the previous chunk has been scanned
        for (int u = tid; u < nc; u += blockDim.x) {
          const int t = t0 + u;
          int a = 0, b = kWave - 1;    // stencil entry holding candidate t
          while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (st_pre[mid] <= t) a = mid; else b = mid - 1;
          }
          const int j = cell_atoms[cell_start[st_cell[a]] + (t - st_pre[a])];
          float4 pj = pos[j];
          pj.w = __int_as_float(j);
          cpos[u] = pj;
          ccode[u] = st_code[a];
        }
        __syncthreads();
        for (int h = wave; h < nh; h += blockDim.x / kWave) {
          const int i = hidx[h];
          const float4 p = hpos[h];
          int cnt = hcnt[h];
          int2 *out = nbr + nbr_row(d, i, cap);
          for (int b0 = 0; b0 < nc; b0 += kWave) {
            const int u = b0 + lane;
            bool inside = false;
            int j = 0, code = 0;
            if (u < nc) {
              const float4 pj = cpos[u];
              j = __float_as_int(pj.w);
              code = ccode[u];
              int ix, iy, iz;
              unpack_image(code, ix, iy, iz);
              const float dx = (pj.x - p.x) + (float)ix * d.L[0];
              const float dy = (pj.y - p.y) + (float)iy * d.L[1];
              const float dz = (pj.z - p.z) + (float)iz * d.L[2];
              inside = dx * dx + dy * dy + dz * dz < rc2 && !(code == home_code && j == i);
            }
            const unsigned long long m = __ballot(inside);
            const int at = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
            if (inside && at < cap) out[at] = make_int2(j - d.atom_off, code);
            cnt += __popcll(m);
          }
          if (lane == 0) hcnt[h] = cnt;
        }
      }
    }
    __syncthreads();
    for (int t = tid; t < nh; t += blockDim.x) {
      const int i = hidx[t], cnt = hcnt[t];
      nbr_cnt[d.state_off + (i - d.atom_off)] = cnt;
      if (cnt > cap) atomicOr(status, kStatOverflow);
      if (cnt > __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(status + 1, cnt);
    }
    __syncthreads();   // hidx / hcnt are reused by the next group of home atoms
  }
}

// Small non-periodic systems (every system of the call at most kSmallSystem
// atoms, no box): one wave per atom scans its whole system in j order, in
// place of the cell grid, its scan and sort and the stencil walk.  The
// distance test is the one the cell walk uses; rows list neighbours in
// increasing j.
__global__ void __launch_bounds__(256)
k_nbr_small(const float4 *__restrict__ pos, const int *__restrict__ sys_of,
            const SysDesc *__restrict__ sys, Live N, float rc_list, int cap,
            int2 *__restrict__ nbr, int *__restrict__ nbr_cnt, int *__restrict__ status) {
  const int lane = threadIdx.x % kWave;
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= N.get()) return;
  const SysDesc d = sys[sys_of[i]];
  if (!d.rebuild) return;
  const float4 p = pos[i];
  const float rc2 = rc_list * rc_list;
  const int code = pack_image(0, 0, 0);
  int cnt = 0;
  int2 *out = nbr + nbr_row(d, i, cap);
  for (int base = d.atom_off; base < d.atom_off + d.n; base += kWave) {
    const int j = base + lane;
    bool inside = false;
    if (j < d.atom_off + d.n && j != i) {
      const float4 pj = pos[j];
      const float dx = pj.x - p.x, dy = pj.y - p.y, dz = pj.z - p.z;
      inside = dx * dx + dy * dy + dz * dz < rc2;
    }
    const unsigned long long m = __ballot(inside);
    const int at = cnt + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
    if (inside && at < cap) out[at] = make_int2(j - d.atom_off, code);
    cnt += __popcll(m);
  }
  if (lane == 0) {
    nbr_cnt[d.state_off + (i - d.atom_off)] = cnt;
    if (cnt > cap) atomicOr(status, kStatOverflow);
    if (cnt > __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(status + 1, cnt);
  }
}

void launch_nbr_small(const float4 *pos, const int *sys_of, const SysDesc *sys, Live N, float rc_list,
                      int cap, int2 *nbr, int *nbr_cnt, int *status, hipStream_t st) {
  if (N.v <= 0) return;
  k_nbr_small<<<(N.v + 3) / 4, 256, 0, st>>>(pos, sys_of, sys, N, rc_list, cap, nbr, nbr_cnt, status);
}

void launch_nbr_build(const float4 *pos, const int *sys_of, const SysDesc *sys, Live n_sys, int n_cells,
                      const int *cell_start, const int *cell_atoms, Live N, float rc_list, int cap,
                      int2 *nbr, int *nbr_cnt, int *status, hipStream_t st) {
  if (N.v <= 0) return;
  // staging a cell's stencil pays off once cells hold several atoms (dense
  // boxes); sparse grids of small solutes are faster with a wave per atom
  // (decided on the launch sizes)
  if (n_cells > 0 && N.v >= 8 * (long long)n_cells) {
    k_nbr_cell<<<n_cells, 256, 0, st>>>(pos, sys, n_sys, cell_start, cell_atoms, rc_list, cap, nbr,
                                        nbr_cnt, status);
    return;
  }
  k_nbr_build<<<(N.v + 3) / 4, 256, 0, st>>>(pos, sys_of, sys, cell_start, cell_atoms, N, rc_list,
                                           cap, nbr, nbr_cnt, status);
}

// ----------------------------------------------------------- species buckets
// Stable counting sort of atoms by species into row ranges padded to the MLP
// row tile, so one dense-layer tile never mixes element networks
// (section "Neural Network Potentials": one network per element).
constexpr int kBucketBlock = 1024;

__global__ void __launch_bounds__(kBucketBlock)
k_species_count(const float4 *__restrict__ pos, const int *__restrict__ wave_atom, Live N_, int S,
                int *__restrict__ block_counts) {
  __shared__ int cnt[kMaxSpecies];
  const int N = N_.get();
  if (threadIdx.x < kMaxSpecies) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int w = blockIdx.x * kBucketBlock + threadIdx.x;
  if (w < N) {
    const int i = wave_atom ? wave_atom[w] : w;
    const int s = __float_as_int(pos[i].w);
    if (s >= 0) atomicAdd(&cnt[s], 1);   // slot -1: outside the caller's mask
  }
  __syncthreads();
  if (threadIdx.x < kMaxSpecies) block_counts[blockIdx.x * kMaxSpecies + threadIdx.x] = cnt[threadIdx.x];
}

// One workgroup: per-species exclusive scan over blocks, padded bucket
// offsets, and -1 in the padding rows.  Blocks are taken 256 at a time, a
// thread per block: the counts of all species load at once, wave scans by
// shuffles, and the four waves' totals combine through LDS.
__global__ void __launch_bounds__(256)
k_species_scan(int *__restrict__ block_counts, int n_blocks, int S, int *__restrict__ bucket_off,
               int *__restrict__ bucket_cnt, int *__restrict__ perm) {
  constexpr int kWaves = 256 / kWave;
  __shared__ int wsum[kWaves][kMaxSpecies];
  __shared__ int tot[kMaxSpecies];
  __shared__ int off[kMaxSpecies + 1];
  const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
  int run[kMaxSpecies];  // totals of the earlier chunks (the same in every thread)
#pragma unroll
  for (int s = 0; s < kMaxSpecies; ++s) run[s] = 0;
  for (int b0 = 0; b0 < n_blocks; b0 += 256) {
    const int b = b0 + t;
    const bool in = b < n_blocks;
    int ex[kMaxSpecies];
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      const int v = in && s < S ? block_counts[b * kMaxSpecies + s] : 0;
      int x = v;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
      }
      if (lane == kWave - 1) wsum[wv][s] = x;
      ex[s] = x - v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      int before = run[s], chunk = 0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) {
        before += q < wv ? wsum[q][s] : 0;
        chunk += wsum[q][s];
      }
      if (in && s < S) block_counts[b * kMaxSpecies + s] = before + ex[s];
      run[s] += chunk;
    }
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (t < S) {
    int v = run[0];
#pragma unroll
    for (int s = 1; s < kMaxSpecies; ++s) v = t == s ? run[s] : v;
    tot[t] = v;
  }
  __syncthreads();
  if (t == 0) {
    int o = 0;
    for (int s = 0; s < S; ++s) {
      off[s] = o;
      o += (tot[s] + kTileM - 1) / kTileM * kTileM;
    }
    off[S] = o;
    for (int s = 0; s <= S; ++s) bucket_off[s] = off[s];
    for (int s = 0; s < S; ++s) bucket_cnt[s] = tot[s];
  }
  __syncthreads();
  for (int s = 0; s < S; ++s)
    for (int r = off[s] + tot[s] + t; r < off[s + 1]; r += blockDim.x) perm[r] = -1;
}

__global__ void __launch_bounds__(kBucketBlock)
k_species_scatter(const float4 *__restrict__ pos, const int *__restrict__ wave_atom, Live N_,
                  const int *__restrict__ block_base, const int *__restrict__ bucket_off, int *__restrict__ perm,
                  int *__restrict__ row_of_atom) {
  const int N = N_.get();
  __shared__ int wave_cnt[kBucketBlock / kWave][kMaxSpecies];
  const int t = blockIdx.x * kBucketBlock + threadIdx.x;
  const int i = wave_atom && t < N ? wave_atom[t] : t;
  int w = threadIdx.x / kWave;
  int s = t < N ? __float_as_int(pos[i].w) : -1;
  int rank_in_wave = 0;
  for (int q = 0; q < kMaxSpecies; ++q) {
    unsigned long long m = __ballot(s == q);
    if (s == q)
      rank_in_wave = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
    if ((threadIdx.x & (kWave - 1)) == 0) wave_cnt[w][q] = __popcll(m);
  }
  __syncthreads();
  if (s >= 0) {
    int before = 0;
    for (int v = 0; v < w; ++v) before += wave_cnt[v][s];
    int row = bucket_off[s] + block_base[blockIdx.x * kMaxSpecies + s] + before + rank_in_wave;
    perm[row] = i;
    row_of_atom[i] = row;
  } else if (t < N) {
    row_of_atom[i] = -1;   // no network row: the AEV kernels skip the atom
  }
}

// Calls of at most kPlaceBlocks bucketing blocks skip the scan kernel: each
// scatter workgroup sums the per-block counts itself (one count per thread,
// LDS atomics) into the species totals and its own offsets, and workgroup 0
// publishes the bucket offsets and clears the padding rows.
constexpr int kPlaceBlocks = 128;

__global__ void __launch_bounds__(kBucketBlock)
k_species_place(const float4 *__restrict__ pos, const int *__restrict__ wave_atom, Live N_,
                const int *__restrict__ block_counts, int n_blocks, int S, int *__restrict__ bucket_off,
                int *__restrict__ bucket_cnt, int *__restrict__ perm, int *__restrict__ row_of_atom) {
  const int N = N_.get();
  __shared__ int tot[kMaxSpecies], before_blk[kMaxSpecies], off[kMaxSpecies + 1];
  __shared__ int wave_cnt[kBucketBlock / kWave][kMaxSpecies];
  if (threadIdx.x < kMaxSpecies) {
    tot[threadIdx.x] = 0;
    before_blk[threadIdx.x] = 0;
  }
  __syncthreads();
  // the counts of every block: species totals and this block's base
  for (int k = threadIdx.x; k < n_blocks * kMaxSpecies; k += blockDim.x) {
    const int b = k / kMaxSpecies, sp = k - b * kMaxSpecies;
    const int c = block_counts[k];
    if (c) {
      atomicAdd(&tot[sp], c);
      if (b < (int)blockIdx.x) atomicAdd(&before_blk[sp], c);
    }
  }
  const int t = blockIdx.x * kBucketBlock + threadIdx.x;
  const int i = wave_atom && t < N ? wave_atom[t] : t;
  const int w = threadIdx.x / kWave;
  const int s = t < N ? __float_as_int(pos[i].w) : -1;
  int rank_in_wave = 0;
  for (int q = 0; q < kMaxSpecies; ++q) {
    unsigned long long m = __ballot(s == q);
    if (s == q)
      rank_in_wave = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
    if ((threadIdx.x & (kWave - 1)) == 0) wave_cnt[w][q] = __popcll(m);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int o = 0;
    for (int q = 0; q < S; ++q) {
      off[q] = o;
      o += (tot[q] + kTileM - 1) / kTileM * kTileM;
    }
    off[S] = o;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (threadIdx.x <= S) bucket_off[threadIdx.x] = off[threadIdx.x];
    if (threadIdx.x < S) bucket_cnt[threadIdx.x] = tot[threadIdx.x];
    for (int q = 0; q < S; ++q)
      for (int r = off[q] + tot[q] + threadIdx.x; r < off[q + 1]; r += blockDim.x) perm[r] = -1;
  }
  if (s >= 0) {
    int before = 0;
    for (int v = 0; v < w; ++v) before += wave_cnt[v][s];
    const int row = off[s] + before_blk[s] + before + rank_in_wave;
    perm[row] = i;
    row_of_atom[i] = row;
  } else if (t < N) {
    row_of_atom[i] = -1;   // no network row: the AEV kernels skip the atom
  }
}

void launch_species_bucket(const float4 *pos, const int *wave_atom, Live N, int S, int *block_counts,
                           int n_blocks, int *bucket_off, int *bucket_cnt, int *perm, int *row_of_atom,
                           int rows_cap, hipStream_t st) {
  (void)rows_cap;
  // blocks past the live atoms (launches sized for more) count zeros
  if (N.v > 0) k_species_count<<<n_blocks, kBucketBlock, 0, st>>>(pos, wave_atom, N, S, block_counts);
  if (N.v > 0 && n_blocks <= kPlaceBlocks) {
    k_species_place<<<n_blocks, kBucketBlock, 0, st>>>(pos, wave_atom, N, block_counts, n_blocks, S, bucket_off,
                                                       bucket_cnt, perm, row_of_atom);
    return;
  }
  k_species_scan<<<1, 256, 0, st>>>(block_counts, N.v > 0 ? n_blocks : 0, S, bucket_off,
                                    bucket_cnt, perm);
  if (N.v > 0)
    k_species_scatter<<<n_blocks, kBucketBlock, 0, st>>>(pos, wave_atom, N, block_counts, bucket_off, perm,
                                                         row_of_atom);
}

// ----------------------------------------------------------------- utilities
// Copies bytes (rounded up to 16) from host memory mapped for the device
// (coherent pinned staging) into device memory with a kernel on the
// stream's own queue: the per-call descriptors reach the device without a
// copy-engine hand-off (about 25 us of latency per call).
__global__ void __launch_bounds__(256) k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                size_t n16) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += (size_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

void launch_copy_from_host(const void *src, void *dst, size_t bytes, hipStream_t st) {
  const size_t n16 = (bytes + 15) / 16;
  if (n16 == 0) return;
  const size_t blocks = (n16 + 255) / 256;
  k_copy16<<<(unsigned)(blocks < 256 ? blocks : 256), 256, 0, st>>>((const uint4 *)src, (uint4 *)dst, n16);
}

__global__ void k_fill(float *__restrict__ p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void launch_fill(float *p, size_t n, float v, hipStream_t st) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
}

__global__ void k_fill_i32(int *__restrict__ p, size_t n, int v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

void launch_fill_i32(int *p, size_t n, int v, hipStream_t st) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_fill_i32<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
}

__global__ void k_gather_rows(const float *__restrict__ src, int ld, const int *__restrict__ row_of_atom,
                              int N, int D, float *__restrict__ dst) {
  int i = blockIdx.x;
  if (i >= N) return;
  const int r = row_of_atom[i];
  float *d = dst + (size_t)i * D;
  if (r < 0) {   // no network row: no features
    for (int k = threadIdx.x; k < D; k += blockDim.x) d[k] = 0.f;
    return;
  }
  const float *s = src + (size_t)r * ld;
  for (int k = threadIdx.x; k < D; k += blockDim.x) d[k] = s[k];
}

void launch_gather_rows(const float *src, int ld, const int *row_of_atom, int N, int D, float *dst,
                        hipStream_t st) {
  if (N <= 0) return;
  k_gather_rows<<<N, 256, 0, st>>>(src, ld, row_of_atom, N, D, dst);
}

__global__ void k_export_nbr(const int2 *__restrict__ nbr, const int *__restrict__ nbr_cnt, int cap,
                             const SysDesc *__restrict__ sys, const int *__restrict__ sys_of, int N,
                             int *__restrict__ counts, int *__restrict__ entries, int out_cap) {
  int i = blockIdx.x;
  if (i >= N) return;
  const SysDesc d = sys[sys_of[i]];
  int n = nbr_cnt[d.state_off + (i - d.atom_off)];
  if (threadIdx.x == 0) counts[i] = n;
  int w = min(min(n, cap), out_cap);
  const int2 *row = nbr + nbr_row(d, i, cap);
  for (int e = threadIdx.x; e < w; e += blockDim.x) {
    int2 v = row[e];
    int x, y, z;
    unpack_image(v.y, x, y, z);
    int *o = entries + ((size_t)i * out_cap + e) * 4;
    o[0] = v.x + d.atom_off; o[1] = x; o[2] = y; o[3] = z;
  }
}

void launch_export_nbr(const int2 *nbr, const int *nbr_cnt, int cap, const SysDesc *sys,
                       const int *sys_of, int N, int *counts, int *entries, int out_cap,
                       hipStream_t st) {
  if (N <= 0) return;
  k_export_nbr<<<N, 64, 0, st>>>(nbr, nbr_cnt, cap, sys, sys_of, N, counts, entries, out_cap);
}

__global__ void k_f32_to_bf16(const float *__restrict__ src, uint16_t *__restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // round to nearest even
  unsigned u = __float_as_uint(src[i]);
  unsigned lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  dst[i] = (uint16_t)(u >> 16);
}

void launch_f32_to_bf16(const float *src, uint16_t *dst, size_t n, hipStream_t st) {
  if (n == 0) return;
  k_f32_to_bf16<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, dst, n);
}


// ---- caller pair lists (the pair-list entry point)
//
// A host program that keeps its own neighbour list (the paper's platform
// hands the network positions and a pair list) passes it as pairs (i, j)
// with integer lattice shifts n: r_j + n * L is a neighbour of i.  A half
// list names each unordered pair once and both directions are added; a
// full list names each direction.  Pairs with an atom outside the mask, or
// at a distance at or beyond the cutoff, are dropped here (the AEV kernels
// apply the cutoff again with their own arithmetic).
__global__ void k_pairs_append(const int *__restrict__ pairs, const int *__restrict__ shifts,
                               long long n_pairs, int half, const unsigned char *__restrict__ mask,
                               const float4 *__restrict__ pos, int N, float L0, float L1, float L2,
                               float rc2, int cap, int2 *__restrict__ nbr, int *__restrict__ nbr_cnt,
                               int *__restrict__ status) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x % kWave;
  bool keep = false;
  int i = 0, j = 0, nx = 0, ny = 0, nz = 0;
  if (p < n_pairs) {
    i = pairs[2 * p];
    j = pairs[2 * p + 1];
    if (shifts) { nx = shifts[3 * p]; ny = shifts[3 * p + 1]; nz = shifts[3 * p + 2]; }
    const bool bad = (unsigned)i >= (unsigned)N || (unsigned)j >= (unsigned)N ||
                     (i == j && nx == 0 && ny == 0 && nz == 0) ||
                     nx < -511 || nx > 511 || ny < -511 || ny > 511 || nz < -511 || nz > 511;
    if (bad) {
      atomicOr(status, kStatBadPairs);
    } else if (!mask || (mask[i] && mask[j])) {
      const float4 pi = pos[i], pj = pos[j];
      const float dx = (pj.x - pi.x) + (float)nx * L0;
      const float dy = (pj.y - pi.y) + (float)ny * L1;
      const float dz = (pj.z - pi.z) + (float)nz * L2;
      keep = dx * dx + dy * dy + dz * dz < rc2;
    }
  }
  // slots in row i.  Lists usually come grouped by i, so many lanes of a
  // wave add to one counter: lanes sharing the first remaining lane's i take
  // their slots with one atomic; once such groups become small, the rest
  // add one by one.
  unsigned long long act = __ballot(keep);
  int a = -1;
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int key = __shfl(i, leader);
    const unsigned long long grp = __ballot(keep && i == key) & act;
    const int n = __popcll(grp);
    if (n < 4) break;
    int base = 0;
    if (lane == leader) base = atomicAdd(&nbr_cnt[key], n);
    base = __shfl(base, leader);
    if ((grp >> lane) & 1ull)
      a = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(grp >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)grp, 0));
    act &= ~grp;
  }
  if ((act >> lane) & 1ull) a = atomicAdd(&nbr_cnt[i], 1);
  if (!keep) return;
  if (a < cap) nbr[(size_t)i * cap + a] = make_int2(j, pack_image(nx, ny, nz));
  if (half) {
    const int b = atomicAdd(&nbr_cnt[j], 1);
    if (b < cap) nbr[(size_t)j * cap + b] = make_int2(i, pack_image(-nx, -ny, -nz));
  }
}

// One wave per atom: each row, filled in arbitrary (atomic) order, is put in
// (j, image) order so that results do not depend on it; a repeated entry
// (a pair listed twice) raises kStatBadPairs; a row past the capacity raises
// kStatOverflow and the largest count is kept for the caller's retry.
__global__ void __launch_bounds__(256)
k_pairs_rows(int N, int cap, int2 *__restrict__ nbr, const int *__restrict__ nbr_cnt,
             int *__restrict__ status) {
  extern __shared__ unsigned long long row_keys[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int i = blockIdx.x * (blockDim.x / kWave) + wave;
  if (i >= N) return;
  unsigned long long *K = row_keys + (size_t)wave * cap;
  const int cnt = nbr_cnt[i];
  if (lane == 0 && cnt > cap) {
    atomicOr(status, kStatOverflow);
    if (cnt > __hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(status + 1, cnt);
  }
  const int n = min(cnt, cap);
  int2 *row = nbr + (size_t)i * cap;
  for (int e = lane; e < n; e += kWave) {
    const int2 v = row[e];
    K[e] = ((unsigned long long)(unsigned)v.x << 32) | (unsigned)v.y;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  bool dup = false;
  for (int e = lane; e < n; e += kWave) {
    const unsigned long long k = K[e];
    int r = 0;
    for (int t = 0; t < n; ++t) {
      const unsigned long long kt = K[t];
      r += kt < k ? 1 : 0;
      dup |= kt == k && t != e;
    }
    row[r] = make_int2((int)(k >> 32), (int)(unsigned)k);
  }
  if (__ballot(dup) != 0ull && lane == 0) atomicOr(status, kStatBadPairs);
}

void launch_pairs_to_rows(const int *pairs, const int *shifts, long long n_pairs, int half,
                          const unsigned char *mask, const float4 *pos, int N, const float L[3],
                          float rc, int cap, int2 *nbr, int *nbr_cnt, int *status, hipStream_t st) {
  if (N <= 0) return;
  launch_fill_i32(nbr_cnt, (size_t)N, 0, st);
  if (n_pairs > 0) {
    const float rc2 = rc * rc * (1.0f + 1e-5f);
    k_pairs_append<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(
        pairs, shifts, n_pairs, half, mask, pos, N, L[0], L[1], L[2], rc2, cap, nbr, nbr_cnt, status);
  }
  k_pairs_rows<<<(N + 3) / 4, 256, (size_t)4 * cap * sizeof(unsigned long long), st>>>(N, cap, nbr, nbr_cnt,
                                                                                      status);
}

}  // namespace nnp
