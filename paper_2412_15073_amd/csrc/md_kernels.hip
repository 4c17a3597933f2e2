// md_kernels.hip — HIP kernels of libjumpmd for gfx950 (CDNA4, wave64), apart
// from the jump chains (md_chain.hip).
//
//  k_local     the non-chain part of a step program, one atom per lane: B / A
//              / O updates (Sec. 2.3) and the displacement check; positions
//              are double-buffered (read one copy, write the other).
//  k_cell_*    counting sort of atoms into per-replica cells.
//  k_build     neighbour rows, one wavefront per atom: the cell stencil
//              passes a float distance filter, the survivors the exact FP64
//              tests; ballot compaction into LDS, bitonic sort, segment starts
//              by binary search.
//  k_force     non-bonded pair forces over fixed-capacity rows, SG lanes per
//              atom, shuffle reduction (with the bonded forces appended when
//              they fit the same round).
//  k_bonded    bonds and angles, per atom over its incident terms.
//  Ewald reciprocal space: the plain structure-factor sum (k_sfac,
//              k_recip_force) and particle-mesh Ewald (spreading, transforms
//              and influence function in LDS, gather).
//  observables: kinetic energy, pair energies, pair histograms.
#include <algorithm>
#include <mutex>

#include "md_device.h"
#include "md_internal.h"

// -------------------------------------------------------------- k_local
// One lane per atom: B / A / O updates and the displacement check of a step
// program without jump chains. Positions are double-buffered (read Xs, write Xd).
__global__ __launch_bounds__(256) void k_local(MDView V, MDProg P, const double4 *__restrict__ Xs,
                                                double4 *__restrict__ Xd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // displacement maximum: per-block LDS max, one global atomic per block
  __shared__ unsigned long long s_d2;
  const int rp_blk = V.rep[min(V.n - 1, (int)(blockIdx.x * blockDim.x))];
  if (threadIdx.x == 0) s_d2 = 0ull;
  __syncthreads();
  if (i < V.nrep && P.reset_slot >= 0) V.rep_maxd2[P.reset_slot * V.nrep + i] = 0ull;
  const bool valid = i < V.n;
  const int ii = valid ? i : V.n - 1;
  double4 xi = Xs[ii];
  const double4 vv = V.v[ii];
  double vx = vv.x, vy = vv.y, vz = vv.z;
  const double me = vv.w;
  const int rp = V.rep[ii];
  const double4 fn = V.fnb[ii], fb = V.fb[ii];
  const int64_t sbase = P.dev_step ? (int64_t)V.ctl->step_base : 0;
  double disp2 = 0.0;
  bool has_disp = false;
  for (int o = 0; o < P.nops; ++o) {
    MDOp op = P.ops[o];
    op.step += sbase;
    switch (op.kind) {
      case OP_B: {
        const double3 f = kick_force(V, op.flags, ii, fn, fb);
        vx += op.h * f.x / me; vy += op.h * f.y / me; vz += op.h * f.z / me;
      } break;
      case OP_A:
        xi.x += op.h * vx; xi.y += op.h * vy; xi.z += op.h * vz;
        break;
      case OP_O: {
        const uint64_t tag = (uint64_t)OP_PHASE_O | ((uint64_t)(uint32_t)op.substep << 8);
        Uni4 u = draw4(V.seed, (uint64_t)rp, op.step, V.loc[ii], tag, 0);
        const double r1 = sqrt(-2.0 * log(u.u[0])), r2 = sqrt(-2.0 * log(u.u[2]));
        const double gx = r1 * cos(2.0 * MD_PI * u.u[1]);
        const double gy = r1 * sin(2.0 * MD_PI * u.u[1]);
        const double gz = r2 * cos(2.0 * MD_PI * u.u[3]);
        const double sd = sqrt(V.kT / me);
        vx = op.c1 * vx + op.c2 * sd * gx;
        vy = op.c1 * vy + op.c2 * sd * gy;
        vz = op.c1 * vz + op.c2 * sd * gz;
        if (op.rstep >= 0 && valid && i < V.ntrace)
          V.trace[(size_t)(op.rstep % V.trace_cap) * V.ntrace + i] = make_double4(vx, vy, vz, 0.0);
      } break;
      case OP_DISP: {
        const double4 xr = V.xref[ii];
        const double dx = xi.x - xr.x, dy = xi.y - xr.y, dz = xi.z - xr.z;
        disp2 = valid ? dx * dx + dy * dy + dz * dz : 0.0;
        has_disp = true;
      } break;
    }
  }
  if (valid) {
    if (!(isfinite(vx) && isfinite(vy) && isfinite(vz))) atomicAdd(&V.ctl->nonfinite, 1ull);
    V.v[i] = make_double4(vx, vy, vz, me);
    if (Xd) Xd[i] = xi;
  }
  if (has_disp) {
    const unsigned long long d = (unsigned long long)__double_as_longlong(disp2);
    if (!valid || rp == rp_blk) atomicMax(&s_d2, d);
    else atomicMax(&V.rep_maxd2[P.disp_slot * V.nrep + rp], d);   // block straddles replicas
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&V.rep_maxd2[P.disp_slot * V.nrep + rp_blk], s_d2);
  }
}

// ------------------------------------------------------------ rebuild
// Every replica decides on its own: rebuild when its maximum displacement
// since its last build exceeds skin/2 (or when forced).
__device__ __forceinline__ bool rebuild_now(const MDView &V, int slot, int forced, int autob, double thr2, int r) {
  if (forced) return true;
  if (!autob) return false;
  double m = __longlong_as_double((long long)V.rep_maxd2[slot * V.nrep + r]);
  return m > thr2;
}

__global__ void k_cell_count(MDView V, const double4 *__restrict__ X, int slot, int forced, int autob,
                             double thr2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const int r = V.rep[i];
  const bool rb = rebuild_now(V, slot, forced, autob, thr2, r);
  if (i == V.rep_off[r] && !forced && !autob) {
    double m = __longlong_as_double((long long)V.rep_maxd2[slot * V.nrep + r]);
    if (m > thr2) atomicAdd(&V.ctl->n_list_err, 1ull);
  }
  if (!rb) return;
  double4 x = X[i];
  int c3[3];
  const double xs[3] = {x.x, x.y, x.z};
  for (int d = 0; d < 3; ++d) {
    double L = V.box[3 * r + d];
    double w = xs[d] - L * floor(xs[d] / L);
    int nd = V.rep_cdim[3 * r + d];
    int c = (int)(w / L * (double)nd);
    c3[d] = c < 0 ? 0 : (c >= nd ? nd - 1 : c);
  }
  int c = V.rep_cell_off[r] + (c3[2] * V.rep_cdim[3 * r + 1] + c3[1]) * V.rep_cdim[3 * r] + c3[0];
  V.atom_cell[i] = c;
  V.atom_slot[i] = atomicAdd(&V.cell_count[c], 1);
  V.xref[i] = x;
}

// One block per replica: exclusive scan of the replica's cell counts into
// cell starts offset to the replica's own atom range, counts cleared for the
// next binning. Replicas that do not rebuild leave their cells untouched.
// Tiles of 256 cells: coalesced loads, a shuffle scan per wave, the four wave
// totals through LDS, and a running carry across tiles.
__global__ __launch_bounds__(256) void k_cell_scan(MDView V, int slot, int forced, int autob, double thr2,
                                                   int count) {
  __shared__ int wsum[4];
  const int r = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (r == 0 && t == 0) V.cell_start[V.ncell_total] = V.n;
  if (!rebuild_now(V, slot, forced, autob, thr2, r)) return;   // uniform over the block
  const int c0 = V.rep_cell_off[r], c1 = V.rep_cell_off[r + 1];
  int carry = V.rep_off[r];
  for (int base = c0; base < c1; base += 256) {
    const int c = base + t;
    const int v = c < c1 ? V.cell_count[c] : 0;
    int x = v;   // inclusive scan within the wave
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = carry;
    for (int q = 0; q < w; ++q) before += wsum[q];
    const int tile = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (c < c1) {
      V.cell_start[c] = before + x - v;
      V.cell_count[c] = 0;
    }
    carry += tile;
    __syncthreads();   // wsum is rewritten by the next tile
  }
  if (count && t == 0) atomicAdd(&V.ctl->n_rebuilds, 1ull);
}

__global__ void k_cell_scatter(MDView V, int slot, int forced, int autob, double thr2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n || !rebuild_now(V, slot, forced, autob, thr2, V.rep[i])) return;
  const int p = V.cell_start[V.atom_cell[i]] + V.atom_slot[i];
  V.cell_atoms[p] = i;
  const double4 x = V.xref[i];
  V.xcell[p] = x;   // positions in cell order: contiguous reads in the row builder
  const int r = V.rep[i];
  const double Lx = V.box[3 * r], Ly = V.box[3 * r + 1], Lz = V.box[3 * r + 2];
  V.xcellf[p] = make_float4((float)(x.x - Lx * floor(x.x / Lx)), (float)(x.y - Ly * floor(x.y / Ly)),
                            (float)(x.z - Lz * floor(x.z / Lz)), 0.0f);
}

__device__ __forceinline__ void bitonic_sort_lds(unsigned *keys, int m) {
  const int lane = threadIdx.x;
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = lane; t < (m >> 1); t += 64) {
        // j is a power of two: a = 2j floor(t / j) + t mod j
        const int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        const int b = a + j;
        const bool up = (a & k) == 0;
        const unsigned ka = keys[a], kb = keys[b];
        if ((ka > kb) == up) { keys[a] = kb; keys[b] = ka; }
      }
      __syncthreads();
    }
  }
}

// Bitonic sort of m = 64 K keys held in registers (element e = K lane + q):
// compare-exchange partners e ^ j are in the same lane for j < K (register
// swaps) and in lane ^ (j / K) otherwise (one cross-lane exchange per key).
// Ascending where (e & k) == 0 for the merge of size k.
template <int K>
__device__ __forceinline__ void bitonic_sort_regs(unsigned (&v)[K], int m) {
  const int lane = threadIdx.x;
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j >= K; j >>= 1) {
      const int lm = j / K;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const int e = lane * K + q;
        const unsigned o = (unsigned)__shfl_xor((int)v[q], lm, 64);
        const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
        v[q] = keep_min ? min(v[q], o) : max(v[q], o);
      }
    }
#pragma unroll
    for (int jj = K / 2; jj > 0; jj >>= 1) {
      if (jj < k) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
          if ((q & jj) == 0) {
            const int e = lane * K + q;
            const bool up = (e & k) == 0;
            const unsigned a = v[q], b = v[q + jj];
            if ((a > b) == up) { v[q] = b; v[q + jj] = a; }
          }
        }
      }
    }
  }
}

// Sort keys[0, n) of LDS in place (padding to a power of two m >= 64 with
// 0xffffffff); registers for m <= 1024, the LDS network above that.
__device__ __forceinline__ void sort_keys(unsigned *keys, int n) {
  const int lane = threadIdx.x;
  int m = 64;
  while (m < n) m <<= 1;
  if (m > 1024) {
    for (int e = n + lane; e < m; e += 64) keys[e] = 0xffffffffu;
    __syncthreads();
    bitonic_sort_lds(keys, m);
    return;
  }
  auto run = [&](auto kk) {
    constexpr int K = decltype(kk)::value;
    unsigned v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int e = lane * K + q;
      v[q] = e < n ? keys[e] : 0xffffffffu;
    }
    bitonic_sort_regs<K>(v, m);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int e = lane * K + q;
      if (e < n) keys[e] = v[q];
    }
    __syncthreads();
  };
  switch (m) {
    case 64: run(std::integral_constant<int, 1>()); break;
    case 128: run(std::integral_constant<int, 2>()); break;
    case 256: run(std::integral_constant<int, 4>()); break;
    case 512: run(std::integral_constant<int, 8>()); break;
    default: run(std::integral_constant<int, 16>()); break;
  }
}

// cells of one stencil dimension: offsets -2..2 when the replica has at least
// 5 cells along it (cell edge >= (r_c + skin)/2), otherwise every cell once
__device__ __forceinline__ void stencil_range(int c, int nd, int &lo, int &hi) {
  if (nd >= 5) { lo = c - 2; hi = c + 2; }
  else { lo = 0; hi = nd - 1; }
}

// One wavefront per atom: rows with want bits 1 = short (r < r_s + skin),
// 2 = full (r < r_c + skin), 4 = candidates (r_s - w - skin <= r < r_c + skin).
// Candidates are read from the cell-ordered copy of positions along
// contiguous x-runs of the 5x5x5 stencil, compacted into LDS with a ballot,
// sorted (32-bit keys: segment << 24 | j, or j) and written out.
__global__ __launch_bounds__(64) void k_build(MDView V, const double4 *__restrict__ X, int want, int slot,
                                              int forced, int autob, double thr2, int pc, int ps) {
  if (!rebuild_now(V, slot, forced, autob, thr2, V.rep[blockIdx.x])) return;
  extern __shared__ unsigned lds[];
  const int i = blockIdx.x, lane = threadIdx.x;
  const double4 xi = X[i];
  const int r = V.rep[i];
  const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
  const bool img = rep_images(L, V.rout);
  // candidate or full keys [pc], and the pass-1 queue of stencil atoms, which
  // also holds the atom itself, its excluded partners and the margin band:
  // 64 slots more; then the short keys [ps]. Pass 2 writes at most one key
  // per queued atom, so keys overwrite only queue slots already read. With
  // explicit images one atom can give several keys: the queue then has its
  // own V.qimg slots after the short keys (at least the replica's atoms).
  unsigned *kc = lds;
  unsigned *ks = lds + pc + 64;
  unsigned *kq = img ? ks + ps : kc;
  const int pq = img ? V.qimg : pc + 64;
  const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
  const int nd[3] = {V.rep_cdim[3 * r], V.rep_cdim[3 * r + 1], V.rep_cdim[3 * r + 2]};
  const int coff = V.rep_cell_off[r];
  const int cl = V.atom_cell[i] - coff;
  const int cx = cl % nd[0], cy = (cl / nd[0]) % nd[1], cz = cl / (nd[0] * nd[1]);
  const int x0 = V.xptr ? V.xptr[i] : 0, x1 = V.xptr ? V.xptr[i + 1] : 0;
  // up to four excluded partners in registers; more are looked up in memory
  int ex[4] = {-1, -1, -1, -1};
  for (int e = x0; e < x1 && e < x0 + 4; ++e) ex[e - x0] = V.xj[e];
  const bool ex_more = x1 - x0 > 4;
  const double rs_out = V.rs + V.skin;
  const int capk = (want & 4) ? V.cap_c : V.cap_f;
  int nk = 0, nsr = 0;
  int zlo, zhi, ylo, yhi, xlo, xhi;
  stencil_range(cz, nd[2], zlo, zhi);
  stencil_range(cy, nd[1], ylo, yhi);
  stencil_range(cx, nd[0], xlo, xhi);
  // The stencil as at most 50 contiguous spans of the cell-ordered arrays:
  // (z, y) rows of x-runs, each run split in two where it wraps. Lane t
  // resolves span t; an inclusive scan gives every candidate a flat index,
  // so the whole stencil streams through 64-wide chunks with independent loads.
  const int ny = yhi - ylo + 1, nz = zhi - zlo + 1;
  int sb = 0, sl = 0;
  if (lane < 2 * ny * nz) {
    const int part = lane & 1, yz = lane >> 1;
    const int zz = zlo + yz / ny, yy = ylo + yz % ny;
    const int ccz = (zz + nd[2]) % nd[2], ccy = (yy + nd[1]) % nd[1];
    const int row0 = coff + (ccz * nd[1] + ccy) * nd[0];
    int lo = -1, hi = -2;
    if (xlo >= 0 && xhi < nd[0]) { if (part == 0) { lo = xlo; hi = xhi; } }
    else if (xlo < 0) { if (part == 0) { lo = xlo + nd[0]; hi = nd[0] - 1; } else { lo = 0; hi = xhi; } }
    else { if (part == 0) { lo = xlo; hi = nd[0] - 1; } else { lo = 0; hi = xhi - nd[0]; } }
    if (hi >= lo) { sb = V.cell_start[row0 + lo]; sl = V.cell_start[row0 + hi + 1] - sb; }
  }
  int incl = sl;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  __shared__ int s_beg[64], s_pre[65];
  s_beg[lane] = sb;
  s_pre[lane + 1] = incl;
  if (lane == 0) s_pre[0] = 0;
  __syncthreads();
  const int total = s_pre[64];
  int span = 0;   // per lane: the span holding its current flat index (indices only grow)
  // Pass 1: a float distance filter over the whole stencil queues the
  // cell-array indices of the atoms that may lie within the outer cutoff
  // (in kc, which pass 2 overwrites only at slots it has already read). It
  // reads the float copy of the positions wrapped into the box (16 B per
  // stencil atom instead of 32). The margin covers the rounding of the
  // wrapped coordinates, of their difference and of the minimum image (each
  // a few float ulps of L) with a factor above 8.
  const double rcut = (want & 6) ? V.rout : rs_out;
  const float Lf[3] = {(float)L[0], (float)L[1], (float)L[2]};
  const float iLf[3] = {(float)iL[0], (float)iL[1], (float)iL[2]};
  const float margin0 = 1e-3f + 3e-6f * (Lf[0] + Lf[1] + Lf[2]);
  const float rcf = (float)rcut;
  const float xiw = (float)(xi.x - L[0] * floor(xi.x / L[0]));
  const float yiw = (float)(xi.y - L[1] * floor(xi.y / L[1]));
  const float ziw = (float)(xi.z - L[2] * floor(xi.z / L[2]));
  int nq = 0;
  // the next chunk's cell index and position are loaded while this chunk is tested
  int qn = 0;
  float4 xn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (lane < total) {
    while (s_pre[span + 1] <= lane) ++span;
    qn = s_beg[span] + (lane - s_pre[span]);
    xn = V.xcellf[qn];
  }
  for (int base = 0; base < total; base += 64) {
    const int f = base + lane;
    const int q = qn;
    const float4 xj = xn;
    if (f + 64 < total) {
      while (s_pre[span + 1] <= f + 64) ++span;
      qn = s_beg[span] + (f + 64 - s_pre[span]);
      xn = V.xcellf[qn];
    }
    bool keep = false;
    if (f < total) {
      float dx = xiw - xj.x, dy = yiw - xj.y, dz = ziw - xj.z;
      const float rc_m = rcf + margin0 + 1e-6f * (fabsf(dx) + fabsf(dy) + fabsf(dz));
      dx -= Lf[0] * rintf(dx * iLf[0]);
      dy -= Lf[1] * rintf(dy * iLf[1]);
      dz -= Lf[2] * rintf(dz * iLf[2]);
      keep = dx * dx + dy * dy + dz * dz < rc_m * rc_m;
    }
    const unsigned long long mq = __ballot(keep);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (keep) {
      const int pos = nq + __popcll(mq & below);
      if (pos < pq) kq[pos] = (unsigned)q;
    }
    nq += __popcll(mq);
  }
  const int nqq = min(nq, pq);
  wave_lds_sync();
  // Pass 2: exact FP64 decisions for the queued atoms. In a replica with an
  // edge below 2 (r_c + skin) the images of j next to the nearest one (along
  // the short edges) are tested too, and keys carry the image: segment << 27
  // | local j << 14 | image number << 9 | image code (the lattice vector mod 8
  // of the row entry); the image number (s_x+1) + 3 (s_y+1) + 9 (s_z+1) of
  // the offset s from the nearest image orders the images of one j.
  // Otherwise keys are segment << 24 | j (candidates) or j.
  const int rep0 = V.rep_off[r];
  // the next chunk's atom and position are loaded while this chunk is tested; keys
  // overwrite only queue slots of chunks already read
  int jn = -1;
  double4 xjn = make_double4(0.0, 0.0, 0.0, 0.0);
  if (lane < nqq) {
    const int q = (int)kq[lane];
    jn = V.cell_atoms[q];
    xjn = V.xcell[q];
  }
  for (int base = 0; base < nqq; base += 64) {
    int j = jn;
    double4 xj = xjn;
    bool ok = base + lane < nqq;
    if (base + 64 + lane < nqq) {
      const int q = (int)kq[base + 64 + lane];
      jn = V.cell_atoms[q];
      xjn = V.xcell[q];
    }
    wave_lds_sync();   // the queue slots of this chunk and the next are read before keys overwrite them
    ok = ok && j != i && j != ex[0] && j != ex[1] && j != ex[2] && j != ex[3];
    if (ok && ex_more)
      for (int e = x0 + 4; ok && e < x1; ++e) ok = (V.xj[e] != j);
    const double d0x = xi.x - xj.x, d0y = xi.y - xj.y, d0z = xi.z - xj.z;
    const double mx = rint(d0x * iL[0]), my = rint(d0y * iL[1]), mz = rint(d0z * iL[2]);
    // Along an edge below 2 (r_c + skin) the next image on the side the
    // nearest one leans to can also be within reach; the one on the other
    // side is at least an edge away. Combination cb picks, per edge, the
    // nearest image (bit clear) or that neighbour (bit set); uniform over the wave.
    const int ax = d0x - L[0] * mx > 0.0 ? 1 : -1, ay = d0y - L[1] * my > 0.0 ? 1 : -1;
    const int az = d0z - L[2] * mz > 0.0 ? 1 : -1;
    for (int cb = 0; cb < (img ? 8 : 1); ++cb) {
      if (((cb & 1) && !(L[0] < 2.0 * V.rout)) || ((cb & 2) && !(L[1] < 2.0 * V.rout)) ||
          ((cb & 4) && !(L[2] < 2.0 * V.rout)))
        continue;
      const int sx = (cb & 1) ? ax : 0, sy = (cb & 2) ? ay : 0, sz = (cb & 4) ? az : 0;
      const int si = (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1);
      bool bs = false, bk = false;
      unsigned key = 0, skey = 0;
      if (ok) {
        const double nx = mx + (double)sx, ny = my + (double)sy, nz = mz + (double)sz;
        const double ddx = d0x - L[0] * nx, ddy = d0y - L[1] * ny, ddz = d0z - L[2] * nz;
        const double rr = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
        bs = (want & 1) && rr < rs_out;
        const unsigned low = img ? ((unsigned)(j - rep0) << 14) | ((unsigned)si << 9) |
                                       ((unsigned)((int)nx & 7)) | ((unsigned)((int)ny & 7) << 3) |
                                       ((unsigned)((int)nz & 7) << 6)
                                 : (unsigned)j;
        skey = low;
        if (want & 4) {
          bk = rr >= V.rin && rr < V.rout;
          if (bk) {
            int ring = (int)floor((rr - V.rin) / V.rw);
            ring = ring < 0 ? 0 : (ring > V.nr - 1 ? V.nr - 1 : ring);
            key = ((unsigned)(V.type[j] * V.nr + ring) << (img ? 27 : 24)) | low;
          }
        } else if (want & 2) {
          bk = rr < V.rout;
          key = low;
        }
      }
      const unsigned long long mk = __ballot(bk), ms = __ballot(bs);
      const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      if (bk) {
        const int pos = nk + __popcll(mk & below);
        if (pos < pc) kc[pos] = key;
      }
      if (bs) {
        const int pos = nsr + __popcll(ms & below);
        if (pos < ps) ks[pos] = skey;
      }
      nk += __popcll(mk);
      nsr += __popcll(ms);
    }
  }
  // requested lengths beyond capacity: the host regrows the rows and replays
  // the steps since its last good synchronisation
  if (lane == 0) {
    if (nsr > V.cap_s) atomicMax(&V.ctl->ovf_short, nsr);
    if (nk > capk) atomicMax(&V.ctl->ovf_long, nk);
    if (nq > pq) atomicMax(&V.ctl->ovf_queue, nq);
  }
  const int nkk = min(nk, min(capk, pc)), nss = min(nsr, min(V.cap_s, ps));
  // key -> row entry: the partner's global index, with the image code above it
  auto entry = [&](unsigned key) -> int {
    if (!img) return (int)(key & (unsigned)MD_ROW_J_MASK);
    return (int)(((unsigned)rep0 + ((key >> 14) & 0x1fffu)) | ((key & 0x1ffu) << MD_ROW_IMG_SHIFT));
  };
  if (want & 6) {
    __syncthreads();
    sort_keys(kc, nkk);
    int *row = (want & 4) ? V.crow + (size_t)i * V.cap_c : V.frow + (size_t)i * V.cap_f;
    for (int e = lane; e < nkk; e += 64) row[e] = entry(kc[e]);
    if (lane == 0) { if (want & 4) V.ccnt[i] = nkk; else V.fcnt[i] = nkk; }
    if (want & 4) {
      for (int sg = lane; sg <= V.S; sg += 64) {
        int lo = 0, hi = nkk;
        if (sg < V.S) {   // (S << 27 would not fit 32 bits)
          const unsigned probe = (unsigned)sg << (img ? 27 : 24);
          while (lo < hi) { int mid = (lo + hi) >> 1; if (kc[mid] < probe) lo = mid + 1; else hi = mid; }
        } else {
          lo = nkk;
        }
        V.segst[(size_t)i * (V.S + 1) + sg] = lo;
      }
    }
  }
  if (want & 1) {
    __syncthreads();
    sort_keys(ks, nss);
    int *row = V.srow + (size_t)i * V.cap_s;
    for (int e = lane; e < nss; e += 64) row[e] = entry(ks[e]);
    if (lane == 0) V.scnt[i] = nss;
  }
}

// -------------------------------------------------------------- forces
// bonded force on atom i: harmonic bonds and angles over its incident terms
__device__ __forceinline__ void bonded_atom(const MDView &V, const double4 *__restrict__ X, int i) {
  const int r = V.rep[i];
  const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
  const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
  double f[3] = {0.0, 0.0, 0.0};
  for (int e = V.bptr[i]; e < V.bptr[i + 1]; ++e) {
    int code = V.bterm[e], t = code >> 1;
    if (!(code & 1)) {
      int p = V.bond_ij[2 * t], q = V.bond_ij[2 * t + 1];
      double4 xp = X[p], xq = X[q];
      double d[3] = {min_img(xp.x - xq.x, L[0], iL[0]), min_img(xp.y - xq.y, L[1], iL[1]),
                     min_img(xp.z - xq.z, L[2], iL[2])};
      double b = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      double db = b - V.bond_r0[t];
      double sgn = (i == p) ? 1.0 : -1.0;
      for (int c = 0; c < 3; ++c) f[c] += sgn * (-V.bond_k[t] * db * d[c] / b);
    } else {
      int p = V.angle_ijk[3 * t], m = V.angle_ijk[3 * t + 1], q = V.angle_ijk[3 * t + 2];
      double4 xp = X[p], xm = X[m], xq = X[q];
      double u[3] = {min_img(xp.x - xm.x, L[0], iL[0]), min_img(xp.y - xm.y, L[1], iL[1]),
                     min_img(xp.z - xm.z, L[2], iL[2])};
      double w[3] = {min_img(xq.x - xm.x, L[0], iL[0]), min_img(xq.y - xm.y, L[1], iL[1]),
                     min_img(xq.z - xm.z, L[2], iL[2])};
      double ru = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      double rw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
      double cs = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) / (ru * rw);
      cs = fmin(1.0, fmax(-1.0, cs));
      double th = acos(cs), sn = sqrt(1.0 - cs * cs);
      double dUdth = V.angle_k[t] * (th - V.angle_t0[t]);
      for (int c = 0; c < 3; ++c) {
        double fi = dUdth * (w[c] / (ru * rw) - cs * u[c] / (ru * ru)) / sn;
        double fk = dUdth * (u[c] / (ru * rw) - cs * w[c] / (rw * rw)) / sn;
        if (i == p) f[c] += fi;
        else if (i == q) f[c] += fk;
        else f[c] -= fi + fk;
      }
    }
  }
  V.fb[i] = make_double4(f[0], f[1], f[2], 0.0);
}

// MODE 0: -grad chi U over r < r_s (short rows); MODE 1: -grad U over r < r_c (full rows);
// MODE 2: -grad (1 - chi) U over r < r_c (full rows) into V.flong.
// BONDED: blocks from nb_pair on compute the bonded forces instead (one atom
// per lane), so that they run beside the pair blocks in one launch (a
// separate instantiation: the bonded path's registers would cost the plain
// pair kernel occupancy).
// FP32 pair arithmetic with FP64 accumulation (mixed-precision path)
// types whose LJ table the FP32 pair kernel keeps in LDS (more types read it from memory)
#define MD_FORCE_LDS_TYPES 8
template <int MODE, int SG, bool BONDED>
__global__ __launch_bounds__(256) void k_force_f(MDView V, const double4 *__restrict__ X, int nb_pair) {
  if (BONDED && (int)blockIdx.x >= nb_pair) {
    const int ib = ((int)blockIdx.x - nb_pair) * (int)blockDim.x + (int)threadIdx.x;
    if (ib < V.n) bonded_atom(V, X, ib);
    return;
  }
  // LJ coefficients of every type pair in LDS (up to MD_FORCE_LDS_TYPES types), so that a
  // pair's coefficients follow its partner's type without another global load
  __shared__ float s_lj[3 * MD_FORCE_LDS_TYPES * MD_FORCE_LDS_TYPES];
  const int nt = V.nt;
  const bool tab = nt <= MD_FORCE_LDS_TYPES;
  if (tab) {
    for (int t = threadIdx.x; t < nt * nt; t += blockDim.x) {
      s_lj[3 * t] = (float)V.c12[t];
      s_lj[3 * t + 1] = (float)V.c6[t];
      s_lj[3 * t + 2] = (float)V.ljshift[t];
    }
    __syncthreads();
  }
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / SG, lane = gid % SG;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (i < V.n) {
    const double4 xi = X[i];
    const int a = V.type[i], r = V.rep[i];
    const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
    const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    const bool img = rep_images(L, V.rout);
    const int *row = MODE == 0 ? V.srow + (size_t)i * V.cap_s : V.frow + (size_t)i * V.cap_f;
    const int cnt = MODE == 0 ? V.scnt[i] : V.fcnt[i];
    const float cut = (float)(MODE == 0 ? V.rs : V.rc);
    const float cut2 = cut * cut;
    const float kq = (float)(V.ke * xi.w);
    // software pipeline: the next row entry, its partner's position and type are loaded
    // while the current pair is evaluated
    int e = 0, tj = 0;
    double4 xj = make_double4(0.0, 0.0, 0.0, 0.0);
    if (lane < cnt) {
      e = row[lane];
      xj = X[row_j(e)];
      tj = V.type[row_j(e)];
    }
    for (int k = lane; k < cnt; k += SG) {
      int en = 0, tjn = 0;
      double4 xjn = make_double4(0.0, 0.0, 0.0, 0.0);
      if (k + SG < cnt) {
        en = row[k + SG];
        xjn = X[row_j(en)];
        tjn = V.type[row_j(en)];
      }
      double ddx, ddy, ddz;
      row_disp(xi, xj, L, iL, img, e, ddx, ddy, ddz);
      const float dx = (float)ddx, dy = (float)ddy, dz = (float)ddz;
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < cut2) {
        const float rr = sqrtf(r2);
        const float ir = 1.0f / rr;
        const int ab = a * nt + tj;
        float U = 0.0f, dU = 0.0f;
        const float c12 = tab ? s_lj[3 * ab] : (float)V.c12[ab];
        const float c6 = tab ? s_lj[3 * ab + 1] : (float)V.c6[ab];
        if (c12 != 0.0f || c6 != 0.0f)
          lj_pair_f(ir, c12, c6, tab ? s_lj[3 * ab + 2] : (float)V.ljshift[ab], U, dU);
        const float kqq = kq * (float)xj.w;
        if (kqq != 0.0f) {
          float Uc, dUc;
          dsf_pair_f(rr, ir, kqq, V, Uc, dUc);
          U += Uc; dU += dUc;
        }
        float g = dU;
        if (MODE == 0) {
          float chi, dchi;
          switch_fn_f(rr, V, chi, dchi);
          g = chi * dU + dchi * U;
        } else if (MODE == 2) {
          float chi, dchi;
          switch_fn_f(rr, V, chi, dchi);
          g = (1.0f - chi) * dU - dchi * U;
        }
        const float sc = -g * ir;
        fx += (double)(sc * dx); fy += (double)(sc * dy); fz += (double)(sc * dz);
      }
      e = en; xj = xjn; tj = tjn;
    }
  }
#pragma unroll
  for (int off = SG / 2; off > 0; off >>= 1) {
    fx += __shfl_xor(fx, off, SG);
    fy += __shfl_xor(fy, off, SG);
    fz += __shfl_xor(fz, off, SG);
  }
  if (i < V.n && lane == 0) (MODE == 2 ? V.flong : V.fnb)[i] = make_double4(fx, fy, fz, 0.0);
}

template <int MODE, int SG, bool BONDED>
__global__ __launch_bounds__(256) void k_force(MDView V, const double4 *__restrict__ X, int nb_pair) {
  if (BONDED && (int)blockIdx.x >= nb_pair) {
    const int ib = ((int)blockIdx.x - nb_pair) * (int)blockDim.x + (int)threadIdx.x;
    if (ib < V.n) bonded_atom(V, X, ib);
    return;
  }
  // LJ coefficients of every type pair in LDS (up to MD_FORCE_LDS_TYPES types)
  __shared__ double s_lj[3 * MD_FORCE_LDS_TYPES * MD_FORCE_LDS_TYPES];
  const int nt = V.nt;
  const bool tab = nt <= MD_FORCE_LDS_TYPES;
  if (tab) {
    for (int t = threadIdx.x; t < nt * nt; t += blockDim.x) {
      s_lj[3 * t] = V.c12[t];
      s_lj[3 * t + 1] = V.c6[t];
      s_lj[3 * t + 2] = V.ljshift[t];
    }
    __syncthreads();
  }
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid / SG, lane = gid % SG;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (i < V.n) {
    const double4 xi = X[i];
    const int a = V.type[i], r = V.rep[i];
    const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
    const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    const bool img = rep_images(L, V.rout);
    const int *row = MODE == 0 ? V.srow + (size_t)i * V.cap_s : V.frow + (size_t)i * V.cap_f;
    const int cnt = MODE == 0 ? V.scnt[i] : V.fcnt[i];
    const double cut = MODE == 0 ? V.rs : V.rc;
    const double cut2 = cut * cut;
    // pair term of row entry e (partner j at xj, of type tj, or read here when tj < 0)
    auto pair = [&](int e, int j, const double4 &xj, int tj) {
      double dx, dy, dz;
      row_disp(xi, xj, L, iL, img, e, dx, dy, dz);
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < cut2) {
        double rr = sqrt(r2);
        const double ir = 1.0 / rr;
        const int ab = a * nt + (tj >= 0 ? tj : V.type[j]);
        double U = 0.0, dU = 0.0;
        const double c12 = tab ? s_lj[3 * ab] : V.c12[ab], c6 = tab ? s_lj[3 * ab + 1] : V.c6[ab];
        if (c12 != 0.0 || c6 != 0.0) lj_pair(ir, c12, c6, tab ? s_lj[3 * ab + 2] : V.ljshift[ab], U, dU);
        double qq = xi.w * xj.w;
        if (qq != 0.0) {
          double Uc, dUc;
          dsf_pair(rr, ir, V.ke * qq, V, Uc, dUc);
          U += Uc; dU += dUc;
        }
        double g = dU;
        if (MODE == 0) {
          double chi, dchi;
          switch_fn(rr, V, chi, dchi);
          g = chi * dU + dchi * U;
        } else if (MODE == 2) {
          double chi, dchi;
          switch_fn(rr, V, chi, dchi);
          g = (1.0 - chi) * dU - dchi * U;
        }
        double sc = -g * ir;
        fx += sc * dx; fy += sc * dy; fz += sc * dz;
      }
    };
    if (MODE == 0) {
      // short rows: the next row entry, its partner's position and type are loaded while
      // the current pair is evaluated (the full-range sweeps are bound by their arithmetic
      // and keep the plain loop, which measured faster there)
      int e = 0, tj = 0;
      double4 xj = make_double4(0.0, 0.0, 0.0, 0.0);
      if (lane < cnt) {
        e = row[lane];
        xj = X[row_j(e)];
        tj = V.type[row_j(e)];
      }
      for (int k = lane; k < cnt; k += SG) {
        int en = 0, tjn = 0;
        double4 xjn = make_double4(0.0, 0.0, 0.0, 0.0);
        if (k + SG < cnt) {
          en = row[k + SG];
          xjn = X[row_j(en)];
          tjn = V.type[row_j(en)];
        }
        pair(e, row_j(e), xj, tj);
        e = en; xj = xjn; tj = tjn;
      }
    } else {
      for (int k = lane; k < cnt; k += SG) {
        const int e = row[k], j = row_j(e);
        pair(e, j, X[j], -1);
      }
    }
  }
#pragma unroll
  for (int off = SG / 2; off > 0; off >>= 1) {
    fx += __shfl_xor(fx, off, SG);
    fy += __shfl_xor(fy, off, SG);
    fz += __shfl_xor(fz, off, SG);
  }
  if (i < V.n && lane == 0) (MODE == 2 ? V.flong : V.fnb)[i] = make_double4(fx, fy, fz, 0.0);
}

// bonds (k/2)(b-b0)^2 and angles (k/2)(theta-theta0)^2, per atom over incident terms
__global__ void k_bonded(MDView V, const double4 *__restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < V.n) bonded_atom(V, X, i);
}

// --------------------------------------------------------- observables
__global__ __launch_bounds__(256) void k_ke(MDView V, double *part) {
  __shared__ double sm[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < V.n) {
    double4 v = V.v[i];
    e = 0.5 * v.w * (v.x * v.x + v.y * v.y + v.z * v.z);
  }
  sm[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// per-atom pair energies: which = 0 -> chi U from short rows, 1 -> (1-chi) U
// from candidate rows, 2 -> both parts from full rows; halves of each pair.
__global__ void k_pair_energy(MDView V, const double4 *__restrict__ X, int which, double *es, double *el) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const double4 xi = X[i];
  const int a = V.type[i], r = V.rep[i];
  const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
  const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
  const bool img = rep_images(L, V.rout);
  const int *row; int cnt;
  if (which == 0) { row = V.srow + (size_t)i * V.cap_s; cnt = V.scnt[i]; }
  else if (which == 1) { row = V.crow + (size_t)i * V.cap_c; cnt = V.ccnt[i]; }
  else { row = V.frow + (size_t)i * V.cap_f; cnt = V.fcnt[i]; }
  double s = 0.0, l = 0.0;
  for (int k = 0; k < cnt; ++k) {
    const int e = row[k], j = row_j(e);
    double4 xj = X[j];
    double dx, dy, dz;
    row_disp(xi, xj, L, iL, img, e, dx, dy, dz);
    double r2 = dx * dx + dy * dy + dz * dz, rr = sqrt(r2);
    if (rr >= V.rc) continue;
    int ab = a * V.nt + V.type[j];
    double U = 0.0, dU = 0.0;
    const double ir = 1.0 / rr;
    if (V.c12[ab] != 0.0 || V.c6[ab] != 0.0) lj_pair(ir, V.c12[ab], V.c6[ab], V.ljshift[ab], U, dU);
    double qq = xi.w * xj.w;
    if (qq != 0.0) { double Uc, dUc; dsf_pair(rr, ir, V.ke * qq, V, Uc, dUc); U += Uc; }
    double chi, dchi;
    switch_fn(rr, V, chi, dchi);
    if (which == 0 || which == 2) s += 0.5 * chi * U;
    if (which == 1 || which == 2) l += 0.5 * (1.0 - chi) * U;
  }
  es[i] = s; el[i] = l;
}

// bonded energy per term: bonds occupy [0, nb), angles [nb, nb + na)
__global__ void k_bonded_energy(MDView V, const double4 *__restrict__ X, int nb, int na, double *e) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb + na) return;
  if (t < nb) {
    int p = V.bond_ij[2 * t], q = V.bond_ij[2 * t + 1];
    const int r = V.rep[p];
    double4 xp = X[p], xq = X[q];
    double d[3] = {min_img(xp.x - xq.x, V.box[3 * r], 1.0 / V.box[3 * r]),
                   min_img(xp.y - xq.y, V.box[3 * r + 1], 1.0 / V.box[3 * r + 1]),
                   min_img(xp.z - xq.z, V.box[3 * r + 2], 1.0 / V.box[3 * r + 2])};
    double b = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - V.bond_r0[t];
    e[t] = 0.5 * V.bond_k[t] * b * b;
  } else {
    int a = t - nb;
    int p = V.angle_ijk[3 * a], m = V.angle_ijk[3 * a + 1], q = V.angle_ijk[3 * a + 2];
    const int r = V.rep[m];
    double4 xp = X[p], xm = X[m], xq = X[q];
    double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
    double u[3] = {min_img(xp.x - xm.x, L[0], 1.0 / L[0]), min_img(xp.y - xm.y, L[1], 1.0 / L[1]),
                   min_img(xp.z - xm.z, L[2], 1.0 / L[2])};
    double w[3] = {min_img(xq.x - xm.x, L[0], 1.0 / L[0]), min_img(xq.y - xm.y, L[1], 1.0 / L[1]),
                   min_img(xq.z - xm.z, L[2], 1.0 / L[2])};
    double cs = (u[0] * w[0] + u[1] * w[1] + u[2] * w[2]) /
                (sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]));
    cs = fmin(1.0, fmax(-1.0, cs));
    double dth = acos(cs) - V.angle_t0[a];
    e[t] = 0.5 * V.angle_k[a] * dth * dth;
  }
}

__global__ void k_rdf(MDView V, const double4 *__restrict__ X, const int *rep_off, int ta, int tb,
                      double rmax, int nbins, unsigned long long *hist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const int a = V.type[i];
  if (a != ta && a != tb) return;
  const int r = V.rep[i];
  const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
  const double4 xi = X[i];
  const double dr = rmax / nbins;
  for (int j = i + 1; j < rep_off[r + 1]; ++j) {
    int b = V.type[j];
    if (!((a == ta && b == tb) || (a == tb && b == ta))) continue;
    double4 xj = X[j];
    double dx = min_img(xi.x - xj.x, L[0], 1.0 / L[0]);
    double dy = min_img(xi.y - xj.y, L[1], 1.0 / L[1]);
    double dz = min_img(xi.z - xj.z, L[2], 1.0 / L[2]);
    double rr = sqrt(dx * dx + dy * dy + dz * dz);
    if (rr >= rmax) continue;
    int bin = (int)(rr / dr);
    if (bin < nbins) atomicAdd(&hist[bin], 1ull);
  }
}

// unordered pairs (j > i) of the given rows closer than cut: which 0 = short rows, 1 = full rows
__global__ void k_count_pairs(MDView V, const double4 *__restrict__ X, int which, double cut,
                              unsigned long long *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const double4 xi = X[i];
  const int r = V.rep[i];
  const double L[3] = {V.box[3 * r], V.box[3 * r + 1], V.box[3 * r + 2]};
  const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
  const bool img = rep_images(L, V.rout);
  const int *row = which == 0 ? V.srow + (size_t)i * V.cap_s : V.frow + (size_t)i * V.cap_f;
  const int cnt = which == 0 ? V.scnt[i] : V.fcnt[i];
  unsigned long long c = 0;
  for (int k = 0; k < cnt; ++k) {
    const int e = row[k], j = row_j(e);
    if (j <= i) continue;
    double4 xj = X[j];
    double dx, dy, dz;
    row_disp(xi, xj, L, iL, img, e, dx, dy, dz);
    if (dx * dx + dy * dy + dz * dz < cut * cut) ++c;
  }
  if (c) atomicAdd(out, c);
}

// ----------------------------------------------------------- Ewald sum
// Reciprocal-space part of the Ewald sum (one replica): with k over the half
// space (k and -k give equal terms), w_k = exp(-k^2 / (4 alpha^2)) / k^2 and
// the structure factor S(k) = sum_j q_j exp(i k.x_j),
//   E_k = 2 (2 pi k_e / V) sum_k w_k |S(k)|^2,
//   f_i = 2 (4 pi k_e / V) q_i sum_k w_k k (Re S sin(k.x_i) - Im S cos(k.x_i)),
// plus, for every excluded pair, the force of -k_e q_i q_j erf(alpha r) / r
// (their real-space term is left out, so their reciprocal-space interaction
// is taken back).
// Partial structure factors. Block (kc, ar) covers k-vectors
// [kc * EW_KPB, (kc + 1) * EW_KPB), EW_KPT per thread, and the atoms of range
// ar in tiles of V.ew_ta atoms (at most EW_TA). For each tile the block tabulates in LDS the factors
// e^{i 2 pi m x / L_x} (m = 0..K) and e^{i 2 pi m y / L_y}, e^{i 2 pi m z / L_z}
// (m = -K..K) of every atom, so that each (atom, k) term is a product of three
// table entries instead of a sine and a cosine of its own.
constexpr int EW_TA = 16, EW_KPT = 4, EW_KPB = 256 * EW_KPT;
static size_t ewald_lds_bytes(int kmax, int ta) { return sizeof(double2) * ta * (5 * kmax + 3) + sizeof(double) * ta; }
__global__ __launch_bounds__(256) void k_sfac(MDView V, const double4 *__restrict__ X, double2 *__restrict__ part) {
  extern __shared__ double2 ew_tab[];   // ew_ta atoms x (5K + 3) factors, then their charges
  const int K = V.kmax, W = 5 * K + 3, TA = V.ew_ta;
  double *qs = (double *)(ew_tab + TA * W);
  const double iL[3] = {1.0 / V.box[0], 1.0 / V.box[1], 1.0 / V.box[2]};
  int ox[EW_KPT], oy[EW_KPT], oz[EW_KPT];
  double sr[EW_KPT], si[EW_KPT];
#pragma unroll
  for (int j = 0; j < EW_KPT; ++j) {
    const int k = blockIdx.x * EW_KPB + j * 256 + threadIdx.x;
    const int4 nk = k < V.nk ? V.kint[k] : make_int4(0, 0, 0, 0);
    ox[j] = nk.x; oy[j] = K + 1 + nk.y + K; oz[j] = 3 * K + 2 + nk.z + K;
    sr[j] = 0.0; si[j] = 0.0;
  }
  const int a0 = blockIdx.y * V.ew_apb, a1 = min(V.n, a0 + V.ew_apb);
  for (int t0 = a0; t0 < a1; t0 += TA) {
    const int na = min(TA, a1 - t0);
    __syncthreads();   // the previous tile's reads are complete
    for (int e = threadIdx.x; e < na * W; e += 256) {
      const int at = e / W, m = e - at * W;
      const double4 x = X[t0 + at];
      double ph;   // phase / pi
      if (m <= K) ph = 2.0 * m * x.x * iL[0];
      else if (m <= 3 * K + 1) ph = 2.0 * (m - (2 * K + 1)) * x.y * iL[1];
      else ph = 2.0 * (m - (4 * K + 2)) * x.z * iL[2];
      double sn, cs;
      sincospi(ph, &sn, &cs);
      ew_tab[e] = make_double2(cs, sn);
    }
    if ((int)threadIdx.x < na) qs[threadIdx.x] = X[t0 + threadIdx.x].w;
    __syncthreads();
    for (int at = 0; at < na; ++at) {
      const double q = qs[at];
      const double2 *ta = ew_tab + at * W;
#pragma unroll
      for (int j = 0; j < EW_KPT; ++j) {
        const double2 cx = ta[ox[j]], cy = ta[oy[j]], cz = ta[oz[j]];
        const double xr = cx.x * cy.x - cx.y * cy.y, xi = cx.x * cy.y + cx.y * cy.x;
        sr[j] += q * (xr * cz.x - xi * cz.y);
        si[j] += q * (xr * cz.y + xi * cz.x);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < EW_KPT; ++j) {
    const int k = blockIdx.x * EW_KPB + j * 256 + threadIdx.x;
    if (k < V.nk) part[(size_t)blockIdx.y * V.nk + k] = make_double2(sr[j], si[j]);
  }
}

// S(k) = sum over atom ranges in range order (deterministic)
__global__ void k_sfac_sum(MDView V, const double2 *__restrict__ part, double2 *__restrict__ S) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= V.nk) return;
  double sr = 0.0, si = 0.0;
  for (int t = 0; t < V.ew_ranges; ++t) {
    const double2 p = part[(size_t)t * V.nk + k];
    sr += p.x;
    si += p.y;
  }
  S[k] = make_double2(sr, si);
}

// Reciprocal-space forces. Block (ab, kr) covers 256 atoms, one per lane,
// and k-range kr of V.ew_krange k-vectors, staged in LDS with S(k); the
// block writes the range's partial forces (summed in range order by
// k_recip_sum). Along a column (nx, ny fixed, nz rising by one) e^{i k.x}
// advances by the factor e^{i 2 pi z / L_z}; the first k-vector of each
// column, and of each range, takes its sine and cosine directly.
__global__ __launch_bounds__(256) void k_recip_force(MDView V, const double4 *__restrict__ X,
                                                     const double2 *__restrict__ S, double4 *__restrict__ fpart) {
  __shared__ double4 ks[256];
  __shared__ double2 ss[256];
  __shared__ int fs[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int kb = blockIdx.y * V.ew_krange, ke = min(V.nk, kb + V.ew_krange);
  const double4 xi = i < V.n ? X[i] : make_double4(0.0, 0.0, 0.0, 0.0);
  double ezs, ezc;
  sincospi(2.0 * xi.z / V.box[2], &ezs, &ezc);
  double er = 1.0, ei = 0.0;   // e^{i k.x} of the current k-vector
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int k0 = kb; k0 < ke; k0 += 256) {
    __syncthreads();
    if (k0 + (int)threadIdx.x < ke) {
      ks[threadIdx.x] = V.kvec[k0 + threadIdx.x];
      ss[threadIdx.x] = S[k0 + threadIdx.x];
      fs[threadIdx.x] = V.kint[k0 + threadIdx.x].w || k0 + (int)threadIdx.x == kb;
    }
    __syncthreads();
    const int m = min(256, ke - k0);
    for (int q = 0; q < m; ++q) {
      const double4 kv = ks[q];
      const double2 sq = ss[q];
      if (fs[q]) {
        sincos(kv.x * xi.x + kv.y * xi.y + kv.z * xi.z, &ei, &er);
      } else {
        const double t = er * ezc - ei * ezs;
        ei = er * ezs + ei * ezc;
        er = t;
      }
      const double a = kv.w * (sq.x * ei - sq.y * er);
      fx += a * kv.x; fy += a * kv.y; fz += a * kv.z;
    }
  }
  if (i < V.n) fpart[(size_t)blockIdx.y * V.n + i] = make_double4(fx, fy, fz, 0.0);
}

// Force on atom i of -k_e q_i q_j erf(alpha r) / r over its excluded partners
// (their real-space term is left out, so their reciprocal-space
// interaction is taken back)
__device__ __forceinline__ void excluded_recip_force(const MDView &V, const double4 *__restrict__ X, int i,
                                                     double4 xi, double &fx, double &fy, double &fz) {
  if (!V.xptr) return;
  const double L[3] = {V.box[0], V.box[1], V.box[2]};
  const double a = V.alpha;
  for (int e = V.xptr[i]; e < V.xptr[i + 1]; ++e) {
    const int j = V.xj[e];
    const double4 xj = X[j];
    const double dx = min_img(xi.x - xj.x, L[0], 1.0 / L[0]);
    const double dy = min_img(xi.y - xj.y, L[1], 1.0 / L[1]);
    const double dz = min_img(xi.z - xj.z, L[2], 1.0 / L[2]);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double qq = V.ke * xi.w * xj.w;
    const double dEdr = -qq * (V.two_a_sqpi * exp(-a * a * r * r) / r - erf(a * r) / (r * r));
    fx -= dEdr * dx / r; fy -= dEdr * dy / r; fz -= dEdr * dz / r;
  }
}

// Forces = prefactor x (sum of the k-range partials in range order), plus
// the excluded-pair correction
__global__ void k_recip_sum(MDView V, const double4 *__restrict__ X, const double4 *__restrict__ fpart, int nkr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const double4 xi = X[i];
  double fx = 0.0, fy = 0.0, fz = 0.0;
  for (int t = 0; t < nkr; ++t) {
    const double4 p = fpart[(size_t)t * V.n + i];
    fx += p.x; fy += p.y; fz += p.z;
  }
  const double c = V.ew_fcoef * xi.w;
  fx *= c; fy *= c; fz *= c;
  excluded_recip_force(V, X, i, xi, fx, fy, fz);
  V.frec[i] = make_double4(fx, fy, fz, 0.0);
}

// ------------------------------------------------ smooth particle-mesh Ewald
// An atom at scaled coordinate u = K x / L = k0 + w (k0 = floor(u)) puts
// weight M_p(u - k) = M_p(w + j) on grid points k = k0 - j, j = 0..p-1, with
// M_p the cardinal B-spline of order p. T[j] = M_p(w + j) from the recursion
// M_n(u) = (u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)) / (n - 1), M_2(u) = 1 - |u - 1|,
// taken over j from the top so that one array serves every order; the
// derivative is dM_p(u) = M_{p-1}(u) - M_{p-1}(u - 1).
template <int P>
__device__ __forceinline__ void bspline_weights(double w, double *T, double *dT) {
  T[0] = w;
  T[1] = 1.0 - w;
#pragma unroll
  for (int j = 2; j < P; ++j) T[j] = 0.0;
#pragma unroll
  for (int n = 3; n <= P; ++n) {
    if (n == P && dT) {
#pragma unroll
      for (int j = 0; j < P; ++j) dT[j] = T[j] - (j > 0 ? T[j - 1] : 0.0);
    }
    const double inv = 1.0 / (n - 1);
#pragma unroll
    for (int j = n - 1; j >= 0; --j) T[j] = ((w + j) * T[j] + (j > 0 ? (n - w - j) * T[j - 1] : 0.0)) * inv;
  }
}

// k mod K in [0, K) for a mesh edge K that is a power of two
__device__ __forceinline__ int wrap_index(int k, int K) { return k & (K - 1); }

// charge spreading: 8 lanes per atom, lane j0 < p the p^2 grid points of
// the slice k0 - j0 along the first axis, atomic sums into the real parts of
// the (zeroed) complex grid
template <int P>
__global__ __launch_bounds__(256) void k_pme_spread(MDView V, const double4 *__restrict__ X) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = gid >> 3, j0 = gid & 7;
  if (i >= V.n || j0 >= P) return;
  const double4 x = X[i];
  if (x.w == 0.0) return;
  const double xs[3] = {x.x, x.y, x.z};
  double T[3][P];
  int k0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double u = V.pk[d] * xs[d] / V.box[d];
    const double fl = floor(u);
    k0[d] = (int)fl;
    bspline_weights<P>(u - fl, T[d], nullptr);
  }
  double *g = (double *)V.pgrid;
  double t0 = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) t0 = j == j0 ? T[0][j] : t0;
  const int g0 = wrap_index(k0[0] - j0, V.pk[0]) * V.pk[1];
  for (int j1 = 0; j1 < P; ++j1) {
    const int g01 = (g0 + wrap_index(k0[1] - j1, V.pk[1])) * V.pk[2];
    const double w01 = x.w * t0 * T[1][j1];
#pragma unroll
    for (int j2 = 0; j2 < P; ++j2)
      unsafeAtomicAdd(g + 2 * (size_t)(g01 + wrap_index(k0[2] - j2, V.pk[2])), w01 * T[2][j2]);
  }
}

// Charge spreading by planes: block x owns mesh plane x (first index) in LDS,
// adds the contributions of every atom whose support covers the plane (LDS
// atomics), then writes the plane whole (real parts, zero imaginary parts):
// no global atomics and no zeroing pass.
template <int P>
__global__ __launch_bounds__(256) void k_pme_spread_planes(MDView V, const double4 *__restrict__ X) {
  extern __shared__ double pl[];
  const int px = blockIdx.x;
  const int K0 = V.pk[0], K1 = V.pk[1], K2 = V.pk[2];
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) pl[e] = 0.0;
  __syncthreads();
  for (int i = threadIdx.x; i < V.n; i += blockDim.x) {
    const double4 x = X[i];
    if (x.w == 0.0) continue;
    const double u0 = K0 * x.x / V.box[0], f0 = floor(u0);
    const int d = wrap_index((int)f0 - px, K0);   // the atom's slice index j0 on this plane
    if (d >= P) continue;
    double T0[P], T1[P], T2[P];
    bspline_weights<P>(u0 - f0, T0, nullptr);
    const double u1 = K1 * x.y / V.box[1], f1 = floor(u1);
    const double u2 = K2 * x.z / V.box[2], f2 = floor(u2);
    bspline_weights<P>(u1 - f1, T1, nullptr);
    bspline_weights<P>(u2 - f2, T2, nullptr);
    double t0 = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) t0 = j == d ? T0[j] : t0;
    for (int j1 = 0; j1 < P; ++j1) {
      const int r1 = wrap_index((int)f1 - j1, K1) * K2;
      const double w01 = x.w * t0 * T1[j1];
#pragma unroll
      for (int j2 = 0; j2 < P; ++j2) atomicAdd(&pl[r1 + wrap_index((int)f2 - j2, K2)], w01 * T2[j2]);
    }
  }
  __syncthreads();
  double2 *g = V.pgrid + (size_t)px * K1 * K2;
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) g[e] = make_double2(pl[e], 0.0);
}

// In-place transform F(m) = sum_k x_k exp(+2 pi i m k / N) along one axis of
// the grid, N a power of two: each line of the axis is loaded into LDS in
// bit-reversed order and combined in log2 N radix-2 stages (iterative
// Cooley-Tukey), N / 2 threads per line, several lines per block.
__global__ __launch_bounds__(256) void k_fft_axis(double2 *__restrict__ g, const double2 *__restrict__ tw, int twn,
                                                  int K0, int K1, int K2, int axis) {
  extern __shared__ double2 fbuf[];
  const int Na = axis == 0 ? K0 : (axis == 1 ? K1 : K2);
  const int logN = 31 - __clz(Na);
  const int half = Na >> 1;
  const int lpb = blockDim.x / half;
  // contiguous axis: a line's elements on consecutive threads; strided axes:
  // consecutive lines (adjacent in memory) on consecutive threads
  const int lq = axis == 2 ? (int)threadIdx.x / half : (int)threadIdx.x % lpb;
  const int t = axis == 2 ? (int)threadIdx.x - lq * half : (int)threadIdx.x / lpb;
  const int nlines = (K0 * K1 * K2) / Na;
  const int line = blockIdx.x * lpb + lq;
  const bool ok = line < nlines;
  int base, stride;
  if (axis == 2) { base = line * K2; stride = 1; }
  else if (axis == 1) { const int a = line / K2, c = line - a * K2; base = a * K1 * K2 + c; stride = K2; }
  else { base = line; stride = K1 * K2; }
  double2 *Lb = fbuf + lq * (Na + 1);   // one element of padding per line (LDS banks)
  if (ok)
    for (int e = t; e < Na; e += half) Lb[__brev((unsigned)e) >> (32 - logN)] = g[(size_t)base + (size_t)e * stride];
  __syncthreads();
  for (int st = 1; st <= logN; ++st) {
    const int m = 1 << st, hm = m >> 1;
    const int grp = t / hm, j = t - grp * hm;
    const int i0 = grp * m + j, i1 = i0 + hm;
    if (ok) {
      const double2 w = tw[j * (twn / m)];
      const double2 u = Lb[i0], v = Lb[i1];
      const double vr = v.x * w.x - v.y * w.y, vi = v.x * w.y + v.y * w.x;
      Lb[i0] = make_double2(u.x + vr, u.y + vi);
      Lb[i1] = make_double2(u.x - vr, u.y - vi);
    }
    __syncthreads();
  }
  if (ok)
    for (int e = t; e < Na; e += half) g[(size_t)base + (size_t)e * stride] = Lb[e];
}

// ---- particle-mesh Ewald in four launches, for meshes whose (y, z) plane
// fits LDS as complex FP64 (K1 K2 <= 4096): spreading plus the y and z
// transforms plane by plane; then one x-line kernel takes the x transform,
// the influence function and the x part of the second transform; then the
// y and z part of the second transform plane by plane; then the gather.
// In between, a plane is stored with both of its indices bit-reversed (the
// output order of the decimation-in-frequency passes), which the second
// transform's decimation-in-time passes take as their input order.

// element (y, z) of a K1 x K2 plane in LDS: rows of K2 with the z index
// xor-ed by y, so that a column (fixed z) spreads over the LDS banks
__device__ __forceinline__ int plane_at(int y, int z, int K2) { return y * K2 + (z ^ (y & (K2 - 1))); }

// position of the n-th (from 0) set bit of m; n < popcount(m)
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int n) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    const int c = __popcll(m & ((1ull << w) - 1ull));
    if (n >= c) { n -= c; m >>= w; pos += w; }
  }
  return pos;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 w) {
  return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Transforms F(m) = sum_k x_k exp(+2 pi i m k / N) of nl lines of length N
// (a power of two) in LDS (element e of line l at addr(l, e)), all threads
// of the block taking the work of a pass in turn. DIF: natural order in,
// bit-reversed out; otherwise (DIT) bit-reversed in, natural out. Two
// radix-2 stages per pass (four elements per thread in registers), one
// single stage last when log2 N is odd. tw[j] = exp(+2 pi i j / twn).
template <bool DIF, typename Addr>
__device__ __forceinline__ void lds_fft_lines(double2 *buf, int nl, int N, const double2 *__restrict__ tw, int twn,
                                              Addr addr) {
  const int logN = 31 - __clz(N);
  for (int s = 0; s < logN;) {
    if (s + 1 < logN) {
      // quads {e, e + q, e + 2q, e + 3q}: DIT spans 2q then 4q, DIF 4q then 2q
      const int lq = DIF ? logN - s - 2 : s, q = 1 << lq;
      const int lnq = logN - 2;   // log2 of the quads per line
      const int nb = nl << lnq;
      const int t2 = twn >> (lq + 1), t4 = twn >> (lq + 2);   // twiddle strides of spans 2q, 4q
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const int l = b >> lnq, t = b & ((1 << lnq) - 1);
        const int j = t & (q - 1);
        const int e = ((t >> lq) << (lq + 2)) + j;
        const int a0 = addr(l, e), a1 = addr(l, e + q), a2 = addr(l, e + 2 * q), a3 = addr(l, e + 3 * q);
        double2 x0 = buf[a0], x1 = buf[a1], x2 = buf[a2], x3 = buf[a3];
        const double2 w2 = tw[j * t2], w4 = tw[j * t4], w4q = tw[(j + q) * t4];
        if (DIF) {
          double2 y0 = cadd(x0, x2), y2 = cmul(csub(x0, x2), w4);
          double2 y1 = cadd(x1, x3), y3 = cmul(csub(x1, x3), w4q);
          x0 = cadd(y0, y1); x1 = cmul(csub(y0, y1), w2);
          x2 = cadd(y2, y3); x3 = cmul(csub(y2, y3), w2);
        } else {
          const double2 v1 = cmul(x1, w2), v3 = cmul(x3, w2);
          const double2 y0 = cadd(x0, v1), y1 = csub(x0, v1), y2 = cadd(x2, v3), y3 = csub(x2, v3);
          const double2 u2 = cmul(y2, w4), u3 = cmul(y3, w4q);
          x0 = cadd(y0, u2); x2 = csub(y0, u2);
          x1 = cadd(y1, u3); x3 = csub(y1, u3);
        }
        buf[a0] = x0; buf[a1] = x1; buf[a2] = x2; buf[a3] = x3;
      }
      s += 2;
    } else {
      const int st = DIF ? logN - s : s + 1;   // span 2^st
      const int hm = 1 << (st - 1), lh = logN - 1;
      const int ts = twn >> st;
      const int nb = nl << lh;
      for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const int l = b >> lh, t = b & ((1 << lh) - 1);
        const int j = t & (hm - 1);
        const int e0 = ((t >> (st - 1)) << st) + j, e1 = e0 + hm;
        const double2 w = tw[j * ts];
        const int a0 = addr(l, e0), a1 = addr(l, e1);
        const double2 u = buf[a0], v = buf[a1];
        if (DIF) {
          buf[a0] = cadd(u, v);
          buf[a1] = cmul(csub(u, v), w);
        } else {
          const double2 vw = cmul(v, w);
          buf[a0] = cadd(u, vw);
          buf[a1] = csub(u, vw);
        }
      }
      s += 1;
    }
    __syncthreads();
  }
}

// Spreading, split over MD_PME_PARTS parts per plane so that K0 x parts
// blocks fill the device: block (x, part) accumulates the charges of its
// atoms with support on plane x in a real plane in LDS and writes it to its
// partial plane. The atoms are dealt out in chunks of 64, chunk c to wave
// c mod (parts x waves per block) over all blocks of a plane, so that atoms
// stored in spatial order (those near a plane in a run of chunks) spread
// over the plane's blocks and waves. Each wave tests 4 chunks at a time
// (independent loads);
// the ones with support (about p / K0 of them) are packed P lanes each (lane:
// atom, y offset j1), with their mesh coordinates passed between lanes, so
// that the LDS atomics run on full waves.
template <int P>
__global__ __launch_bounds__(256) void k_pme_spread_part(MDView V, const double4 *__restrict__ X,
                                                         double *__restrict__ part) {
  extern __shared__ double pr[];
  const int px = blockIdx.x, pp = blockIdx.y;
  const int K0 = V.pk[0], K1 = V.pk[1], K2 = V.pk[2];
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) pr[e] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int slot = lane / P, j1 = lane - slot * P;
  constexpr int APW = 64 / P;   // atoms per packed batch
  constexpr int U = 4;          // chunks of 64 atoms per wave and iteration
  const int nch = (V.n + 63) >> 6;
  const int wpb = (int)blockDim.x >> 6;
  const int cstride = (int)gridDim.y * wpb;               // chunks between two of this wave's
  const int cw = pp * wpb + ((int)threadIdx.x >> 6);      // this wave's first chunk
  for (int c0 = cw; c0 < nch; c0 += U * cstride) {
    double4 xq[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int i = ((c0 + q * cstride) << 6) + lane;
      xq[q] = i < V.n ? X[i] : make_double4(0.0, 0.0, 0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      // mesh coordinates K x / L, as the gather and the reference form them
      const double u0 = K0 * xq[q].x / V.box[0], f0 = floor(u0);
      const bool on = xq[q].w != 0.0 && wrap_index((int)f0 - px, K0) < P;
      const unsigned long long m = __ballot(on);
      if (m == 0ull) continue;
      double u1 = 0.0, u2 = 0.0;
      if (on) { u1 = K1 * xq[q].y / V.box[1]; u2 = K2 * xq[q].z / V.box[2]; }
      const int np = __popcll(m);
      for (int b0 = 0; b0 < np; b0 += APW) {
        const int src = nth_set_bit(m, min(b0 + slot, np - 1));
        const double v0 = __shfl(u0, src), v1 = __shfl(u1, src), v2 = __shfl(u2, src);
        const double qa = __shfl(xq[q].w, src);
        if (slot < APW && b0 + slot < np) {
          const double g0 = floor(v0), g1 = floor(v1), g2 = floor(v2);
          double T0[P], T1[P], T2[P];
          bspline_weights<P>(v0 - g0, T0, nullptr);
          bspline_weights<P>(v1 - g1, T1, nullptr);
          bspline_weights<P>(v2 - g2, T2, nullptr);
          const int d = wrap_index((int)g0 - px, K0);
          double t0 = 0.0, t1 = 0.0;
#pragma unroll
          for (int j = 0; j < P; ++j) {
            t0 = j == d ? T0[j] : t0;
            t1 = j == j1 ? T1[j] : t1;
          }
          const int r1 = wrap_index((int)g1 - j1, K1) * K2;
          const double w01 = qa * t0 * t1;
#pragma unroll
          for (int j2 = 0; j2 < P; ++j2) atomicAdd(&pr[r1 + wrap_index((int)g2 - j2, K2)], w01 * T2[j2]);
        }
      }
    }
  }
  __syncthreads();
  double *o = part + ((size_t)pp * K0 + px) * K1 * K2;
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) o[e] = pr[e];
}

// plane x: the sum of its partial planes, then the z and y transforms (DIF)
__global__ __launch_bounds__(512) void k_pme_yz_fwd(MDView V, const double *__restrict__ part, int nparts) {
  extern __shared__ double2 pcx[];
  const int px = blockIdx.x, K1 = V.pk[1], K2 = V.pk[2];
  const size_t np = (size_t)K1 * K2, stride = (size_t)V.pk[0] * np;
  const double *pin = part + (size_t)px * np;
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) {
    double q = 0.0;
    for (int k = 0; k < nparts; ++k) q += pin[k * stride + e];
    pcx[plane_at(e / K2, e % K2, K2)] = make_double2(q, 0.0);
  }
  __syncthreads();
  lds_fft_lines<true>(pcx, K1, K2, V.ptw, V.ptw_n, [K2](int l, int k) { return plane_at(l, k, K2); });
  lds_fft_lines<true>(pcx, K2, K1, V.ptw, V.ptw_n, [K2](int l, int k) { return plane_at(k, l, K2); });
  double2 *g = V.pgrid + (size_t)px * np;
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) g[e] = pcx[plane_at(e / K2, e % K2, K2)];
}

// x lines (lpb per block, adjacent in memory): the x transform (DIF), then
// G conj(F) with G from the influence table in the same bit-reversed layout
// (e: the energy terms G |F|^2 instead, and done), then the x part of the
// second transform (DIT), back in natural x order.
__global__ __launch_bounds__(256) void k_pme_xline(MDView V, int lpb, double *__restrict__ e) {
  extern __shared__ double2 xbuf[];
  const int K0 = V.pk[0], nyz = V.pk[1] * V.pk[2];
  const int l0 = blockIdx.x * lpb, pitch = K0 + 1;   // one element of padding per line
  for (int t = threadIdx.x; t < lpb * K0; t += blockDim.x) {
    const int l = t % lpb, x = t / lpb;
    xbuf[l * pitch + x] = V.pgrid[(size_t)x * nyz + l0 + l];
  }
  __syncthreads();
  lds_fft_lines<true>(xbuf, lpb, K0, V.ptw, V.ptw_n, [pitch](int l, int k) { return l * pitch + k; });
  for (int t = threadIdx.x; t < lpb * K0; t += blockDim.x) {
    const int l = t % lpb, x = t / lpb;
    const size_t m = (size_t)x * nyz + l0 + l;
    const double G = V.pinf[m];
    const double2 F = xbuf[l * pitch + x];
    if (e) e[m] = G * (F.x * F.x + F.y * F.y);
    else xbuf[l * pitch + x] = make_double2(G * F.x, -G * F.y);
  }
  if (e) return;
  __syncthreads();
  lds_fft_lines<false>(xbuf, lpb, K0, V.ptw, V.ptw_n, [pitch](int l, int k) { return l * pitch + k; });
  for (int t = threadIdx.x; t < lpb * K0; t += blockDim.x) {
    const int l = t % lpb, x = t / lpb;
    V.pgrid[(size_t)x * nyz + l0 + l] = xbuf[l * pitch + x];
  }
}

// the y and z part of the second transform, plane by plane: bit-reversed (y, z)
// in, natural order out
__global__ __launch_bounds__(512) void k_pme_yz_back(MDView V) {
  extern __shared__ double2 pcy[];
  const int K1 = V.pk[1], K2 = V.pk[2];
  double2 *g = V.pgrid + (size_t)blockIdx.x * K1 * K2;
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) pcy[plane_at(e / K2, e % K2, K2)] = g[e];
  __syncthreads();
  lds_fft_lines<false>(pcy, K1, K2, V.ptw, V.ptw_n, [K2](int l, int k) { return plane_at(l, k, K2); });
  lds_fft_lines<false>(pcy, K2, K1, V.ptw, V.ptw_n, [K2](int l, int k) { return plane_at(k, l, K2); });
  for (int e = threadIdx.x; e < K1 * K2; e += blockDim.x) g[e] = pcy[plane_at(e / K2, e % K2, K2)];
}

// grid <- G(m) conj(F(m)); e (if given) receives G(m) |F(m)|^2, the energy terms
__global__ void k_pme_influence(MDView V, double *__restrict__ e) {
  const int ng = V.pk[0] * V.pk[1] * V.pk[2];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ng) return;
  const double G = V.pinf[m];
  const double2 F = V.pgrid[m];
  if (e) e[m] = G * (F.x * F.x + F.y * F.y);
  V.pgrid[m] = make_double2(G * F.x, -G * F.y);
}

// forces from Psi (the real part of the grid after the second transform):
// f_id = -2 q_i (K_d / L_d) sum_k Psi(k) dM(u_d - k_d) prod_{d' != d} M(u_d' - k_d'),
// 8 lanes per atom (lane j0 < p sums the slice k0 - j0, then a shuffle
// reduction), plus the excluded-pair correction
template <int P>
__global__ __launch_bounds__(256) void k_pme_gather(MDView V, const double4 *__restrict__ X) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = gid >> 3, j0 = gid & 7;
  const bool live = i0 < V.n;
  const int i = live ? i0 : V.n - 1;
  const double4 x = X[i];
  const double xs[3] = {x.x, x.y, x.z};
  double T[3][P], D[3][P];
  int k0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double u = V.pk[d] * xs[d] / V.box[d];
    const double fl = floor(u);
    k0[d] = (int)fl;
    bspline_weights<P>(u - fl, T[d], D[d]);
  }
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (j0 < P) {
    double t0 = 0.0, d0 = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      t0 = j == j0 ? T[0][j] : t0;
      d0 = j == j0 ? D[0][j] : d0;
    }
    const int g0 = wrap_index(k0[0] - j0, V.pk[0]) * V.pk[1];
    for (int j1 = 0; j1 < P; ++j1) {
      const int g01 = (g0 + wrap_index(k0[1] - j1, V.pk[1])) * V.pk[2];
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int j2 = 0; j2 < P; ++j2) {
        const double psi = V.pgrid[g01 + wrap_index(k0[2] - j2, V.pk[2])].x;
        a += psi * T[2][j2];
        b += psi * D[2][j2];
      }
      s0 += d0 * T[1][j1] * a;
      s1 += t0 * D[1][j1] * a;
      s2 += t0 * T[1][j1] * b;
    }
  }
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 8);
    s1 += __shfl_xor(s1, off, 8);
    s2 += __shfl_xor(s2, off, 8);
  }
  if (!live || j0 != 0) return;
  double fx = -2.0 * x.w * (V.pk[0] / V.box[0]) * s0;
  double fy = -2.0 * x.w * (V.pk[1] / V.box[1]) * s1;
  double fz = -2.0 * x.w * (V.pk[2] / V.box[2]) * s2;
  excluded_recip_force(V, X, i, x, fx, fy, fz);
  V.frec[i] = make_double4(fx, fy, fz, 0.0);
}

// each atom's half of its excluded pairs' correction -k_e q_i q_j erf(alpha r) / r into e[i]
__global__ void k_excl_energy(MDView V, const double4 *__restrict__ X, double *__restrict__ e) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V.n) return;
  const double4 xi = X[i];
  double u = 0.0;
  if (V.xptr) {
    const double L[3] = {V.box[0], V.box[1], V.box[2]};
    for (int q = V.xptr[i]; q < V.xptr[i + 1]; ++q) {
      const double4 xj = X[V.xj[q]];
      const double dx = min_img(xi.x - xj.x, L[0], 1.0 / L[0]);
      const double dy = min_img(xi.y - xj.y, L[1], 1.0 / L[1]);
      const double dz = min_img(xi.z - xj.z, L[2], 1.0 / L[2]);
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      u -= 0.5 * V.ke * xi.w * xj.w * erf(V.alpha * r) / r;
    }
  }
  e[i] = u;
}

// Ewald energy terms: w_k |S(k)|^2 per k into e[0, nk), and each atom's half
// of its excluded pairs' correction -k_e q_i q_j erf(alpha r) / r into e[nk + i]
__global__ void k_ewald_energy(MDView V, const double4 *__restrict__ X, const double2 *__restrict__ S,
                               double *__restrict__ e) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < V.nk) {
    const double2 sq = S[t];
    e[t] = V.kvec[t].w * (sq.x * sq.x + sq.y * sq.y);
  } else if (t < V.nk + V.n) {
    const int i = t - V.nk;
    const double4 xi = X[i];
    double u = 0.0;
    if (V.xptr) {
      const double L[3] = {V.box[0], V.box[1], V.box[2]};
      for (int q = V.xptr[i]; q < V.xptr[i + 1]; ++q) {
        const double4 xj = X[V.xj[q]];
        const double dx = min_img(xi.x - xj.x, L[0], 1.0 / L[0]);
        const double dy = min_img(xi.y - xj.y, L[1], 1.0 / L[1]);
        const double dz = min_img(xi.z - xj.z, L[2], 1.0 / L[2]);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        u -= 0.5 * V.ke * xi.w * xj.w * erf(V.alpha * r) / r;
      }
    }
    e[t] = u;
  }
}

// counts to doubles (the histogram of the allocation-free entry point)
__global__ void k_u64_to_double(const unsigned long long *__restrict__ a, double *__restrict__ b, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ void k_set_step(MDCtl *ctl, long long step) { ctl->step_base = step; }

// fill with a value (a kernel rather than a memset: safe under graph capture)
__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------- launchers
#define CHK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) return e_; } while (0)

// ---------------------------------------- allocation-free pair histogram
// Device scratch of md_rdf_noalloc: the counts (u64), then the histogram
// converted to doubles, MD_RDF_NOALLOC_MAX_BINS of each (256 KiB in all).
// Every device holds its own copy for the life of the process; all calls on
// one device share it. In host code the name is only a stand-in: kernels get
// the device address that hipGetSymbolAddress returned for that device.
static __device__ __align__(256) unsigned long long scratch[2 * MD_RDF_NOALLOC_MAX_BINS];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[MD_MAX_DEVICES] = {};
}  // namespace

// Once per device, with that device current (context creation): look up and
// keep the device address of the scratch array.
hipError_t rdf_scratch_setup(int dev) {
  if (dev < 0 || dev >= MD_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = p;
  return hipSuccess;
}

// device address of the scratch array on dev (nullptr before its setup)
unsigned long long *rdf_scratch_ptr(int dev) {
  if (dev < 0 || dev >= MD_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (unsigned long long *)g_scratch_ptr[dev];
}

// the pair histogram into the scratch array at sp (counts cleared first by a
// fill kernel), then converted to doubles in its second half
hipError_t launch_rdf_noalloc(const MDView &V, const double4 *X, const int *rep_off, int ta, int tb, double rmax,
                              int nbins, unsigned long long *sp, hipStream_t s) {
  if (!sp || nbins <= 0 || nbins > MD_RDF_NOALLOC_MAX_BINS) return hipErrorInvalidValue;
  const int nbk = (nbins + 255) / 256;
  hipLaunchKernelGGL(k_fill_u64, dim3(nbk), dim3(256), 0, s, sp, nbins, 0ull);
  CHK(hipGetLastError());
  hipLaunchKernelGGL(k_rdf, dim3((V.n + 255) / 256), dim3(256), 0, s, V, X, rep_off, ta, tb, rmax, nbins, sp);
  CHK(hipGetLastError());
  hipLaunchKernelGGL(k_u64_to_double, dim3(nbk), dim3(256), 0, s, sp, (double *)(sp + MD_RDF_NOALLOC_MAX_BINS),
                     nbins);
  return hipGetLastError();
}

hipError_t launch_local(const MDView &V, const MDProg &P, const double4 *Xs, double4 *Xd, hipStream_t s) {
  const int nb = (V.n + 255) / 256;
  hipLaunchKernelGGL(k_local, dim3(nb), dim3(256), 0, s, V, P, Xs, Xd);
  return hipGetLastError();
}

hipError_t launch_rebuild(const MDView &V, const double4 *X, int want, int slot, int forced, int autob,
                          double thr2, int pc, int ps, bool check_only, int count, hipStream_t s) {
  int nb = (V.n + 255) / 256;
  hipLaunchKernelGGL(k_cell_count, dim3(nb), dim3(256), 0, s, V, X, slot, forced, autob, thr2);
  CHK(hipGetLastError());
  if (check_only) return hipSuccess;
  hipLaunchKernelGGL(k_cell_scan, dim3(V.nrep), dim3(256), 0, s, V, slot, forced, autob, thr2, count);
  CHK(hipGetLastError());
  hipLaunchKernelGGL(k_cell_scatter, dim3(nb), dim3(256), 0, s, V, slot, forced, autob, thr2);
  CHK(hipGetLastError());
  size_t lds = sizeof(unsigned) * (size_t)(pc + 64 + ps + V.qimg);   // keys + queue margin, short keys, image queue
  hipLaunchKernelGGL(k_build, dim3(V.n), dim3(64), lds, s, V, X, want, slot, forced, autob, thr2, pc, ps);
  return hipGetLastError();
}

// whether the pair-force launch of this mode with the bonded blocks appended
// is resident in one round (then the bonded blocks hide beside the pair
// blocks; beyond that their registers cost the pair blocks occupancy)
bool force_fused_fits(const MDView &V, int mode) {
  const bool f32 = V.precision == MD_FP32_MIXED;
  const long long nb = mode == 0 ? ((long long)V.n * 8 + 255) / 256 : ((long long)V.n * 16 + 255) / 256;
  const long long nbb = (V.n + 255) / 256;
  int dev = 0, ncu = 0, bpc = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
  hipError_t e;
  if (mode == 0) e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_force_f<0, 8, true>, 256, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_force<0, 8, true>, 256, 0);
  else e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_force_f<1, 16, true>, 256, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_force<1, 16, true>, 256, 0);
  return e == hipSuccess && bpc > 0 && nb + nbb <= (long long)ncu * bpc;
}

hipError_t launch_force(const MDView &V, const double4 *X, int mode, bool with_bonded, hipStream_t s) {
  const bool f32 = V.precision == MD_FP32_MIXED;
  const int nbb = with_bonded ? (V.n + 255) / 256 : 0;   // bonded blocks after the pair blocks
  const dim3 blk(256);
  if (mode == 0) {
    const int nb = (int)(((long long)V.n * 8 + 255) / 256);
    const dim3 grid(nb + nbb);
    if (f32) {
      if (with_bonded) hipLaunchKernelGGL((k_force_f<0, 8, true>), grid, blk, 0, s, V, X, nb);
      else hipLaunchKernelGGL((k_force_f<0, 8, false>), grid, blk, 0, s, V, X, nb);
    } else {
      if (with_bonded) hipLaunchKernelGGL((k_force<0, 8, true>), grid, blk, 0, s, V, X, nb);
      else hipLaunchKernelGGL((k_force<0, 8, false>), grid, blk, 0, s, V, X, nb);
    }
  } else if (mode == 1) {
    const int nb = (int)(((long long)V.n * 16 + 255) / 256);
    const dim3 grid(nb + nbb);
    if (f32) {
      if (with_bonded) hipLaunchKernelGGL((k_force_f<1, 16, true>), grid, blk, 0, s, V, X, nb);
      else hipLaunchKernelGGL((k_force_f<1, 16, false>), grid, blk, 0, s, V, X, nb);
    } else {
      if (with_bonded) hipLaunchKernelGGL((k_force<1, 16, true>), grid, blk, 0, s, V, X, nb);
      else hipLaunchKernelGGL((k_force<1, 16, false>), grid, blk, 0, s, V, X, nb);
    }
  } else {   // long real part (no bonded blocks)
    const int nb = (int)(((long long)V.n * 16 + 255) / 256);
    if (f32) hipLaunchKernelGGL((k_force_f<2, 16, false>), dim3(nb), blk, 0, s, V, X, nb);
    else hipLaunchKernelGGL((k_force<2, 16, false>), dim3(nb), blk, 0, s, V, X, nb);
  }
  return hipGetLastError();
}

hipError_t launch_bonded(const MDView &V, const double4 *X, hipStream_t s) {
  int nb = (V.n + 255) / 256;
  hipLaunchKernelGGL(k_bonded, dim3(nb), dim3(256), 0, s, V, X);
  return hipGetLastError();
}

hipError_t launch_ke(const MDView &V, double *part, int *nblocks, hipStream_t s) {
  int nb = (V.n + 255) / 256;
  *nblocks = nb;
  hipLaunchKernelGGL(k_ke, dim3(nb), dim3(256), 0, s, V, part);
  return hipGetLastError();
}

hipError_t launch_pair_energy(const MDView &V, const double4 *X, int which, double *es, double *el,
                              hipStream_t s) {
  int nb = (V.n + 255) / 256;
  hipLaunchKernelGGL(k_pair_energy, dim3(nb), dim3(256), 0, s, V, X, which, es, el);
  return hipGetLastError();
}

hipError_t launch_bonded_energy(const MDView &V, const double4 *X, int nb, int na, double *e, hipStream_t s) {
  int nt = nb + na;
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bonded_energy, dim3((nt + 255) / 256), dim3(256), 0, s, V, X, nb, na, e);
  return hipGetLastError();
}

hipError_t launch_count_pairs(const MDView &V, const double4 *X, int which, double cut, unsigned long long *out,
                              hipStream_t s) {
  int nb = (V.n + 255) / 256;
  hipLaunchKernelGGL(k_count_pairs, dim3(nb), dim3(256), 0, s, V, X, which, cut, out);
  return hipGetLastError();
}

hipError_t launch_set_step(MDCtl *ctl, long long step, hipStream_t s) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, ctl, step);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// structure factors into S ([nk]) through the partials part ([ew_ranges * nk])
static hipError_t launch_sfac(const MDView &V, const double4 *X, double2 *part, double2 *S, hipStream_t s) {
  const size_t lds = ewald_lds_bytes(V.kmax, V.ew_ta);
  hipLaunchKernelGGL(k_sfac, dim3((V.nk + EW_KPB - 1) / EW_KPB, V.ew_ranges), dim3(256), lds, s, V, X, part);
  CHK(hipGetLastError());
  hipLaunchKernelGGL(k_sfac_sum, dim3((V.nk + 255) / 256), dim3(256), 0, s, V, part, S);
  return hipGetLastError();
}

// atom tile of the structure-factor launch (its tables within 60 KiB of LDS)
// and atom ranges: enough blocks to cover the device about four times over,
// each range a whole number of tiles
void ewald_ranges(int n, int nk, int kmax, int &ranges, int &apb, int &ta, int &krange) {
  ta = std::max(1, std::min(EW_TA, (60 * 1024 - 8 * EW_TA) / (16 * (5 * kmax + 3))));
  const int kc = (nk + EW_KPB - 1) / EW_KPB;
  const int tiles = (n + ta - 1) / ta;
  ranges = std::max(1, std::min(tiles, (1024 + kc - 1) / kc));
  apb = ((tiles + ranges - 1) / ranges) * ta;
  ranges = (n + apb - 1) / apb;
  // force launch: k-ranges of whole 256-vector chunks, about 1024 blocks in all
  const int ab = (n + 255) / 256, chunks = (nk + 255) / 256;
  const int nkr = std::max(1, std::min(chunks, (1024 + ab - 1) / ab));
  krange = ((chunks + nkr - 1) / nkr) * 256;
}

// reciprocal-space forces into V.frec; fpart: [ceil(nk / ew_krange) * n] partial forces
hipError_t launch_recip(const MDView &V, const double4 *X, double2 *part, double2 *S, double4 *fpart,
                        hipStream_t s) {
  CHK(launch_sfac(V, X, part, S, s));
  const int nkr = (V.nk + V.ew_krange - 1) / V.ew_krange;
  hipLaunchKernelGGL(k_recip_force, dim3((V.n + 255) / 256, nkr), dim3(256), 0, s, V, X, S, fpart);
  CHK(hipGetLastError());
  hipLaunchKernelGGL(k_recip_sum, dim3((V.n + 255) / 256), dim3(256), 0, s, V, X, fpart, nkr);
  return hipGetLastError();
}

hipError_t launch_ewald_energy(const MDView &V, const double4 *X, double2 *part, double2 *S, double *e,
                               hipStream_t s) {
  CHK(launch_sfac(V, X, part, S, s));
  hipLaunchKernelGGL(k_ewald_energy, dim3((V.nk + V.n + 255) / 256), dim3(256), 0, s, V, X, S, e);
  return hipGetLastError();
}

// three-dimensional transform: the three axes in turn, N / 2 threads per
// line and 256 / (N / 2) lines per block (N <= 512)
static hipError_t launch_fft3(const MDView &V, hipStream_t s) {
  for (int axis = 2; axis >= 0; --axis) {
    const int Na = V.pk[axis], half = Na / 2;
    const int lpb = std::max(1, 256 / half);
    const int nlines = V.pk[0] * V.pk[1] * V.pk[2] / Na;
    hipLaunchKernelGGL(k_fft_axis, dim3((nlines + lpb - 1) / lpb), dim3(lpb * half), sizeof(double2) * lpb * (Na + 1), s,
                       V.pgrid, V.ptw, V.ptw_n, V.pk[0], V.pk[1], V.pk[2], axis);
    CHK(hipGetLastError());
  }
  return hipSuccess;
}

// SPME: zeroed grid, spreading, transform, influence function (e: energy
// terms [NG] or NULL), and for forces the second transform and the gather
static hipError_t pme_to_influence(const MDView &V, const double4 *X, double *e, hipStream_t s) {
  const int ng = V.pk[0] * V.pk[1] * V.pk[2];
  const size_t plane = sizeof(double) * V.pk[1] * V.pk[2];
  if (plane <= 64 * 1024) {   // one block per mesh plane, the plane in LDS
    const dim3 gp(V.pk[0]);
    switch (V.porder) {
      case 4: hipLaunchKernelGGL(k_pme_spread_planes<4>, gp, dim3(256), plane, s, V, X); break;
      case 6: hipLaunchKernelGGL(k_pme_spread_planes<6>, gp, dim3(256), plane, s, V, X); break;
      default: hipLaunchKernelGGL(k_pme_spread_planes<8>, gp, dim3(256), plane, s, V, X); break;
    }
  } else {                    // larger planes: zeroed mesh and global atomics, 8 lanes per atom
    CHK(launch_fill_u64((unsigned long long *)V.pgrid, 2 * ng, 0ull, s));
    const dim3 ga((8 * V.n + 255) / 256);
    switch (V.porder) {
      case 4: hipLaunchKernelGGL(k_pme_spread<4>, ga, dim3(256), 0, s, V, X); break;
      case 6: hipLaunchKernelGGL(k_pme_spread<6>, ga, dim3(256), 0, s, V, X); break;
      default: hipLaunchKernelGGL(k_pme_spread<8>, ga, dim3(256), 0, s, V, X); break;
    }
  }
  CHK(hipGetLastError());
  CHK(launch_fft3(V, s));
  hipLaunchKernelGGL(k_pme_influence, dim3((ng + 255) / 256), dim3(256), 0, s, V, e);
  return hipGetLastError();
}

// fused path: spreading with the y, z transforms; the x line kernel (e:
// energy terms only, and stop)
static hipError_t pme_fused_forward(const MDView &V, const double4 *X, double *part, double *e, hipStream_t s) {
  if (!part) return hipErrorInvalidValue;
  const size_t plane = sizeof(double) * V.pk[1] * V.pk[2];
  const dim3 gp(V.pk[0], MD_PME_PARTS);
  switch (V.porder) {
    case 4: hipLaunchKernelGGL(k_pme_spread_part<4>, gp, dim3(256), plane, s, V, X, part); break;
    case 6: hipLaunchKernelGGL(k_pme_spread_part<6>, gp, dim3(256), plane, s, V, X, part); break;
    default: hipLaunchKernelGGL(k_pme_spread_part<8>, gp, dim3(256), plane, s, V, X, part); break;
  }
  CHK(hipGetLastError());
  hipLaunchKernelGGL(k_pme_yz_fwd, dim3(V.pk[0]), dim3(512), 2 * plane, s, V, part, MD_PME_PARTS);
  CHK(hipGetLastError());
  const int lpb = V.pk[0] >= 256 ? 8 : 16;   // K1 K2 >= 64 lines, a multiple of lpb
  hipLaunchKernelGGL(k_pme_xline, dim3(V.pk[1] * V.pk[2] / lpb), dim3(256), sizeof(double2) * lpb * (V.pk[0] + 1), s,
                     V, lpb, e);
  return hipGetLastError();
}

hipError_t launch_pme_forces(const MDView &V, const double4 *X, double *part, hipStream_t s) {
  if (pme_fused(V.pk)) {
    CHK(pme_fused_forward(V, X, part, nullptr, s));
    hipLaunchKernelGGL(k_pme_yz_back, dim3(V.pk[0]), dim3(512), sizeof(double2) * V.pk[1] * V.pk[2], s, V);
    CHK(hipGetLastError());
  } else {
    CHK(pme_to_influence(V, X, nullptr, s));
    CHK(launch_fft3(V, s));
  }
  const dim3 ga((8 * V.n + 255) / 256);   // 8 lanes per atom
  switch (V.porder) {
    case 4: hipLaunchKernelGGL(k_pme_gather<4>, ga, dim3(256), 0, s, V, X); break;
    case 6: hipLaunchKernelGGL(k_pme_gather<6>, ga, dim3(256), 0, s, V, X); break;
    default: hipLaunchKernelGGL(k_pme_gather<8>, ga, dim3(256), 0, s, V, X); break;
  }
  return hipGetLastError();
}

// energy terms: e[0, NG) = G |F|^2 per grid point, e[NG + i] = atom i's half of its excluded-pair correction
hipError_t launch_pme_energy(const MDView &V, const double4 *X, double *part, double *e, hipStream_t s) {
  const int ng = V.pk[0] * V.pk[1] * V.pk[2];
  if (pme_fused(V.pk)) CHK(pme_fused_forward(V, X, part, e, s));
  else CHK(pme_to_influence(V, X, e, s));
  hipLaunchKernelGGL(k_excl_energy, dim3((V.n + 255) / 256), dim3(256), 0, s, V, X, e + ng);
  return hipGetLastError();
}

hipError_t launch_rdf(const MDView &V, const double4 *X, const int *rep_off, int ta, int tb, double rmax,
                      int nbins, unsigned long long *hist, hipStream_t s) {
  int nb = (V.n + 255) / 256;
  hipLaunchKernelGGL(k_rdf, dim3(nb), dim3(256), 0, s, V, X, rep_off, ta, tb, rmax, nbins, hist);
  return hipGetLastError();
}
