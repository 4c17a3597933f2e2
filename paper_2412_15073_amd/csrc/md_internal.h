// md_internal.h — host-side declarations shared by the kernel launchers and
// the C ABI implementation of libjumpmd.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/jumpmd.h"
#include "md_device.h"

#define OP_PHASE_O 1
#define OP_PHASE_J1 2
#define OP_PHASE_J2 3
#define OP_PHASE_C1 4
#define OP_PHASE_C2 5

#define MD_RDF_NOALLOC_MAX_BINS 16384   // bins of md_rdf_noalloc (its static device scratch)
#define MD_MAX_DEVICES 64

hipError_t launch_local(const MDView &V, const MDProg &P, const double4 *Xs, double4 *Xd, hipStream_t s);
hipError_t launch_chain(const MDView &V, const MDProg &P, const double4 *X, hipStream_t s);
size_t chain_lds_bytes_host(int G, int S, int precision);   // dynamic LDS of one k_chain wave
int chain_blocks_per_cu(int G, int S, int precision, int bw); // resident blocks of bw waves per CU (0: unknown)
hipError_t launch_rebuild(const MDView &V, const double4 *X, int want, int slot, int forced, int autob,
                          double thr2, int pc, int ps, bool check_only, int count, hipStream_t s);
hipError_t launch_force(const MDView &V, const double4 *X, int mode, bool with_bonded, hipStream_t s);
bool force_fused_fits(const MDView &V, int mode);   // pair + bonded blocks resident in one round
hipError_t launch_bonded(const MDView &V, const double4 *X, hipStream_t s);
hipError_t launch_ke(const MDView &V, double *part, int *nblocks, hipStream_t s);
hipError_t launch_pair_energy(const MDView &V, const double4 *X, int which, double *es, double *el,
                              hipStream_t s);
hipError_t launch_bonded_energy(const MDView &V, const double4 *X, int nb, int na, double *e, hipStream_t s);
hipError_t launch_rdf(const MDView &V, const double4 *X, const int *rep_off, int ta, int tb, double rmax,
                      int nbins, unsigned long long *hist, hipStream_t s);
hipError_t launch_count_pairs(const MDView &V, const double4 *X, int which, double cut, unsigned long long *out,
                              hipStream_t s);
hipError_t launch_set_step(MDCtl *ctl, long long step, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s);
hipError_t launch_theta_screen_err(double lo, double hi, int n, unsigned long long *out, hipStream_t s);
hipError_t rdf_scratch_setup(int dev);            // once per device, that device current
unsigned long long *rdf_scratch_ptr(int dev);     // device address of the static scratch on dev
hipError_t launch_rdf_noalloc(const MDView &V, const double4 *X, const int *rep_off, int ta, int tb, double rmax,
                              int nbins, unsigned long long *sp, hipStream_t s);
hipError_t launch_recip(const MDView &V, const double4 *X, double2 *part, double2 *S, double4 *fpart,
                        hipStream_t s);
void ewald_ranges(int n, int nk, int kmax, int &ranges, int &apb, int &ta, int &krange);
// part: MD_PME_PARTS x K0 K1 K2 doubles of partial planes (four-launch path only)
hipError_t launch_pme_forces(const MDView &V, const double4 *X, double *part, hipStream_t s);
// the four-launch particle-mesh Ewald path applies (a complex FP64 (y, z)
// plane fits 64 KiB of LDS); its influence table is then stored in the
// bit-reversed order of that path (position p along x, then the plane
// position (y', z'), each holding frequency bit-reverse of its index)
inline bool pme_fused(const int *K) { return K[1] * K[2] <= 4096; }
// atom ranges per mesh plane in the spreading of that path (partial planes summed after)
#define MD_PME_PARTS 4
hipError_t launch_pme_energy(const MDView &V, const double4 *X, double *part, double *e, hipStream_t s);
hipError_t launch_ewald_energy(const MDView &V, const double4 *X, double2 *part, double2 *S, double *e,
                               hipStream_t s);
