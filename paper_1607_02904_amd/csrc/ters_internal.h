// Host-side internals of libtersoff shared by the C-ABI layer and the kernel
// launchers.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "tersoff.h"

namespace ters {

#define TERS_HIP_TRY(expr)                                              \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) throw HipError(e_, #expr, __FILE__, __LINE__); \
  } while (0)

struct HipError {
  hipError_t code;
  std::string what;
  HipError(hipError_t c, const char *expr, const char *file, int line)
      : code(c), what(std::string(hipGetErrorString(c)) + " in " + expr + " (" + file + ":" +
                      std::to_string(line) + ")") {}
};

struct StatusError {
  ters_status code;
  std::string what;
  StatusError(ters_status c, std::string w) : code(c), what(std::move(w)) {}
};

// Grow-only device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) TERS_HIP_TRY(hipFree(p));
    p = nullptr;
    bytes = 0;
    TERS_HIP_TRY(hipMalloc(&p, b));
    bytes = b;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Per-configuration geometry for neighbour binning (device copy).
struct ConfDesc {
  double box[3];
  double inv_box[3];
  int32_t nc[3];      // cells per axis (1, or >= 3)
  int32_t cell_off;   // first global cell of this configuration
  int32_t atom_off;   // first atom
  int32_t natoms;
};

// Device error word bits (latched by kernels, read at sync points).
enum : uint32_t {
  kErrNlistOverflow = 1u,
  kErrNotFinite = 2u,
  kErrTooManyInCutoff = 4u,
  kErrListAsymmetric = 8u,
  kErrBadType = 16u
};

// One-pass scans of the list build: the cell pass takes tiles of kCellTile
// cells, the slot scan tiles of kSlotTile atoms.  lb_words(m, n): 8-byte
// words of scan state for m = cells + 1 and n atoms (one word of two ticket
// counters, then one flag per tile of each scan).
constexpr int64_t kCellTile = 1024, kSlotTile = 4096;
constexpr int kCellBucket = 8;  // atoms per cell held in the cell's bucket
constexpr int64_t lb_words(int64_t m, int64_t n) {
  return 1 + (m + kCellTile - 1) / kCellTile + (n + 1 + kSlotTile - 1) / kSlotTile;
}

// Neighbour list state.  One list per configuration set (a single system is
// a set of one).
struct NList {
  int32_t n = 0, cap = 0, nconf = 0;
  int64_t ncell = 0;
  double rlist = 0.0, skin = 0.0;
  double box_max = 0.0;  // longest box side of the set (rounding margin of the FP32 build)
  bool small_axis = false;  // some configuration has an axis of fewer than 3 cells
  bool valid = false;
  std::vector<ConfDesc> conf_h;
  DevBuf conf;        // ConfDesc[nconf]
  DevBuf conf_of;     // int32[n] (only for nconf > 1)
  DevBuf count;       // int32[n]: row lengths, by cell-order position
  DevBuf list;        // int32[n][cap]: row t = neighbours (atoms) of the atom at position t
  DevBuf order;       // int32[n]: atoms in cell order
  DevBuf order_u;     // int32[n]: the atoms of crowded cells before their order is fixed
  DevBuf cell_count;  // int32[ncell + 1]: atoms per cell during a build, zero between builds
  DevBuf cell_bucket; // int32[ncell][kCellBucket]: the first atoms of each cell
  DevBuf cell_next;   // int32[n]: the next atom of the atom's overflow list, or -1
  DevBuf cell_head;   // int32[ncell + 1]: first atom of each overflow list, -1 if empty
  DevBuf cell_start;  // int32[ncell + 1]
  DevBuf lbstate;     // uint64[lb_words(ncell + 1, n)]: one-pass scan state
  DevBuf xref;        // double[n][3]
  DevBuf maxcount;    // int32[1]: longest row of the last build if longer than cap, else 0
  DevBuf rev;         // int32[n][cap]: incoming force slot at j of row entry (t, j)
  DevBuf xs;          // float4[n]: positions at build time, in cell order, wrapped into the box
                      // (FP32), atom index in the fourth word
  DevBuf pos;         // int32[n]: position of each atom in the cell order (inverse of order)
  DevBuf cell_at;     // int32[n]: cell of the atom at each cell-order position
  DevBuf plist;       // int32[n][cap]: positions of the row entries (list build and reverse map)
  DevBuf srange;      // int2[n]: (soff[a], soff[a + 1]) of the atom a at each cell-order position
  DevBuf srange_a;    // int2[n]: the same by atom, (soff[a], soff[a + 1])
  DevBuf soff;        // int32[n + 1]: first incoming force slot of each atom (atom order)
};

// Forward / adjoint launch description.
// The list rows (count, list, rev) are indexed by cell-order position and
// hold atoms; order maps a position to its atom, which indexes the per-atom
// arrays (x, type, fbar, conf_of and the outputs).
struct FwdArgs {
  int32_t n;
  const double *x;         // [n][3] positions, by atom
  const int32_t *type;     // [n] types, by atom
  const double *fbar;      // adjoint direction, by atom (dual kernels) or null
  const ConfDesc *conf;    // device
  const int32_t *conf_of;  // configuration id by atom, or null (single configuration)
  const int32_t *order;    // cell-order position -> atom
  const int32_t *count;
  const int32_t *list;
  int32_t cap;
  int32_t ntypes;
  const void *kparam;      // KParam<B>[ntypes^3]
  const void *filt2;       // B[ntypes^2]: squared filter radius per (ti, tk)
  int32_t cut_consistent;  // 1 if the k-cutoff never depends on tj
  int32_t kmax;
  int32_t no_filter;       // wavefront schedule: every list entry takes a lane (ablation)
  uint32_t flags;
  double *forces;          // [n][3] (atomic accumulate) or null
  double *e_atom;          // [n] or null
  double *partials;        // [nblocks][partial_stride] energy / virial (per config if batched)
  double *pgrad;           // [ntypes^3][14] accumulated, or null
  double ebar;             // adjoint: scalar cotangent of E (single system)
  const double *ebar_conf; // adjoint: per-configuration cotangent (batch) or null
  double *xgrad;           // adjoint output [n][3]
  // owner-gather mode (no atomics): when fslot is set, the force that the
  // terms rooted at the atom at position t exert on its list neighbour j
  // (slot s of row t) goes to j's incoming slot fslot[rev[t*cap + s]*3 ..]
  // (zero when the pair is outside the cutoff) and the force on the atom
  // itself to fown[a*3 ..] (a = order[t], the atom); the incoming forces of
  // atom a then sit contiguously in slots [soff[a], soff[a + 1]) for the gather.
  // Slots hold the kernel's base type: FP64, or FP32 in the mixed path.
  void *fslot;
  double *fown;
  const int32_t *rev;
  int32_t *clear_flag;     // set to 0 by the kernel (molecular dynamics) or null
  uint32_t *err;
  // persistent form of the wavefront schedule (batches): chunks (first
  // cell-order position, atoms), items[0, qbound[8]), split into eight work
  // queues; queue[x] counts what has been taken of [qbound[x], qbound[x + 1])
  // and starts at 0.  Null: one chunk per wavefront from its workgroup id.
  const int2 *items;
  const int32_t *qbound;
  int32_t *queue;
  int32_t nitems;          // persistent form: items (qbound[8]); the launch takes at most
                           // the workgroups that these keep busy
  int32_t grid;            // persistent form: workgroups of the launch (at most)
  int32_t grab;            // persistent form: items per atomic take (0: static shares)
};

// launchers (implemented in the .hip files)
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, const int32_t *cond, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
// type (device [n], may be null) is checked against [0, ntypes) by the binning
// pass, which latches kErrBadType
void nlist_build(NList &nl, const double *x, const int32_t *type, int ntypes, const int32_t *cond,
                 uint32_t *err, hipStream_t s, int64_t *rebuild_counter = nullptr);
void nlist_check(const NList &nl, const double *x, int32_t *flag, hipStream_t s);
// F[a] (+)= fown[a] + sum of the incoming slots fslot[soff[a] .. soff[a + 1])
// (the range read from srange_a)
// (FP32 slots when slot_f32), summed in FP64 in slot order
void launch_gather(const NList &nl, const void *fslot, bool slot_f32, const double *fown,
                   double *F, int accumulate, hipStream_t s);
void launch_forward(const FwdArgs &a, int precision, int atoms_per_block, int nblocks_out[1],
                    hipStream_t s);
void launch_adjoint(const FwdArgs &a, int precision, int atoms_per_block, hipStream_t s);
int forward_blocks(int n, int atoms_per_block);
// wavefront schedule: atoms per wavefront (<= 32)
void launch_forward_wave(const FwdArgs &a, int precision, int atoms_per_wave, hipStream_t s);
void launch_adjoint_wave(const FwdArgs &a, int precision, int atoms_per_wave, hipStream_t s);
int wave_blocks(int n, int atoms_per_wave, bool param_grad);
// persistent form: workgroups that fill the device at the kernel's occupancy
int wave_persistent_grid(int precision, bool adjoint, bool multi_species);
// persistent form: workgroups launched for nitems items taken grab at a time,
// at most grid (pg: the parameter-gradient kernel's workgroup size)
int wave_persistent_launch(int grid, int nitems, int grab, bool pg);
// pair potential (truncated Lennard-Jones) over the list: one thread per atom
// in cell order, own forces only (full list, no atomics)
struct PairArgs {
  int32_t n;
  const double *x;         // [n][3] positions, by atom
  const ConfDesc *conf;    // the configuration (single system)
  const int32_t *order, *count, *list;
  int32_t cap;
  double eps, sigma, rc2;
  double *forces;          // [n][3] or null
  int32_t accumulate;
  double *partials;        // [blocks][8]: energy, virial
};
void launch_pair_lj(const PairArgs &p, int precision, hipStream_t s);
int pair_blocks(int n);
// thread-per-atom schedule (forward only, FP64 atomic scatter of the forces)
void launch_forward_thread(const FwdArgs &a, int precision, hipStream_t s);
int thread_blocks(int n);
void launch_reduce_partials(const double *partials, int nblocks, int stride, double *energy,
                            double *virial, int accumulate, hipStream_t s,
                            double *trace = nullptr, int32_t *step = nullptr);
// species outside [0, nt) read mass[0] (the list build reports them)
void launch_vv_first(int n, double *x, double *v, double *f, const int32_t *type,
                     const double *mass, int nt, double dt, const NList &nl, int32_t *flag, int zero_f,
                     hipStream_t s);
void launch_vv_second(int n, double *v, const double *f, const int32_t *type, const double *mass,
                      int nt, double dt, int32_t *flag, hipStream_t s);
// molecular dynamics, owner-gather mode: the gather above and the second half
// kick of this step, then (do_next) the first half kick, drift and rebuild test
// of the next; when trace is set, the force kernel's energy partials are also
// summed (fixed order) into energy[0] and trace[*step], and *step advances;
// energy points to a zero-initialised scratch of 8 + 16 doubles and a counter
void launch_vv_gather_kick_drift(const NList &nl, double *x, double *v, double *F,
                                 const void *fslot, bool slot_f32, const double *fown,
                                 const int32_t *type, const double *mass, int nt, double dt,
                                 int32_t *flag, int do_next, const double *partials, int nblocks,
                                 double *energy, double *trace, int32_t *step, hipStream_t s);

}  // namespace ters
