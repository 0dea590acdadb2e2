// Fragmentation of the collapsed medium into halos (section "Fragmentation"): host-side
// interface of fragment.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace pin {

struct FragParams {
  double fa, fra, fs, fm, frm;   // eq. accretion and eq. merging constants (Table 1)
};

// Device workspace of one fragmentation call on an N^3 grid (owned by the plan, kept between
// calls) and the host tables it needs.
struct FragWorkspace {
  size_t vol = 0;
  void* block = nullptr;          // one allocation holding everything below
  size_t bytes = 0;
  uint64_t* keys[2] = {nullptr, nullptr};
  int32_t* vals[2] = {nullptr, nullptr};
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  int32_t* parent = nullptr;
  int32_t* hn = nullptr;
  double* hs = nullptr;           // [6][vol]: sums of offsets (3) and of displacements (3)
  unsigned long long* res_cell = nullptr;
  unsigned long long* res_halo = nullptr;
  int32_t* items = nullptr;       // per window slot: count + up to 6 halo ids
  int32_t* ctl = nullptr;         // head, next head, error, participants, halos, selected, mergers, overflow
  unsigned long long* ev_key = nullptr;  // merger events: (order position << 8 | pair), capacity vol
  double* ev_f = nullptr;                // F of the particle whose step merged
  int32_t* ev_ids = nullptr;             // keep, gone, N_keep before, N_gone
  double* rtab = nullptr;         // halo radius for N_h = 1..kRadiusTable
  double* stab = nullptr;         // sigma(R) nodes
  int stab_n = 0;
  double s_r0 = 0, s_step = 0;
  double s_for[4] = {0, 0, 0, 0};   // box, amplitude, gamma, ns the nodes were computed for
  int32_t* host_ctl = nullptr;    // pinned mirror of ctl
  int n_halos = -1;               // halos of the last fragment_run (-1: none yet)
  int n_mergers = 0;              // its merger events
  int n = 0;                      // its grid size
};

// Bytes of the workspace for an N^3 grid.
size_t fragment_workspace_bytes(int n);

// Allocate (first call) and fill the radius table and the sigma nodes (top-hat rms of the linear
// field at z = 0, 64 nodes per octave in R from the radius of one particle; recomputed only when
// the box or the spectrum changes); returns on completion.
void fragment_prepare(FragWorkspace& w, int n, double box, double amplitude, double gamma, double ns,
                      hipStream_t s);
void fragment_free(FragWorkspace& w);

// Run the fragmentation: F [vol] and v [3][vol] of the plan's precision (v in Mpc/h, converted to
// grid units with uscale = N / L); label [vol] and optional halo_size [vol] are written.  Returns
// the number of halos.  Synchronous: the rounds are driven from the host.
int fragment_run(FragWorkspace& w, bool fp64, int n, const void* F, const void* v, double uscale, double f_min,
                 const FragParams& prm, int32_t* label, int32_t* halo_size, hipStream_t s);

// Catalogue of the last fragment_run: for each halo in increasing id, its id, N_h, Lagrangian
// centre of mass (founder + mean offset, wrapped into [0, N), times cell) and mean displacement
// (times cell), centre and disp [3][capacity] float64.  Synchronous; returns the halo count.
int fragment_catalog(FragWorkspace& w, double cell, int32_t* id, int32_t* nh, double* centre, double* disp,
                     int capacity, hipStream_t s);

// Merger history of the last fragment_run, in the order the mergers happened: F of the particle
// that caused each, the kept and the absorbed halo ids and their N_h before the merger.  Device
// outputs of `capacity` entries; synchronous; returns the number of mergers.
int fragment_mergers(FragWorkspace& w, double* f, int32_t* keep, int32_t* gone, int32_t* n_keep, int32_t* n_gone,
                     int capacity, hipStream_t s);

}  // namespace pin
