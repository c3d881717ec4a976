// Kernel argument blocks and launchers of the MI355X PIC-MCC library.
#pragma once
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {

struct PushArgs {
    DevPtrs d;
    int32_t diag;                 // accumulate electron energy deposit and EEPF
    float eepf_inv_bin;           // 1 / bin width (eV)
    int32_t nodes_max_dyn, cells_max_dyn;
};

// The events kernel: the push's events of a step (collisions, renewals,
// secondary emission) with the push's tile shape.
constexpr int kEvThreads = 256;
struct EvArgs {
    DevPtrs d;
    int32_t T;                    // particles of the push's tile
    int32_t push_grid;            // the push's workgroups (each recorded its own tile range's events)
    int32_t births_per_tile;      // staging slots of a tile
    int32_t diag;
    float eepf_inv_bin;
};

// finalize modes
constexpr int kFinStep = 0;       // append births, deposit -> field at t^{n+1}, step++
constexpr int kFinSolve = 1;      // deposit -> field at t = step dt, no state change but the field
constexpr int kFinExternal = 2;   // field of rho_ext at t_ext into phi_out / e_out only

struct FinArgs {
    DevPtrs d;
    int32_t mode;
    int32_t diag;
    int32_t only_b;               // -1: all discharges (grid = B), else this one (grid = 1)
    int32_t births_per_tile;      // staging slots of a push tile (0: the step cannot have births)
    float eepf_inv_bin;           // 1 / bin width (eV) of the bulk electron energy distribution
    double t_ext;
    const double* rho_ext;
    double* phi_out;
    double* e_out;
};

struct LoadArgs {
    DevPtrs d;
    int32_t b, s;
    int64_t n;
    int32_t load;
    double vth, drift[3];
    double perturb_eps;
    int32_t perturb_mode;
};

struct ProfileArgs {
    DevPtrs d;
    int32_t b, s, m;
    int64_t n;
    const double* dens;           // [m] density at the points
    const double* cum;            // [m] integral of the density from 0 to each point
    const double* temp;           // [m] temperature (eV) at the points
    double e_over_m;              // e / m of the species
};

hipError_t launch_profile_load(const ProfileArgs& a, hipStream_t st);
hipError_t launch_push(const PushArgs& a, int ppt, int threads, bool general, bool fuse, int64_t grid,
                       hipStream_t st);
// whether a push of this shape can do its workgroups' own events
bool push_fusable(int ppt, int threads, bool general);
void push_shape(int& ppt, int& threads, bool general);
hipError_t launch_events(const EvArgs& a, int64_t grid, hipStream_t st);
int events_occupancy();
hipError_t launch_finalize(const FinArgs& a, hipStream_t st);
hipError_t launch_load(const LoadArgs& a, hipStream_t st);
hipError_t launch_deposit(const DevPtrs& d, int only_b, int64_t max_count, hipStream_t st);
hipError_t launch_halfstep(const DevPtrs& d, int only_b, int64_t max_count, hipStream_t st);
hipError_t launch_sort(const DevPtrs& d, int s, int64_t max_tiles, void* scratch, size_t scratch_bytes,
                       hipStream_t st);
hipError_t launch_compact(const DevPtrs& d, int64_t max_tiles, int n_cu, hipStream_t st);
// population control of one species (then a compaction); see pic_thin
hipError_t launch_thin(const DevPtrs& d, int32_t species, int64_t above, int64_t keep, int64_t max_count,
                       int64_t max_tiles, int n_cu, hipStream_t st);
int64_t compact_tiles_for(int64_t padded_count);
size_t sort_scratch_bytes(int64_t max_tiles, int B, int cells_max);
int64_t sort_tiles_for(int64_t padded_count);
size_t push_lds_bytes(int n_nodes, int n_cells, int diag);
int push_occupancy(int ppt, int threads, bool general, bool fuse, size_t lds);

}  // namespace pic
