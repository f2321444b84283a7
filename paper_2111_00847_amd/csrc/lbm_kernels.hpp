// lbm_kernels.hpp -- host-side launchers of the gfx950 kernels.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

// nsteps levels; `copy`: the host's guess of the copy holding the state on
// entry, updated to where the launches leave it
template <typename T>
hipError_t launch_step(const KParams<T>& P, char* state, const Layout& L, int64_t nsteps, hipStream_t s,
                       int ty, int by, int& copy);
// two levels of the plain Allen-Cahn step in one launch (lbm_step2.hip)
template <typename T>
void launch_step2(const KParams<T>& P, char* state, const Layout& L, hipStream_t s);
// the Allen-Cahn step (either gradient scheme, not the corrected model) on a
// lattice of at least one tile per CU whose copy fits 32-bit offsets: two
// levels per launch
bool two_level_path(const Layout& L, int nx, int ny, int pf, int model, int grad);
template <typename T>
hipError_t launch_moments(const KParams<T>& P, const char* state, const Layout& L, T* phi, T* u, T* p,
                          hipStream_t s);
template <typename T>
hipError_t launch_init(const KParams<T>& P, char* state, const Layout& L, const T* phi0, const T* u0,
                       const T* p0, int dtype, hipStream_t s);
template <typename T>
hipError_t launch_hydrostatic(const KParams<T>& P, const T* phi0, T* p0, hipStream_t s);
template <typename T>
hipError_t launch_import(const KParams<T>& P, char* state, const Layout& L, const T* f, const T* g,
                         const T* hist, int64_t step, int dtype, hipStream_t s);
template <typename T>
hipError_t launch_export(const KParams<T>& P, const char* state, const Layout& L, T* f, T* g, T* hist,
                         hipStream_t s);
// the Allen-Cahn step / moments with the local gradient scheme (lbm_local.hip)
template <typename T, int MODE>
void launch_local(const KParams<T>& P, char* state, const Layout& L, hipStream_t s, T* phi, T* u, T* p);
template <typename T>
hipError_t launch_diagnostics(const KParams<T>& P, const char* state, const Layout& L, double* host_out,
                              hipStream_t s);

}  // namespace lbm
