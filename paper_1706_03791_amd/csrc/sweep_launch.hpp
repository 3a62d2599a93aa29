// Host-side dispatch of the sweep kernel instantiations.  Each element type
// and dimensionality lives in its own translation unit so the 96 kernel
// variants compile in parallel.
#pragma once

#include "common.hpp"
#include "sweep.hpp"
#include "wsweep.hpp"

namespace szh {

// Tile shapes (rows per workgroup) per element type and dimensionality.
template <typename T, int DIM> struct TileShape;
template <> struct TileShape<float, 3> { static constexpr int RZ = 16, RY = 16; };
template <> struct TileShape<double, 3> { static constexpr int RZ = 8, RY = 16; };
template <> struct TileShape<float, 2> { static constexpr int RZ = 1, RY = 256; };
template <> struct TileShape<double, 2> { static constexpr int RZ = 1, RY = 128; };
template <> struct TileShape<float, 1> { static constexpr int RZ = 1, RY = 256; };
template <> struct TileShape<double, 1> { static constexpr int RZ = 1, RY = 128; };

// Launches pass the body's LDS as dynamic LDS (raising the per-kernel limit
// when a variant needs more than 64 KiB).
template <typename T, typename CT, int DIM, int NL, bool COMP, int RZ, int RY>
inline void launch_sweep_variant(const SweepArgs& a, int grid, hipStream_t st) {
  constexpr size_t lds = SweepLds<T, CT, DIM, NL, COMP, RZ, RY>::BYTES;
  auto k = sweep_kernel<T, CT, DIM, NL, COMP, RZ, RY>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(RZ * RY), lds, st, a);
}

template <typename T, int DIM, int NL, bool COMP>
inline hipError_t launch_one(int cw, const SweepArgs& a, int grid, hipStream_t st) {
  constexpr int RZ = TileShape<T, DIM>::RZ, RY = TileShape<T, DIM>::RY;
  if (cw == 1)
    launch_sweep_variant<T, uint8_t, DIM, NL, COMP, RZ, RY>(a, grid, st);
  else
    launch_sweep_variant<T, uint16_t, DIM, NL, COMP, RZ, RY>(a, grid, st);
  return hipGetLastError();
}

template <typename T, int DIM>
inline hipError_t launch_sweep_t(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st) {
  switch (nl) {
    case 1: return comp ? launch_one<T, DIM, 1, true>(cw, a, grid, st) : launch_one<T, DIM, 1, false>(cw, a, grid, st);
    case 2: return comp ? launch_one<T, DIM, 2, true>(cw, a, grid, st) : launch_one<T, DIM, 2, false>(cw, a, grid, st);
    case 3: return comp ? launch_one<T, DIM, 3, true>(cw, a, grid, st) : launch_one<T, DIM, 3, false>(cw, a, grid, st);
    case 4: return comp ? launch_one<T, DIM, 4, true>(cw, a, grid, st) : launch_one<T, DIM, 4, false>(cw, a, grid, st);
  }
  return hipErrorInvalidValue;
}

// Defined in sweep_<type>_d<dim>.hip
hipError_t sweep_f32_d1(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_f32_d2(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_f32_d3(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_f64_d1(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_f64_d2(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st);
hipError_t sweep_f64_d3(int nl, bool comp, int cw, const SweepArgs& a, int grid, hipStream_t st);

// Wave-tiled sweep (one layer): waves per workgroup and z sub-rows per lane.
// 3D fields take NW waves of AZ sub-rows for each element type (two waves
// per SIMD; one 16-byte exchange record per step); 2D fields, a single z-row,
// take one wave per tile.
template <typename T> struct WaveShape;
template <> struct WaveShape<float> { static constexpr int NW = 8, AZ = 2; };
template <> struct WaveShape<double> { static constexpr int NW = 8, AZ = 1; };
inline int wave_az(int dtype, int ndim) {
  return ndim == 2 ? 1 : (dtype == SZ_F32 ? WaveShape<float>::AZ : WaveShape<double>::AZ);
}
inline int wave_nw(int dtype, int ndim) {
  return ndim == 2 ? 1 : (dtype == SZ_F32 ? WaveShape<float>::NW : WaveShape<double>::NW);
}

template <typename T, typename CT, bool COMP, bool DBG, int NW, int AZ>
inline void launch_wsweep_variant(const WArgs& a, int grid, hipStream_t st) {
  constexpr size_t lds = WSweepLds<T, NW, AZ>::BYTES;
  auto k = wsweep_kernel<T, CT, COMP, NW, AZ, DBG>;
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(NW * 64), lds, st, a);
}

template <typename T, int NW, int AZ>
inline void launch_wsweep_shape(bool comp, int cw, const WArgs& a, int grid, hipStream_t st) {
  if (comp && a.export_all) {
    if (cw == 1)
      launch_wsweep_variant<T, uint8_t, true, true, NW, AZ>(a, grid, st);
    else
      launch_wsweep_variant<T, uint16_t, true, true, NW, AZ>(a, grid, st);
  } else if (comp) {
    if (cw == 1)
      launch_wsweep_variant<T, uint8_t, true, false, NW, AZ>(a, grid, st);
    else
      launch_wsweep_variant<T, uint16_t, true, false, NW, AZ>(a, grid, st);
  } else {
    if (cw == 1)
      launch_wsweep_variant<T, uint8_t, false, false, NW, AZ>(a, grid, st);
    else
      launch_wsweep_variant<T, uint16_t, false, false, NW, AZ>(a, grid, st);
  }
}

template <typename T>
inline hipError_t launch_wsweep_t(bool comp, int cw, int nw, int az, const WArgs& a, int grid, hipStream_t st) {
  if (nw == WaveShape<T>::NW && az == WaveShape<T>::AZ)
    launch_wsweep_shape<T, WaveShape<T>::NW, WaveShape<T>::AZ>(comp, cw, a, grid, st);
  else if (nw == 1 && az == 1)
    launch_wsweep_shape<T, 1, 1>(comp, cw, a, grid, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
// Defined in wsweep_<type>.hip
hipError_t wsweep_f32(bool comp, int cw, int nw, int az, const WArgs& a, int grid, hipStream_t st);
hipError_t wsweep_f64(bool comp, int cw, int nw, int az, const WArgs& a, int grid, hipStream_t st);

inline void tile_shape(int dtype, int ndim, int& rz, int& ry) {
  if (dtype == SZ_F32) {
    rz = ndim == 3 ? TileShape<float, 3>::RZ : 1;
    ry = ndim == 3 ? TileShape<float, 3>::RY : (ndim == 2 ? TileShape<float, 2>::RY : TileShape<float, 1>::RY);
  } else {
    rz = ndim == 3 ? TileShape<double, 3>::RZ : 1;
    ry = ndim == 3 ? TileShape<double, 3>::RY : (ndim == 2 ? TileShape<double, 2>::RY : TileShape<double, 1>::RY);
  }
}

}  // namespace szh
