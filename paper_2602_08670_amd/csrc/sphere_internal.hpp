// Internal interface of the spherical shallow-water path (sphere_kernels.hip,
// sphere_api.cpp).  Grid 2n x n cells; arrays are [component][row][column].
#pragma once

#include <hip/hip_runtime.h>

#include "fv_internal.hpp"

namespace sph {

// Device geometry, in the solver's precision (area also in double for the
// totals).
template <typename T> struct Geometry {
    T *cen;        // [3][n][2n] cell centres (unit vectors)
    T *nsum;       // [3][n][2n] sum over the cell's edges of outward normal times length
    T *inv_area;   // [n][2n]
    T *rate_fac;   // [n][2n] perimeter / (2 area): the CFL rate per unit wave speed
    double *area;  // [n][2n]
    T *xf;         // [10][n][2n] the cell's low x face: n[3], t[3], r[3], length
    T *yf;         // [10][n+1][2n] y face rows 0..n: n[3], t[3], r[3], length
};

template <typename T> struct CellArgs {
    const T *qs, *q0;
    T *out;
    Geometry<T> G;
    int n;
    T g, omega, a0, a1;
    double cfl, dt_fixed;
    fvk::Ctl *ctl;
    unsigned long long *rates;
    int rate_in, rate_out, rate_clear, last;
};

template <typename T> hipError_t geometry(const Geometry<T> &G, int n, hipStream_t st);
// One Runge-Kutta stage (a.qs -> a.out) in one launch over tiles of cells.
template <typename T> hipError_t stage(int flux, int recon, const CellArgs<T> &a, hipStream_t st);
template <typename T>
hipError_t rate(const T *q, const Geometry<T> &G, int n, double g, fvk::Ctl *ctl, unsigned long long *rates, int slot,
                hipStream_t st);
template <typename T>
hipError_t totals(const T *q, const double *area, int n, double g, double *partials, int max_blocks, double *out,
                  hipStream_t st);

}  // namespace sph
