// Kernel parameter blocks and enums shared by the library's host launchers and its kernels.
#pragma once
#include <stdint.h>

#define HX_CART 0
#define HX_SPH 1
#define HX_HLL 0
#define HX_HLLC 1
#define HX_LIM_NONE 0
#define HX_LIM_MINMOD 1
#define HX_LIM_VANLEER 2
#define HX_LIM_VANALBADA 3
#define HX_LIM_MLP 4
#define HX_BC_PERIODIC 0
#define HX_BC_TRANSMISSIVE 1
#define HX_BC_REFLECTIVE 2
#define HX_GRAV_NONE 0
#define HX_GRAV_UNIFORM 1
#define HX_GRAV_POINT 2
#define HX_GRAV_POINT_MONOPOLE 3

namespace hx {

// Per-axis geometry tables (FP64, device), all indexed by cell index + ng on active axes
// (ghost cells included), by 0 on inactive axes:
//   cm, cp : the upper face's extrapolation distance over the left / right centre distance (scaled
//            one-sided differences: the limited upper face increment is limiter(cm dm, cp dp))
//   kap    : the lower face's extrapolation distance over the upper one (1 with face-midpoint
//            centres; with volume centroids (x_c - x_-) / (x_+ - x_c))
//   w      : coordinate width of the cell's image (dx; dr, dtheta, dphi)
// Spherical extras, indexed the same way:
//   rabs   : |r_c| of the image cell (axis 0),  sabs : |sin theta_c| of the image cell (axis 1)
// and interior-only tables (indexed by interior index):
//   rf[n1+1] r faces, vr[n1] (r+^3-r-^3)/3, hr[n1] (r+^2-r-^2)/2, ct[n2] cos th- - cos th+,
//   sf[n2+1] sin of theta faces.
struct Geo {
    const double* cm[3];
    const double* cp[3];
    const double* kap[3];
    const double* w[3];
    const double* rabs;
    const double* sabs;
    const double* rf;
    const double* vr;
    const double* hr;
    const double* ct;
    const double* sf;
};

struct SweepParams {
    const void* U;       // U^n, SoA [nvar][n3][n2][n1], FP64 or FP32
    void* Unew;          // U^{n+1}, same layout
    int n[3];
    int ng;
    long long plane;     // n1*n2*n3
    int bc[3][2];
    double gamma;
    double dt_host;
    const double* dt_dev;  // if non-null, the step reads dt here
    int limiter;
    int riemann;
    int gravity;
    double g0[3];
    const double* gr;    // radial acceleration per interior r index (point / monopole)
    Geo geo;
    int* flag;           // set to 1 when a non-physical state is met
    double* dtpart;      // per-workgroup maximum CFL rate of U^{n+1}
    int kz;              // z planes per block (3D)
    const float* mlp;    // learned limiter weights (FP32 master copy)
    double de_eps;       // criterion of the internal-energy monitor's blend factor
    double eos_R;        // gas + radiation EoS: specific gas constant and radiation constant
    double eos_arad;
    int ni;              // 56Ni decay heating: field index (5 + scalar) of rho f_Ni, or -1 (off)
    double ni_Q[2];      // energy per decay of 56Ni and 56Co
    double ni_tau[2];    // lifetimes of 56Ni and 56Co
    double ni_m;         // mass of a 56Ni nucleus
    const double* t_in;  // the decay clock at the start of the step (advanced after the sweep)
    int centroid;        // 1: reconstruction about the volume centroids of spherical cells
};

}  // namespace hx
