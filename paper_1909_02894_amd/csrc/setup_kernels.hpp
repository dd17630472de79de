// setup_kernels.hpp -- parameters and host launchers of the table, conversion
// and reduction kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace dirac {

struct SetupAxisParams {
    int n;
    double a, c, dt;
    int pml_width, pml_type;
    double sigma0, ctheta;
    int fp32;
    int k_printed; // symbol of eq. (step2bis) as printed: K (1 - (c dt xi)^2)
    void* inv_s;   // n reals
    void* K;       // n complex: (cos, sin)(c dt xi) / n
    void* D;       // n reals: xi / n
    void* tw;      // n complex: exp(-2 pi i k / n)
};

struct SetupPointParams {
    int n1, n2;
    double a1, a2, dt, c, m;
    int kind, spin;
    double bump_A, bump_s;
    const double* fields;   // FIELDS: 6 planes (phi, psi, phi_x, phi_y, psi_x, psi_y)
    int pml_width, pml_type;
    double sigma0, ctheta;
    int fp32;
    void* a_out;            // per point a (or null)
    void* E_out;            // per point (e0 re, e0 im, e1 re, e1 im) (or null)
    void* da_out;           // per point (d_x a, d_y a) (or null)
    const double* em_planes;// electromagnetic profiles V, A_x, A_y (3 FP64 planes) or null
    double charge;          // e
    void* em_out;           // per point (sx, sy, wz, qx, qy, q0, a, 0) (or null)
    double* obs_em;         // 3 FP64 planes: e c a A_x, e c a A_y, e V (or null)
    double* obs;            // 5 planes: w, c a, gx, gy, V
    double* partial;        // 3 doubles per workgroup of 256
};

hipError_t launch_setup_axis(const SetupAxisParams& p, hipStream_t s);
hipError_t launch_setup_points(const SetupPointParams& p, double* fold_out, hipStream_t s);
// out[i][j] = in[j][i] for an n2 x n1 row-major array of `elem`-byte (4 or 8) values.
hipError_t launch_transpose(const void* in, void* out, int n1, int n2, int elem, hipStream_t s);
hipError_t launch_c128_to_f32(const double* src, float* dst, size_t count, hipStream_t s);
hipError_t launch_f32_to_c128(const float* src, double* dst, size_t count, hipStream_t s);
hipError_t launch_reduce_partials(const double* part, int nparts, double* out, hipStream_t s);

}  // namespace dirac
