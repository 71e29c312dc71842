// sidm_host.hpp -- the static analytic host potential (Sec. 4.1): an NFW halo
// (Eq. nfw_potential), and for the Milky-Way host also a Hernquist bulge
// (Eq. hernquist_potential) and four Miyamoto-Nagai discs in the host's z = 0
// plane (Eq. disk_potential).  Positions relative to the host centre.
#pragma once

#include "sidm_internal.hpp"

namespace sidm {

// NFW: Phi = -K ln(1 + s)/r with s = r/r_s, K = 4 pi G rho_s r_s^3; the force
// follows from the enclosed mass, a = -K [ln(1+s) - s/(1+s)] d / r^3 (series in
// s below 1e-4).
__device__ inline void nfw_field(const HaloDev& H, double dx, double dy, double dz, double& ax,
                                 double& ay, double& az, double& phi)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) {
        ax = ay = az = 0.0;
        phi = -H.host_K / H.host_r_s;
        return;
    }
    const double r = sqrt(r2);
    const double s = r / H.host_r_s;
    const double l1p = log1p(s);
    double mu;
    if (s < 1e-4) mu = s * s * (0.5 - s * (2.0 / 3.0 - s * (0.75 - 0.8 * s)));
    else mu = l1p - s / (1.0 + s);
    const double f = -H.host_K * mu / (r2 * r);
    ax = f * dx; ay = f * dy; az = f * dz;
    phi = -H.host_K * l1p / r;
}

// Hernquist: Phi = -GM / (r + a), a = -GM d / (r (r + a)^2).
__device__ inline void hernquist_field(double GM, double a, double dx, double dy, double dz,
                                       double& ax, double& ay, double& az, double& phi)
{
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    phi = -GM / (r + a);
    if (r == 0.0) {
        ax = ay = az = 0.0;
        return;
    }
    const double f = -GM / (r * (r + a) * (r + a));
    ax = f * dx; ay = f * dy; az = f * dz;
}

// Miyamoto-Nagai: Phi = -GM / D, D^2 = R^2 + (a + zeta)^2, zeta = sqrt(z^2 + b^2);
// a = -GM (x, y, z (a + zeta) / zeta) / D^3.
__device__ inline void disk_field(double GM, double a, double b, double dx, double dy, double dz,
                                  double& ax, double& ay, double& az, double& phi)
{
    const double zeta = sqrt(dz * dz + b * b);
    const double s = a + zeta;
    const double D2 = dx * dx + dy * dy + s * s;
    const double D = sqrt(D2);
    phi = -GM / D;
    const double f = -GM / (D2 * D);
    ax = f * dx;
    ay = f * dy;
    az = zeta > 0.0 ? f * dz * s / zeta : 0.0;
}

// Total host acceleration and potential at p.
__device__ inline void host_field(const HaloDev& H, double px, double py, double pz, double& ax,
                                  double& ay, double& az, double& phi)
{
    const double dx = px - H.host_c[0], dy = py - H.host_c[1], dz = pz - H.host_c[2];
    ax = ay = az = phi = 0.0;
    if (H.host_kind == 0) return;
    if (H.host_K != 0.0) nfw_field(H, dx, dy, dz, ax, ay, az, phi);
    if (H.host_kind != 2) return;
    double gx, gy, gz, gp;
    if (H.hern_GM != 0.0) {
        hernquist_field(H.hern_GM, H.hern_a, dx, dy, dz, gx, gy, gz, gp);
        ax += gx; ay += gy; az += gz; phi += gp;
    }
    for (int d = 0; d < 4; ++d) {
        if (H.disk_GM[d] == 0.0) continue;
        disk_field(H.disk_GM[d], H.disk_a[d], H.disk_b[d], dx, dy, dz, gx, gy, gz, gp);
        ax += gx; ay += gy; az += gz; phi += gp;
    }
}

__device__ inline double host_potential(const HaloDev& H, double px, double py, double pz)
{
    double ax, ay, az, phi;
    host_field(H, px, py, pz, ax, ay, az, phi);
    return phi;
}

}  // namespace sidm
