// Time update of one particle (Section 2.2): Verlet scheme, eqs. sphu1,
// sphr1, sphrho1, and the Euler reset of eqs. sphu2, sphr2, sphrho2.  Fluid
// particles update r, u, rho; dynamic boundary particles rho, and r with their
// own constant velocity (zero for a fixed wall, nonzero for a moving gate).  The new
// level is written over the previous one (um, rhom); the caller then swaps the
// (u, um) and (rho, rhom) pointers.  FP64 accumulators for r and u; the mixed
// path keeps rho - rho0 in FP32, updated in FP64 and rounded once.  With kKeys
// and keys_next set, the update also writes the particle's sort key at its new
// position, which the next step's sort reads instead of the positions (the
// interaction kernels that advance the state themselves leave it out: the key's
// divisions would cost them occupancy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace wcsph {

struct StateArrays {
    double *x, *y, *z;
    const double *ux, *uy, *uz;
    double *uxm, *uym, *uzm;
    const void *rho;
    void *rhom;
    const uint32_t *id;
    uint32_t *keys_next;  // or null
    unsigned int *walls_move;  // DevScalars::walls_move: set when a boundary
                               // particle has a nonzero velocity
    // the other buffers of rho and rhom (the next gather's destinations), or
    // null: a boundary particle's two levels are also written there, so a
    // gather that leaves fixed walls in place need not copy them
    void *rho_alt, *rhom_alt;
};

// Returns the key written (0 without kKeys).
template <bool kMixed, bool kKeys>
__device__ __forceinline__ uint32_t advance(const StateArrays &s, const Inst &ip, int64_t i,
                                            double dt, bool euler, double ax, double ay,
                                            double az, double dr) {
    const double w = euler ? dt : 2.0 * dt;
    const uint32_t id = s.id[i];
    const bool bnd = (id >> 31) != 0;
    if constexpr (kMixed) {
        const float curf = static_cast<const float *>(s.rho)[i];
        const double cur = (double)curf;
        float *pm = static_cast<float *>(s.rhom);
        const double base = euler ? cur : (double)pm[i];
        const float nxt = (float)(base + w * dr);
        pm[i] = nxt;
        if (bnd && s.rho_alt) {  // after the level swap: rho = new, rhom = current
            static_cast<float *>(s.rho_alt)[i] = nxt;
            static_cast<float *>(s.rhom_alt)[i] = curf;
        }
    } else {
        const double cur = static_cast<const double *>(s.rho)[i];
        double *pm = static_cast<double *>(s.rhom);
        const double base = euler ? cur : pm[i];
        const double nxt = base + w * dr;
        pm[i] = nxt;
        if (bnd && s.rho_alt) {
            static_cast<double *>(s.rho_alt)[i] = nxt;
            static_cast<double *>(s.rhom_alt)[i] = cur;
        }
    }
    const double ux = s.ux[i], uy = s.uy[i], uz = s.uz[i];
    if (bnd) {
        // boundary: keeps its velocity (zero for a fixed wall, the prescribed
        // one of a moving gate) and moves with it.  Any nonzero bit (-0 too)
        // marks a moving wall: later steps then sort and gather every particle.
        if ((__double_as_longlong(ux) | __double_as_longlong(uy) | __double_as_longlong(uz)) != 0)
            *s.walls_move = 1u;
        s.uxm[i] = ux;
        s.uym[i] = uy;
        s.uzm[i] = uz;
        const double x = s.x[i] + dt * ux, y = s.y[i] + dt * uy, z = s.z[i] + dt * uz;
        s.x[i] = x;
        s.y[i] = y;
        s.z[i] = z;
        uint32_t key = 0;
        if (kKeys && s.keys_next) {
            key = sort_key(ip, x, y, z, id);
            s.keys_next[i] = key;
        }
        return key;
    }
    const double hdt2 = 0.5 * dt * dt;
    const double bx = euler ? ux : s.uxm[i];
    const double by = euler ? uy : s.uym[i];
    const double bz = euler ? uz : s.uzm[i];
    const double x = s.x[i] + dt * ux + hdt2 * ax;
    const double y = s.y[i] + dt * uy + hdt2 * ay;
    const double z = s.z[i] + dt * uz + hdt2 * az;
    s.x[i] = x;
    s.y[i] = y;
    s.z[i] = z;
    uint32_t key = 0;
    if (kKeys && s.keys_next) {
        key = sort_key(ip, x, y, z, id);
        s.keys_next[i] = key;
    }
    s.uxm[i] = bx + w * ax;
    s.uym[i] = by + w * ay;
    s.uzm[i] = bz + w * az;
    return key;
}

}  // namespace wcsph
