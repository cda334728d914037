// Scheme parameters as the kernels see them, from the public configuration
// (linear weights normalised, K computed once in FP64 from gamma).
#pragma once

#include "../../include/gks.h"
#include "gks_internal.h"

namespace gks {

inline Params params_from_config(const gks_config *cfg)
{
    Params p{};
    p.gamma = cfg->gamma;
    p.K = (5.0 - 3.0 * cfg->gamma) / (cfg->gamma - 1.0);
    p.mu = cfg->mu;
    p.prandtl = cfg->prandtl;
    p.eps_tau = cfg->eps_tau;
    p.c_tau = cfg->c_tau;
    p.eps_weno = cfg->eps_weno;
    const double s2 = cfg->lw2[0] + cfg->lw2[1] + cfg->lw2[2];
    const double s1 = cfg->lw1[0] + cfg->lw1[1];
    p.g22 = cfg->lw2[0] / s2;
    p.g12 = cfg->lw2[1] / s2;
    p.g02 = cfg->lw2[2] / s2;
    p.g11 = cfg->lw1[0] / s1;
    p.g01 = cfg->lw1[1] / s1;
    p.viscous = cfg->viscous;
    p.nonlinear = cfg->nonlinear;
    p.order = cfg->order;
    p.flux = cfg->flux;
    p.wall_T = cfg->wall_T;
    for (int q = 0; q < 5; ++q) p.farfield[q] = cfg->farfield[q];
    return p;
}

}  // namespace gks
