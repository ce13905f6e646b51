// Kernel argument blocks and launchers (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels_common.hpp"

namespace qxa {

struct FormArgs {
    int64_t n_nodes, n_elem;
    const double *coords;  // [dim][n_nodes]
    const int32_t *conn;   // [np][n_elem]
    CoeffDev cm, cc;
    const double *w_m, *w_c;      // [nq]
    const double *phi_m, *phi_c;  // [np][nq]
    const void *Qm, *Qc;          // compute-type tables [ns][nqm], [ns][nqc][ng]
    double *Vm, *Vc;              // [ns][n_elem] outputs (either may be null)
    int *flags;
};

struct GatherArgs {
    int64_t nnz;
    const uint32_t *src_upper, *seg_ptr, *seg_val;
    const double *Vm, *Vc;
    double *M, *C;
};

struct ExpandArgs {
    int64_t n_elem;
    int np;
    const double *Sm, *Sc;  // [ns][n_elem]
    double *Vm, *Vc;        // [np*np][n_elem]
};

bool form_supported(int D, int P, int nqm, int nqc);
hipError_t launch_form(const FormArgs &a, int D, int P, int nqm, int nqc, int precision, hipStream_t st);
hipError_t launch_gather(const GatherArgs &a, hipStream_t st);
hipError_t launch_expand(const ExpandArgs &a, hipStream_t st);

}  // namespace qxa
