// Argument blocks and launchers of the two-pass kernels (local values to HBM, then
// a deterministic gather): formation-only expansion, coefficient and tensor
// products, load vector, isoparametric elements.
#pragma once

#include "kernels.hpp"

namespace qxa {

struct ExpandArgs {
    int64_t n_elem;
    int np;
    const double *Sm, *Sc;  // [ns][n_elem]
    double *Vm, *Vc;        // [np*np][n_elem]
};

struct CoeffProductArgs {
    int64_t n_elem;
    const int32_t *conn;  // [np][n_elem]
    const double *phi;    // [np][nq] basis values of the rule
    CoeffDev c;           // law of the first factor; c.field = u [n_nodes]
    const double *v;      // [n_nodes]
    double *S;            // [nq_out][n_elem]
    int *flags;
    int nq_out;           // nodes of the caller's rule (the compiled rule may be padded)
};

struct CondTensorArgs {
    int64_t n_nodes, n_elem;
    const double *coords;  // [dim][n_nodes]
    const int32_t *conn;   // [np][n_elem]
    const double *w;       // [nq] stiffness rule
    const double *phi;     // [np][nq]
    const double *dphi;    // [nq][np][dim]
    CoeffDev c;            // law of c'; c.field = u [n_nodes]
    int aniso;             // conductivity tensor K instead of the identity
    double K[6];
    const double *v;       // [n_nodes]
    double *T;             // [n_elem][np][np] local matrices (row a, column b)
    int *flags;
};

struct LoadArgs {
    FormInputs in;        // geometry, mass-rule tables; in.cm = the load coefficient f
    const int32_t *conn;  // [np][n_elem]
    double *Fe;           // [np][n_elem] element load vectors
};

struct IsoArgs {
    FormInputs in;         // coefficients, tensor, rules (w, phi)
    const int32_t *tconn;       // [np][n_elem] connectivity in tile order
    const int32_t *elem_order;  // tile position -> element id (per-(q, e) inputs are in mesh order)
    const double *dphi_m;  // [nq_m][np][dim]
    const double *dphi_c;  // [nq_c][np][dim]
    const double *Qm;      // [ns][nq_m] FP64 mass table (symmetric pair rows)
    const double *Qc;      // [ns][nq_c][ng] FP64 conductivity table
    const double *Kq;      // [nq_kq][ng][n_elem] conductivity tensor per node (or null)
    int nq_kq;             // nodes of the caller's stiffness rule
    double *Tm, *Tc;       // [n_elem / 64][ns][64] symmetric local matrices of the tile positions, pair-major per block
};

struct SlotGatherArgs {
    int64_t n_slots;
    const int32_t *ptr;    // [n_slots + 1] (entries below 2^31)
    const int32_t *items;  // indices into src
    const double *src;
    double *out;           // [n_slots]
};


// Elements per block of the isoparametric kernel and of its pair-major layout.
constexpr int kIsoElems = 64;

hipError_t launch_expand(const ExpandArgs &a, hipStream_t st);
hipError_t launch_coeff_product(const CoeffProductArgs &a, int D, int P, int nq, hipStream_t st);
hipError_t launch_cond_tensor(const CondTensorArgs &a, int D, int P, int nq, hipStream_t st);
hipError_t launch_slot_gather(const SlotGatherArgs &a, hipStream_t st);
hipError_t launch_load(const LoadArgs &a, int D, int P, int nq, hipStream_t st);
hipError_t launch_iso(const IsoArgs &a, int D, int P, int nqm, int nqc, hipStream_t st);

}  // namespace qxa
