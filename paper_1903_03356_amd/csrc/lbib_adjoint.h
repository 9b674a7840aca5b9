// Internal declarations of the reverse-mode (adjoint) kernels.
#pragma once

#include "lbib_internal.h"

namespace lbib {

// One reverse grid step n (and the initial-state term, which reuses it).
template <typename T>
struct GridAdjArgs {
    const T* pops;          // P^n, the populations the forward step n pulled from
    const long long* fib;   // F^n - g (fixed point) and its segment flags
    const int* flags;
    const T* lam_in;        // lambda of P^{n+1}
    T* lam_out;             // lambda of P^n (every slot written)
    T* lfm;                 // moment part of lambda F^n (read, then cleared)
    int* lfm_flags;         // its segment flags (read, then cleared)
    T* lft;                 // lambda F^n, written on the active force segments
    double* gacc;           // one body-force gradient slot per block
};

// One reverse IB launch: reverse of [B(n-1)] [start-up] [A(n)].
template <typename T>
struct IBAdjArgs {
    const T* pops;              // P^n
    const long long* fib_prev;  // F^{n-1} - g
    const T* nodes_n;           // node state of level n   ([8][stride], tape)
    const double* ref_n;        // reference points of level n ([caps][2])
    const T* nodes_p;           // node state of level n-1 (when doB)
    const double* ref_p;
    const T* consts;            // stress-free lengths and k_s (the context's node arrays)
    const CapsuleDev* caps;
    const T* lft;               // lambda F^n (active segments)
    T* lam_p;                   // lambda P^n (atomic adds)
    T* lfm;                     // lambda F^{n-1}, moment part (atomic adds)
    int* lfm_flags;
    double* lamx;               // [2][stride] carried: x^n in, x^{n-1} out
    double* lamd;               // [2][stride] carried: d^n in, d^{n-1} out
    double* ksbar;              // [stride] dJ/dk_s per element (accumulated)
    int* status;
    int stride;
    int doA, doB, prime, dynamic;
    int bend;                   // some capsule has k_b != 0 (Eq. 13)
    int patch_cap, max_nv;
};

template <typename T>
hipError_t launch_grid_adj(const GridAdjArgs<T>& a, const GridArgs& g, hipStream_t s);
template <typename T>
hipError_t launch_init_adj(const GridAdjArgs<T>& a, const GridArgs& g, int profile, double nu,
                           hipStream_t s);
hipError_t launch_reduce_sum(const double* v, int n, double* out, hipStream_t s);
template <typename T>
hipError_t launch_adj_seed(const T* nodes, const double* ref, const CapsuleDev* caps, int cap_id,
                           int stride, int objective, double* lamx, double* out, hipStream_t s);
template <typename T>
hipError_t launch_ib_adj(const IBAdjArgs<T>& a, int ncap, size_t lds_bytes, hipStream_t s);
template <typename T>
hipError_t ib_adj_set_lds_limit(size_t bytes);
template <typename T>
size_t ib_adj_lds_bytes(int patch_cap, int max_nv);

}  // namespace lbib
