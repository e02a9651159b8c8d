// Host-side entry points of the device operations.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace fem {

template <typename T>
inline const T* dptr(const fem_mesh& m, size_t off) {
    return reinterpret_cast<const T*>(m.dev + off);
}

template <typename T>
struct ScatterIO {
    const T* x = nullptr;
    const T* x2 = nullptr;
    const T* k = nullptr;
    T* y = nullptr;
    const T* z = nullptr;
    double alpha = 1.0, beta = 0.0;
    int row_mode = ROW_IDENTITY;
    const T* xid = nullptr;
    int mask_cols = 1;
    // interface partial sums: the level's slot area of the mesh buffer (NULL), or this array of
    // slots_bytes (the allocation-free action's file-scope scratch)
    void* slots = nullptr;
    size_t slots_bytes = 0;
};

// kind: K_APPLY, K_DIAG, K_MASS, K_GRAD (T = double).
template <typename T>
fem_status run_scatter(const fem_mesh& m, int level, int kind, bool kvar, const ScatterIO<T>& io, hipStream_t s);

// Lattice transfers between fine_level - 1 and fine_level (transfer.hip): x_f += P x_c, and
// r_c = P^T r_f with boundary rows zero.
template <typename T>
fem_status run_prolong(const fem_mesh& m, int fine_level, const T* xc, T* xf, hipStream_t s);
template <typename T>
fem_status run_restrict(const fem_mesh& m, int fine_level, const T* rf, T* rc, hipStream_t s);

fem_status check_launch(const char* what);

// Device address of the file-scope scratch array of the allocation-free action on the current
// device (looked up once per device), and its size in bytes.
fem_status noalloc_scratch(void** ptr, size_t* bytes);

// Additive vertex-star patch preconditioner, degrees 2 and 3 (patch.hip).
bool patch_supported(const HostLevel& H, std::string& why);
size_t patch_bytes(const HostLevel& H, size_t ts);
template <typename T>
fem_status patch_setup(const fem_mesh& m, int level, const double* k, void* buf, hipStream_t s);
template <typename T>
fem_status patch_apply(const fem_mesh& m, int level, void* buf, const T* r, T* z, hipStream_t s);

}  // namespace fem
