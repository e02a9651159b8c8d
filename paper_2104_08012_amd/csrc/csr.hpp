// Assembled CSR operator: host handle and device launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "ops.hpp"

namespace fem {

// How a stored entry is formed: the sum of its element-matrix contributions, the 1 on the
// diagonal of a Dirichlet row, or 0 (the rest of a Dirichlet row and Dirichlet columns).
enum : uint8_t { CSR_SUM = 0, CSR_ONE = 1, CSR_ZERO = 2 };

void csr_elem_launch(int nloc, int64_t C, int n, int p, int L, const int32_t* map, const double* G,
                     const double* tab, int nq, const double* k, double* E, hipStream_t s);
template <typename T>
void csr_gather_launch(int64_t nnz, const int64_t* cptr, const int32_t* cidx, const uint8_t* flag, const double* E,
                       T* val, hipStream_t s);
template <typename T>
void csr_spmv_launch(int64_t nrows, int lanes, const int32_t* rp, const int32_t* col, const T* val, const T* x, T* y,
                     hipStream_t s);

}  // namespace fem

struct fem_csr {
    const fem_mesh* m = nullptr;
    int level = 0;
    int64_t n = 0, nnz = 0, ncontrib = 0;
    std::vector<int32_t> row_ptr, col;
    std::vector<int64_t> cptr;     // per stored entry: its contributions in cidx
    std::vector<int32_t> cidx;     // element-matrix entry (i nloc + j) C + c, ascending cell order
    std::vector<uint8_t> flag;
    size_t d_rp = 0, d_col = 0, d_cptr = 0, d_cidx = 0, d_flag = 0, d_elem = 0, bytes = 0;
    char* dev = nullptr;
};
