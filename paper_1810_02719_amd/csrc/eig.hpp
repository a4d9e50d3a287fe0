// Symmetric eigen-decomposition of the per-block Rayleigh-Ritz matrices by
// Householder tridiagonalisation (see eig.hip).  Used for ld <= TRI_MAX_LD;
// wider blocks take the Jacobi sweeps of small.hpp.
#pragma once

#include "small.hpp"

namespace mis {

constexpr int TRI_MAX_LD = 320;

bool tri_eig_supported(int max_ld);

// A (ld x ld at m_off, p x p used) -> d, e, beta in tri[4 t_off ..] (layout
// d[p] e[p] lambda[p] beta[p]) and the reflectors in the rows of Hv.  Above
// ld = 192 the reduction works in place in A (its contents are destroyed).
void launch_tri_reduce(const SmallDesc* sd, int nb, int max_ld, double* A, double* Hv,
                       double* tri, int32_t* status, hipStream_t s);
// Eigenvalues ascending -> lambda in tri, ritz[t_off + j], perm[t_off + j] = j,
// a_lo[blk] = largest when adapt.  Flags NOCONV / NONFINITE.
void launch_tri_bisect(const SmallDesc* sd, int nb, int max_p, double* tri, double* ritz,
                       int32_t* perm, double* a_lo, int adapt, int32_t* status, hipStream_t s);
// Unit eigenvectors of T in the columns of ZT (DP, DM: ld x ld scratch).
void launch_tri_vectors(const SmallDesc* sd, int nb, int max_p, const double* tri, double* DP,
                        double* DM, double* ZT, int32_t* status, hipStream_t s);
// Z = Q Z_T (columns = eigenvectors of A, ascending; zero outside p x p).
void launch_tri_back(const SmallDesc* sd, int nb, int max_ld, const double* ZT, const double* Hv,
                     const double* tri, double* Z, hipStream_t s);

}  // namespace mis
