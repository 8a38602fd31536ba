// Host construction of the noisy-gate superoperator M = N2[p] . U.
//
//  * U: Haar-random U(4) from one complex Ginibre draw Z = (re + i im)/sqrt(2);
//    Q of the QR factorisation with a positive real R diagonal (the phase
//    convention that makes Q Haar distributed, Mezzadri 2007).  Computed here
//    by modified Gram-Schmidt with one re-orthogonalisation pass.
//  * unitary part: M_U[(i1 i1')(i2 i2'), (j1 j1')(j2 j2')]
//      = <i1 i2|U|j1 j2> <j1' j2'|U^dagger|i1' i2'>   (App. A, element of M)
//  * noise: N2[p](rho) = (1 - 16p/15) rho + (16p/15) Tr(rho) I/4 (Sec. II.B).
//  * Pauli basis: coefficients on sigma_P/sqrt(2), M_P = (W x W) M (W x W)^H
//    with W[P][2i+i'] = conj(sigma_P[i][i'])/sqrt(2).
#include <complex>
#include <cmath>

#include "../../include/mpo.h"

namespace {
using cd = std::complex<double>;

void haar_from_ginibre(const double* re, const double* im, cd U[4][4]) {
    const double s = 1.0 / std::sqrt(2.0);
    cd z[4][4];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) z[r][c] = cd(re[4 * r + c] * s, im[4 * r + c] * s);
    cd q[4][4];  // q[col][row]
    for (int j = 0; j < 4; ++j) {
        cd v[4];
        for (int r = 0; r < 4; ++r) v[r] = z[r][j];
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                cd d = 0.0;
                for (int r = 0; r < 4; ++r) d += std::conj(q[i][r]) * v[r];
                for (int r = 0; r < 4; ++r) v[r] -= d * q[i][r];
            }
        double nrm = 0.0;
        for (int r = 0; r < 4; ++r) nrm += std::norm(v[r]);
        nrm = std::sqrt(nrm);
        for (int r = 0; r < 4; ++r) q[j][r] = v[r] / nrm;
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) U[r][c] = q[c][r];
}

const cd kPauli[4][2][2] = {
    {{1.0, 0.0}, {0.0, 1.0}},
    {{0.0, 1.0}, {1.0, 0.0}},
    {{0.0, cd(0.0, -1.0)}, {cd(0.0, 1.0), 0.0}},
    {{1.0, 0.0}, {0.0, -1.0}},
};
}  // namespace

extern "C" mpo_status mpo_build_superop(const double* re, const double* im, double p,
                                        mpo_basis basis, double* out, double* u_out) {
    if (!re || !im || !out || !(p >= 0.0 && p <= 1.0) ||
        (basis != MPO_BASIS_PAULI && basis != MPO_BASIS_COMPUTATIONAL))
        return MPO_ERR_ARG;
    cd U[4][4];
    haar_from_ginibre(re, im, U);
    // unitary superoperator, computational basis
    cd S[16][16];
    for (int i1 = 0; i1 < 2; ++i1) for (int i1p = 0; i1p < 2; ++i1p)
    for (int i2 = 0; i2 < 2; ++i2) for (int i2p = 0; i2p < 2; ++i2p)
    for (int j1 = 0; j1 < 2; ++j1) for (int j1p = 0; j1p < 2; ++j1p)
    for (int j2 = 0; j2 < 2; ++j2) for (int j2p = 0; j2p < 2; ++j2p) {
        const int row = 4 * (2 * i1 + i1p) + (2 * i2 + i2p);
        const int col = 4 * (2 * j1 + j1p) + (2 * j2 + j2p);
        S[row][col] = U[2 * i1 + i2][2 * j1 + j2] * std::conj(U[2 * i1p + i2p][2 * j1p + j2p]);
    }
    // depolarizing: (1-q) 1 + (q/4) t t^T, t marks I1, I2 in {0, 3}
    const double q = 16.0 * p / 15.0;
    cd M[16][16];
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c) {
            cd acc = (1.0 - q) * S[r][c];
            const bool tr = ((r >> 2) == 0 || (r >> 2) == 3) && ((r & 3) == 0 || (r & 3) == 3);
            if (tr) {
                cd colsum = 0.0;   // (t^T S)[c]
                for (int k = 0; k < 16; ++k) {
                    const bool tk = ((k >> 2) == 0 || (k >> 2) == 3) && ((k & 3) == 0 || (k & 3) == 3);
                    if (tk) colsum += S[k][c];
                }
                acc += (q / 4.0) * colsum;
            }
            M[r][c] = acc;
        }
    if (basis == MPO_BASIS_PAULI) {
        const double s = 1.0 / std::sqrt(2.0);
        cd W[4][4];
        for (int P = 0; P < 4; ++P)
            for (int i = 0; i < 2; ++i)
                for (int ip = 0; ip < 2; ++ip) W[P][2 * i + ip] = std::conj(kPauli[P][i][ip]) * s;
        cd WW[16][16];
        for (int a = 0; a < 16; ++a)
            for (int b = 0; b < 16; ++b) WW[a][b] = W[a >> 2][b >> 2] * W[a & 3][b & 3];
        cd T[16][16];
        for (int r = 0; r < 16; ++r)
            for (int c = 0; c < 16; ++c) {
                cd acc = 0.0;
                for (int k = 0; k < 16; ++k) acc += WW[r][k] * M[k][c];
                T[r][c] = acc;
            }
        for (int r = 0; r < 16; ++r)
            for (int c = 0; c < 16; ++c) {
                cd acc = 0.0;
                for (int k = 0; k < 16; ++k) acc += T[r][k] * std::conj(WW[c][k]);
                M[r][c] = acc;
            }
    }
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c) {
            out[2 * (16 * r + c)] = M[r][c].real();
            out[2 * (16 * r + c) + 1] = M[r][c].imag();
        }
    if (u_out)
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                u_out[2 * (4 * r + c)] = U[r][c].real();
                u_out[2 * (4 * r + c) + 1] = U[r][c].imag();
            }
    return MPO_OK;
}
