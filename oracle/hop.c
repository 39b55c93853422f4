/*
 * FP64 oracle: the Wilson hopping term D^w of the paper (Sec. 2.2, the
 * definition of D^w_{x,y}) restricted to one checkerboard parity, and its
 * adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU oracle that the
 * tests and the benchmark's CPU baseline use to check the HIP library.  It
 * shares no code with the library and the library never calls it.
 *
 * Definition written out (no spin projection, no blocking):
 *
 *   (D^w psi)(x) = sum_mu [ (1 - g gamma_mu) U_{x,mu}            psi(x + mu)
 *                         + (1 + g gamma_mu) U^dag_{x - mu, mu}   psi(x - mu) ]
 *
 * with g = +1.  Its adjoint as a matrix is the same sum with g = -1 (the
 * gamma matrices are Hermitian), which is what dagger = 1 computes.
 * Periodic boundaries in all four directions.
 *
 * Layouts (complex128 interleaved):
 *   U      [T][Z][Y][X][mu][3][3]
 *   gamma  [mu][4][4]             (passed in by the caller)
 *   in     [Ls][V/2][4][3]        parity 1 - out_parity
 *   out    [Ls][V/2][4][3]        parity out_parity
 * A single-parity field is ordered by lex/2, lex = x + X*(y + Y*(z + Z*t)).
 */
#include <complex.h>
#include <stddef.h>
#include <stdint.h>

typedef double _Complex cplx;

static inline int64_t lex_of(int x, int y, int z, int t, int X, int Y, int Z)
{
    return (int64_t)x + (int64_t)X * ((int64_t)y + (int64_t)Y * ((int64_t)z + (int64_t)Z * t));
}

void oracle_wilson_hop(const cplx *U, const cplx *gamma, const cplx *in, cplx *out,
                       int X, int Y, int Z, int T, int Ls, int out_parity, int dagger)
{
    const int64_t V = (int64_t)X * Y * Z * T;
    const int64_t Vh = V / 2;
    const double g = dagger ? -1.0 : 1.0;
    const int ext[4] = {X, Y, Z, T};

#pragma omp parallel for schedule(static) if (Vh * Ls >= 16384)
    for (int64_t i = 0; i < Vh; ++i) {
        /* coordinates of the output site of this parity */
        const int64_t l0 = 2 * i;
        const int x0 = (int)(l0 % X);
        const int y = (int)((l0 / X) % Y);
        const int z = (int)((l0 / ((int64_t)X * Y)) % Z);
        const int t = (int)(l0 / ((int64_t)X * Y * Z));
        const int x = x0 + ((y + z + t + out_parity) & 1);
        const int c[4] = {x, y, z, t};

        for (int s = 0; s < Ls; ++s) {
            cplx acc[4][3];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 3; ++b)
                    acc[a][b] = 0.0;

            for (int mu = 0; mu < 4; ++mu) {
                for (int dir = 0; dir < 2; ++dir) {      /* 0: +mu, 1: -mu */
                    int n[4] = {c[0], c[1], c[2], c[3]};
                    n[mu] = dir == 0 ? (c[mu] + 1) % ext[mu] : (c[mu] - 1 + ext[mu]) % ext[mu];
                    const int64_t nl = lex_of(n[0], n[1], n[2], n[3], X, Y, Z);
                    const cplx *psi = in + (((int64_t)s * Vh + nl / 2) * 4) * 3;

                    /* link: U_{x,mu} forward, U^dag_{x-mu,mu} backward */
                    const int64_t link_site = dir == 0 ? lex_of(x, y, z, t, X, Y, Z) : nl;
                    const cplx *L = U + (link_site * 4 + mu) * 9;

                    /* v = link * psi (colour), for each of the 4 spins */
                    cplx v[4][3];
                    for (int sp = 0; sp < 4; ++sp)
                        for (int a = 0; a < 3; ++a) {
                            cplx sum = 0.0;
                            for (int b = 0; b < 3; ++b) {
                                const cplx l = dir == 0 ? L[a * 3 + b] : conj(L[b * 3 + a]);
                                sum += l * psi[sp * 3 + b];
                            }
                            v[sp][a] = sum;
                        }

                    /* spin factor (1 -/+ g gamma_mu) */
                    const double sg = dir == 0 ? -g : g;
                    const cplx *gm = gamma + mu * 16;
                    for (int al = 0; al < 4; ++al)
                        for (int a = 0; a < 3; ++a) {
                            cplx sum = v[al][a];
                            for (int be = 0; be < 4; ++be)
                                sum += sg * gm[al * 4 + be] * v[be][a];
                            acc[al][a] += sum;
                        }
                }
            }
            cplx *o = out + (((int64_t)s * Vh + i) * 4) * 3;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 3; ++b)
                    o[a * 3 + b] = acc[a][b];
        }
    }
}
