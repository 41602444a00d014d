// tableau.h -- Butcher tableaux of the embedded Runge-Kutta pairs (host).
#pragma once

#include "mm_internal.h"

namespace mm {

// Butcher tableaux (section "Dynamics"): row s holds a_{s+1, j}, j <= s.
struct Tableau {
    int stages;        // derivatives per step including the first-same-as-last one
    int order_low;     // order of the embedded (error) solution
    double a[7][6];
    double e[7];       // b_j - b*_j
};

inline const Tableau DP45 = {
    7, 4,
    {{0, 0, 0, 0, 0, 0},
     {1.0 / 5, 0, 0, 0, 0, 0},
     {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
     {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
     {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
     {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
     {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}},
    {35.0 / 384 - 5179.0 / 57600, 0, 500.0 / 1113 - 7571.0 / 16695, 125.0 / 192 - 393.0 / 640,
     -2187.0 / 6784 + 92097.0 / 339200, 11.0 / 84 - 187.0 / 2100, -1.0 / 40}};

inline const Tableau BS23 = {
    4, 2,
    {{0, 0, 0, 0, 0, 0},
     {1.0 / 2, 0, 0, 0, 0, 0},
     {0, 3.0 / 4, 0, 0, 0, 0},
     {2.0 / 9, 1.0 / 3, 4.0 / 9, 0, 0, 0},
     {0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0}},
    {2.0 / 9 - 7.0 / 24, 1.0 / 3 - 1.0 / 4, 4.0 / 9 - 1.0 / 3, -1.0 / 8, 0, 0, 0}};

// Heun's method with the Euler step as error estimate (RK12); not first same
// as last: the new state m0 + dt (k1 + k2)/2 is formed after the stages.
inline const Tableau RK12 = {
    2, 1,
    {{0, 0, 0, 0, 0, 0},
     {1.0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0},
     {0, 0, 0, 0, 0, 0}},
    {1.0 / 2 - 1.0, 1.0 / 2, 0, 0, 0, 0, 0}};

// Stage s of tableau tb: combine over the non-zero a_sj, derivative into
// logical buffer s; the last stage also lists the error weights.  Returns
// whether s is the last stage (the error-norm stage).
inline bool fill_stage(const Tableau& tb, int s, StageDesc& sd) {
    const int S = tb.stages;
    sd.nk = 0;
    for (int j = 0; j < s; ++j)
        if (tb.a[s][j] != 0.0) {
            sd.kidx[sd.nk] = j;
            sd.a[sd.nk] = (float)tb.a[s][j];
            ++sd.nk;
        }
    sd.out_k = s;
    sd.nerr = 0;
    if (s != S - 1) return false;
    for (int j = 0; j < S; ++j)
        if (tb.e[j] != 0.0) {
            sd.eidx[sd.nerr] = j;
            sd.e[sd.nerr] = (float)tb.e[j];
            ++sd.nerr;
        }
    return true;
}

}  // namespace mm
