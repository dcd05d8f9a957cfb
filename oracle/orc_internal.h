/* Oracle-private constants and helpers.  TEST INFRASTRUCTURE ONLY. */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H

/* CODATA 2018, SI */
#define ORC_QE    1.602176634e-19
#define ORC_ME    9.1093837015e-31
#define ORC_EPS0  8.8541878128e-12
#define ORC_HBAR  1.054571817e-34
#define ORC_CLIGHT 299792458.0
#define ORC_PI    3.141592653589793
/* e^2 / (4 pi eps0) in eV m, and 3 / (4 pi) */
#define ORC_E2    (ORC_QE / ((4.0 * ORC_PI) * ORC_EPS0))
#define ORC_THREE_OVER_4PI (3.0 / (4.0 * ORC_PI))

int orc_valence(int z, int k);

#endif
