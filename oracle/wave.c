/*
 * FP64 reference implementation ("oracle") of the explicit finite-difference
 * acoustic propagator, its exact discrete adjoint and the adjoint-state
 * gradient.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, by the smoke check and by the
 * CPU-baseline timing of the benchmark. The GPU library never links, loads or
 * calls it, and it shares no code with the library.
 *
 * The body lives in wave_core.inc and is compiled twice: real (double, suffix
 * _d) and complex (double complex, suffix _z; complex-step derivatives only).
 */
#include <complex.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;            /* 2 or 3 */
    int M;               /* half the space order k */
    long nx, ny, nz;     /* computational grid; ny == 1 in 2D */
    double hx, hy, hz;   /* spacing (m) */
    double alpha[17];    /* centred second-difference weights alpha_0 .. alpha_M */
} grid_t;

#define REAL double
#define SFX(name) name##_d
#include "wave_core.inc"
#undef REAL
#undef SFX

#define REAL double complex
#define SFX(name) name##_z
#include "wave_core.inc"
#undef REAL
#undef SFX
