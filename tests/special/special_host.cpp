// Host build of the device special functions (fm_special.h) for the CPU tests.
#include "../../paper_2211_07777_amd/csrc/fm_special.h"

extern "C" {
double sf_bessel_k(int nu, double x) { return fm::bessel_k(nu, x); }
double sf_sine_integral(double x) { return fm::sine_integral(x); }
void sf_scaled_bessel_row(double x, int count, double* row) { fm::scaled_bessel_row(x, count, row); }
}
