// Host-only driver for the state-file reader of libgpdbec (gp_state.cpp), built with the
// address and undefined-behaviour sanitizers by tests/test_state_files.py.  The calls of
// gp_state.cpp into the device part of the library are stubbed: only the readers run.
//
// Usage: state_reader <file>...   prints "<status> <kind> <npoints>" per file.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../../include/gp.h"

extern "C" {
gp_status gp_get_params(gp_ctx*, gp_params*) { return GP_E_STATE; }
gp_status gp_get_psi(gp_ctx*, void*, int) { return GP_E_STATE; }
gp_status gp_set_psi(gp_ctx*, const void*, int) { return GP_E_STATE; }
gp_status gp_energy(gp_ctx*, gp_observables*) { return GP_E_STATE; }
gp_status gp_step_imag(gp_ctx*, int) { return GP_E_STATE; }
gp_status gp_step_real(gp_ctx*, int) { return GP_E_STATE; }
gp_status gp_sync(gp_ctx*) { return GP_E_STATE; }
}

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    gp_state_info info;
    gp_status s = gp_state_read_info(argv[i], &info);
    if (s == GP_OK) {
      // a buffer of exactly the payload size: an overrun is a sanitizer report
      const size_t n = (size_t)info.npoints * (info.kind == GP_STATE_PSI ? 2 : 1);
      std::vector<double> buf(n);
      s = gp_state_read(argv[i], &info, buf.data(), n);
      if (s == GP_OK && n > 0) {
        // a one-short buffer must be refused without a write
        std::vector<double> small(n - 1 > 0 ? n - 1 : 1);
        if (gp_state_read(argv[i], &info, small.data(), n - 1) != GP_E_ARG) return 3;
      }
    }
    printf("%d %d %llu\n", s, s == GP_OK ? info.kind : 0,
           s == GP_OK ? (unsigned long long)info.npoints : 0ull);
  }
  return 0;
}
