// Device layout of the atomic tables copied by init_species.
#pragma once

#include <stdint.h>

namespace xpd {

struct DevTables {
    double bind[14][5];       // eV
    double lotz_a[5];         // cm^2 eV^2
    double lotz_b[5];
    double lotz_c[5];
    double gamma_a[14][3];    // 1/s
    double gamma_x[14][3];
    double e_kalpha[14];      // eV
    double mass_ion;          // kg
    double photo_lnhv0, photo_dlnhv;
    double eos_lnn0, eos_dlnn, eos_lnt0, eos_dlnt;
    int32_t photo_nh, eos_nn, eos_nt, pad;
    int64_t off_lnsig;        // byte offset of [5][photo_nh] from the start of the struct
    int64_t off_eos;          // byte offset of [eos_nn][eos_nt]
};

}  // namespace xpd
