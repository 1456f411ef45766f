// janc_rtc.h -- run-time specialisation of the point-implicit chemistry kernels to the
// structure of a mechanism (host side; see janc_rtc.hip).
#pragma once

#include <string>
#include <vector>

#include "janc_internal.h"

namespace janc {

// Names of the specialised kernels in their code objects.
constexpr const char* CHEM_SPEC_KERNEL = "janc_chem_spec";
constexpr const char* ADJ_CHEM_SPEC_KERNEL = "janc_adj_chem_spec";

// HIP source of the chemistry kernel specialised to d: the reactants and products of every
// reaction (species indices), reversibility, third-body reactions and the non-zero
// stoichiometric changes become compile-time constants, and so do the rate, stoichiometric,
// third-body and molar-mass numbers (exact literals); the NASA-7 coefficients are read from
// the device table. The arithmetic is the generic kernel's, operation for operation.
std::string chem_spec_source(const DevMech& d);

// HIP source of the reversed chemistry kernel of the discrete adjoint (adj_chem) specialised
// the same way: the rate, Jacobian and reverse-sweep loops over the reactions unrolled with
// the species indices, reversibility, third-body pattern and the numbers of the reactions
// as constants. The arithmetic is the generic adj_chem's, operation for operation.
std::string adj_chem_spec_source(const DevMech& d);

// gfx950 code object of `src` (compiled with hipRTC once per distinct source in this
// process); false with the compiler log in *log on failure.
bool chem_spec_code(const std::string& src, std::vector<char>* code, std::string* log);

}  // namespace janc
