// Chemkin-format reader (chemkin.cpp).
#pragma once

#include <string>

namespace pyjac {

// Chemkin-format mechanism (and optional separate thermo text) -> the token
// format build_tables reads.  Returns 0 or a PYJAC_E_* code with msg set.
int chemkin_to_tokens(const std::string& mech, const std::string* thermo, std::string& out, std::string& msg);

}  // namespace pyjac
