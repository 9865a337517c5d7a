// libnfa: error reporting and version.
#include <string>

#include "nfa_internal.h"

namespace nfa {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
nfa_status fail(nfa_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}
}  // namespace nfa

extern "C" const char* nfa_last_error(void) { return nfa::g_last_error.c_str(); }
extern "C" int nfa_version(void) { return 10000; }
