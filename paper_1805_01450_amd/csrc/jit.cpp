// Run-time compilation of generated kernels for gfx950 with hiprtc.
#include <hip/hiprtc.h>

#include <string>
#include <vector>

#include "host.h"

namespace qgm {

bool jit_compile(const std::string& src, const char* name, std::vector<char>& code, std::string& err) {
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, src.c_str(), name, 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    err = "hiprtcCreateProgram failed";
    return false;
  }
  // gfx950 only; packed FP32 instructions disabled as for the prebuilt kernels.
  // -fno-honor-nans / -fno-signed-zeros let multiplications by literal 0 and
  // +-1 fold away; no reassociation is enabled, so no other arithmetic moves.
  // The leading kernel arguments are preloaded into SGPRs at wave launch
  // (gfx950 kernarg preload; the code object keeps a loading prologue for
  // firmware without it), which saves a dependent scalar load per wave.
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-fno-honor-nans", "-fno-signed-zeros",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-mllvm", "-amdgpu-kernarg-preload-count=14"};
  hiprtcResult r = hiprtcCompileProgram(p, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(p, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(p, &log[0]);
    err = std::string("hiprtc: ") + hiprtcGetErrorString(r) + "\n" + log.substr(0, 2000);
    hiprtcDestroyProgram(&p);
    return false;
  }
  size_t n = 0;
  hiprtcGetCodeSize(p, &n);
  code.resize(n);
  hiprtcGetCode(p, code.data());
  hiprtcDestroyProgram(&p);
  return true;
}

}  // namespace qgm
