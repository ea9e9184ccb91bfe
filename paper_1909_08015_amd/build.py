"""Build libamm.so (HIP for gfx950 + host C++) in-tree.

Steps:
  1. host plan builder (g++), code generator tool (g++);
  2. generated straight-line integrand sources for the 1-3 loop graphs
     (_build/gen/gen_<loops>_<graph>.{h,hip}) and their dispatch table;
  3. every HIP translation unit (library kernels, MLP, generated graphs),
     compiled in parallel for gfx950 with -ffp-contract=off (the sampler's
     bit-exact operation order; the integrand uses explicit fma) and with
     packed FP32 instructions disabled;
  4. link.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
OUT = os.path.join(HERE, 'libamm.so')
BUILD = os.path.join(HERE, '_build')
GEN = os.path.join(BUILD, 'gen')
ARCH = os.environ.get('AMM_OFFLOAD_ARCH', 'gfx950')
GEN_LOOPS = [int(x) for x in os.environ.get('AMM_GEN_LOOPS', '1,2,3').split(',') if x]

HIP_FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}', '-ffp-contract=off',
             '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
             '-munsafe-fp-atomics', '-Wno-unused-result', '-Wno-unused-value', '-Wno-unused-variable',
             '-I', CSRC, '-I', GEN]
HOST_FLAGS = ['-O2', '-std=c++17', '-fPIC', '-pthread', '-ffp-contract=off', '-Wno-unknown-pragmas']
NGRAPHS = {1: 1, 2: 2, 3: 10, 4: 74}


def run(cmd, quiet=False):
    if not quiet:
        print(' '.join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True, jobs=None):
    os.makedirs(GEN, exist_ok=True)
    hipcc = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
    jobs = jobs or min(16, os.cpu_count() or 4)
    host_o = os.path.join(BUILD, 'amm_host.o')
    run(['g++'] + HOST_FLAGS + ['-c', os.path.join(CSRC, 'amm_host.cpp'), '-o', host_o])
    gen_tool = os.path.join(BUILD, 'amm_codegen')
    run(['g++'] + HOST_FLAGS + ['-I', CSRC, os.path.join(CSRC, 'amm_codegen.cpp'), host_o, '-o', gen_tool])
    hip_srcs = [os.path.join(CSRC, 'amm_device.hip'), os.path.join(CSRC, 'amm_mlp.hip')]
    for n in GEN_LOOPS:
        for g in range(NGRAPHS[n]):
            run([gen_tool, 'graph', str(n), str(g), GEN], quiet=True)
            hip_srcs.append(os.path.join(GEN, f'gen_{n}_{g}.hip'))
    disp = os.path.join(GEN, 'gen_dispatch.hip')
    run([gen_tool, 'dispatch', disp] + [str(n) for n in GEN_LOOPS])
    hip_srcs.append(disp)

    def compile_one(src):
        o = os.path.join(BUILD, os.path.basename(src).replace('.hip', '.o'))
        subprocess.check_call([hipcc] + HIP_FLAGS + ['-c', src, '-o', o])
        return o

    print(f'compiling {len(hip_srcs)} HIP translation units with {jobs} jobs', flush=True)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, hip_srcs))
    tmp = OUT + '.tmp'
    run([hipcc, '-shared', '-pthread', f'--offload-arch={ARCH}', '-o', tmp, host_o] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == '__main__':
    build()
    sys.exit(0)
