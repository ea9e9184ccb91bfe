"""Build libamm.so (HIP for gfx950 + host C++) in-tree.

Every HIP translation unit is compiled with -ffp-contract=off (the sampler's
bit-exact operation order; the integrand uses explicit fma) and with packed
FP32 instructions disabled."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
OUT = os.path.join(HERE, 'libamm.so')
BUILD = os.path.join(HERE, '_build')
ARCH = os.environ.get('AMM_OFFLOAD_ARCH', 'gfx950')

HIP_FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}', '-ffp-contract=off',
             '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
             '-munsafe-fp-atomics', '-Wno-unused-result', '-Wno-unused-value']
HOST_FLAGS = ['-O2', '-std=c++17', '-fPIC', '-ffp-contract=off', '-Wno-unknown-pragmas']


def run(cmd):
    print(' '.join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
    objs = []
    host_o = os.path.join(BUILD, 'amm_host.o')
    run(['g++'] + HOST_FLAGS + ['-c', os.path.join(CSRC, 'amm_host.cpp'), '-o', host_o])
    objs.append(host_o)
    for src in ('amm_device.hip', 'amm_mlp.hip'):
        o = os.path.join(BUILD, src.replace('.hip', '.o'))
        run([hipcc] + HIP_FLAGS + ['-c', os.path.join(CSRC, src), '-o', o])
        objs.append(o)
    tmp = OUT + '.tmp'
    run([hipcc, '-shared', f'--offload-arch={ARCH}', '-o', tmp] + objs)
    os.replace(tmp, OUT)
    return OUT


if __name__ == '__main__':
    build()
    sys.exit(0)
