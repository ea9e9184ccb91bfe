"""Thin ctypes binding of libamm (include/amm.h).  Argument marshalling only:
every step of the Monte Carlo path runs in the library's HIP kernels.  Device
buffers are torch CUDA tensors; streams are torch streams.  Import fails loudly
when libamm.so has not been built."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libamm.so')

AMM_OK = 0
OPT_GENERATED, OPT_FUSED, OPT_ORDER_BY_COST, OPT_BLOCKS_PER_CU, OPT_GENERATOR, OPT_PLANS = 1, 2, 3, 4, 5, 6


class AmmError(RuntimeError):
    pass


class DensityParams(C.Structure):
    _fields_ = [('cbigz', C.c_double), ('cbigf', C.c_double), ('cadd', C.c_double),
                ('csubi', C.c_double), ('csubse', C.c_double), ('csubo', C.c_double),
                ('c', C.c_double * 4), ('d', C.c_double), ('degmax', C.c_double)]


class RunParams(C.Structure):
    _fields_ = [('seed', C.c_uint64), ('counter0', C.c_uint64), ('n_per_graph', C.c_uint64),
                ('graph_begin', C.c_int), ('graph_end', C.c_int), ('sampler', C.c_int),
                ('force_flag', C.c_int), ('blocks_per_cu', C.c_int), ('accumulate', C.c_int),
                ('accept_tau', C.POINTER(C.c_double))]


class Estimate(C.Structure):
    _fields_ = [('mean', C.c_double), ('sigma', C.c_double), ('sum_y', C.c_double),
                ('sum_y2', C.c_double), ('sum_abs', C.c_double), ('n', C.c_uint64),
                ('n_flag', C.c_uint64), ('n_dd_fail', C.c_uint64), ('n_ood', C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanInfo(C.Structure):
    _fields_ = [('n_insertions', C.c_int), ('n_terms', C.c_int), ('n_terms_expanded', C.c_int),
                ('n_level_evals', C.c_int), ('n_monomials', C.c_int64),
                ('flops_per_sample', C.c_double)]


_lib = None

SYMBOLS = {
    'amm_create': (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    'amm_destroy': (None, [C.c_void_p]),
    'amm_last_error': (C.c_char_p, []),
    'amm_enumerate': (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    'amm_graph_desc': (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    'amm_build_tables': (C.c_int, [C.c_void_p, C.POINTER(DensityParams), C.c_int, C.c_int]),
    'amm_plan_stats': (C.c_int, [C.c_void_p, C.c_int, C.POINTER(PlanInfo)]),
    'amm_sample': (C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    'amm_eval': (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_int, C.c_void_p]),
    'amm_integrate': (C.c_int, [C.c_void_p, C.POINTER(RunParams), C.c_void_p]),
    'amm_integrate_batches': (C.c_int, [C.c_void_p, C.POINTER(RunParams), C.c_uint64, C.c_void_p]),
    'amm_autotune': (C.c_int, [C.c_void_p, C.POINTER(RunParams), C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_double), C.c_void_p]),
    'amm_adaptive_split': (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p]),
    'amm_integrate_adaptive': (C.c_int, [C.c_void_p, C.POINTER(RunParams), C.c_uint64, C.c_int, C.c_double,
                                         C.c_void_p, C.c_void_p, C.c_void_p]),
    'amm_combine': (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    'amm_read': (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(Estimate)]),
    'amm_set_option': (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    'amm_accept_thresholds': (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_uint64, C.c_void_p]),
    'amm_profile': (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    'amm_pilot': (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_int, C.c_int, C.c_void_p]),
    'amm_pilot_table': (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    'amm_mlp_train': (C.c_int, [C.c_void_p, C.c_int, C.c_float, C.c_uint64, C.c_void_p]),
    'amm_mlp_params': (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    'amm_mlp_set_params': (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    'amm_mlp_features': (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.POINTER(C.c_size_t)]),
    'amm_mlp_loss_grad': (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    'amm_set_sector_table': (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    'amm_mlp_get_params': (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    'amm_mlp_adam': (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_float, C.c_int, C.c_void_p]),
    'amm_set_workspace': (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    'amm_workspace_bytes': (C.c_size_t, [C.c_int]),
    'amm_integrate_static': (C.c_int, [C.c_void_p, C.POINTER(RunParams), C.c_void_p]),
}


def lib():
    """Load libamm.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise AmmError(f'{LIB_PATH} is not built; run paper_1909_08015_amd/build.py')
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def adaptive_split(C_, t, budget, floor_frac):
    """Sample split of one adaptive round (amm_adaptive_split; host code)."""
    n = len(C_)
    out = (C.c_uint64 * n)()
    _check(lib().amm_adaptive_split(n, (C.c_double * n)(*C_), (C.c_double * n)(*t), float(budget),
                                    float(floor_frac), out), 'amm_adaptive_split')
    return list(out)


def combine(means1, sigmas1, means2, sigmas2):
    """Graph-by-graph combination of two calculations (amm_combine; host
    code): returns (per-graph means, per-graph sigmas, total mean, total sigma)."""
    n = len(means1)
    arr = lambda v: (C.c_double * n)(*v)
    m, s = (C.c_double * n)(), (C.c_double * n)()
    tm, ts = C.c_double(), C.c_double()
    _check(lib().amm_combine(n, arr(means1), arr(sigmas1), arr(means2), arr(sigmas2), m, s, C.byref(tm),
                             C.byref(ts)), 'amm_combine')
    return list(m), list(s), tm.value, ts.value


def _check(rc, what):
    if rc != AMM_OK:
        raise AmmError(f'{what} failed ({rc}): {lib().amm_last_error().decode()}')


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


CALC2 = dict(cbigz=0.256, cbigf=0.839, cadd=0.786, csubi=0.2, csubse=0.0, csubo=0.2,
             c=(((1.0 - 0.03) - 0.01) - 0.06, 0.03, 0.01, 0.06), d=0.75, degmax=1.0)
# the paper's first calculation (with OPT_GENERATOR = 1, MRG32k3a)
CALC1 = dict(CALC2, c=(((1.0 - 0.03) - 0.035) - 0.035, 0.03, 0.035, 0.035), d=0.75)


class Context:
    """One library context on one device."""

    def __init__(self, device=0):
        h = C.c_void_p()
        _check(lib().amm_create(C.byref(h), device), 'amm_create')
        self.h = h
        self.device = device
        self.loops = None

    def close(self):
        if self.h:
            lib().amm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enumerate(self, loops):
        a, b, m = C.c_int(), C.c_int(), C.c_int()
        _check(lib().amm_enumerate(self.h, loops, C.byref(a), C.byref(b), C.byref(m)), 'amm_enumerate')
        self.loops = loops
        self.n_se, self.n_vertex, self.M = a.value, b.value, m.value
        return self.n_se, self.n_vertex, self.M

    def graph_desc(self, g):
        n = self.loops
        ch = (C.c_int * (2 * n))()
        cl = (C.c_int * (3 * (2 * n - 1)))()
        _check(lib().amm_graph_desc(self.h, g, ch, cl), 'amm_graph_desc')
        chords = tuple(sorted((ch[2 * i], ch[2 * i + 1]) for i in range(n)))
        classes = [tuple(cl[3 * e:3 * e + 3]) for e in range(2 * n - 1)]
        return chords, classes

    def build_tables(self, begin=0, end=None, params=None):
        p = dict(CALC2, **(params or {}))
        dp = DensityParams(p['cbigz'], p['cbigf'], p['cadd'], p['csubi'], p['csubse'], p['csubo'],
                           (C.c_double * 4)(*p['c']), p['d'], p['degmax'])
        end = self.n_se if end is None else end
        _check(lib().amm_build_tables(self.h, C.byref(dp), begin, end), 'amm_build_tables')

    def plan_stats(self, g):
        s = PlanInfo()
        _check(lib().amm_plan_stats(self.h, g, C.byref(s)), 'amm_plan_stats')
        return {k: getattr(s, k) for k, _ in s._fields_}

    def sample(self, g, seed, counter0, n, learned=0, stream=None):
        import torch
        dev = f'cuda:{self.device}'
        M = self.M
        z = torch.empty((n, M), dtype=torch.float64, device=dev)
        gx = torch.empty(n, dtype=torch.float64, device=dev)
        gj = torch.empty(n, dtype=torch.int32, device=dev)
        path = torch.empty((n, M), dtype=torch.int32, device=dev)
        comp = torch.empty(n, dtype=torch.int32, device=dev)
        _check(lib().amm_sample(self.h, g, seed, counter0, n, int(learned), _ptr(z), _ptr(gx), _ptr(gj),
                                _ptr(path), _ptr(comp), _stream(stream)), 'amm_sample')
        return dict(z=z, gx=gx, gj=gj, path=path, comp=comp)

    def eval(self, g, z, precision=0, with_bound=False, stream=None):
        import torch
        n = z.shape[0]
        ne = 2 * self.loops - 1
        I = torch.empty((n, ne), dtype=torch.float64, device=z.device)
        A = torch.empty((n, ne), dtype=torch.float64, device=z.device)
        B = torch.empty((n, ne), dtype=torch.float64, device=z.device) if with_bound else None
        zc = z.contiguous()
        _check(lib().amm_eval(self.h, g, _ptr(zc), n, _ptr(I), _ptr(A), _ptr(B), precision, _stream(stream)),
               'amm_eval')
        return (I, A, B) if with_bound else (I, A)

    def _run_params(self, seed, n_per_graph, graph_begin, graph_end, counter0, sampler, force_flag,
                    blocks_per_cu, accumulate, accept_tau):
        graph_end = self.n_se if graph_end is None else graph_end
        tau = None
        if accept_tau is not None:
            tau = (C.c_double * len(accept_tau))(*accept_tau)
        rp = RunParams(seed, counter0, n_per_graph, graph_begin, graph_end, sampler, force_flag,
                       blocks_per_cu, accumulate,
                       C.cast(tau, C.POINTER(C.c_double)) if tau is not None else None)
        return rp, tau

    def integrate(self, seed, n_per_graph, graph_begin=0, graph_end=None, counter0=0, sampler=0,
                  force_flag=0, blocks_per_cu=0, accumulate=0, accept_tau=None, stream=None):
        rp, _keep = self._run_params(seed, n_per_graph, graph_begin, graph_end, counter0, sampler, force_flag,
                                     blocks_per_cu, accumulate, accept_tau)
        _check(lib().amm_integrate(self.h, C.byref(rp), _stream(stream)), 'amm_integrate')

    def integrate_static(self, seed, n_per_graph, graph_begin=0, graph_end=None, counter0=0, sampler=0,
                         force_flag=0, blocks_per_cu=0, accumulate=0, accept_tau=None, stream=None):
        """amm_integrate with the library's static device scratch (no allocation)."""
        rp, _keep = self._run_params(seed, n_per_graph, graph_begin, graph_end, counter0, sampler, force_flag,
                                     blocks_per_cu, accumulate, accept_tau)
        _check(lib().amm_integrate_static(self.h, C.byref(rp), _stream(stream)), 'amm_integrate_static')

    def set_workspace(self, tensor=None):
        """Caller-owned device workspace (a torch tensor kept alive by the
        caller); None returns to the context's own buffers."""
        if tensor is None:
            _check(lib().amm_set_workspace(self.h, None, 0), 'amm_set_workspace')
        else:
            nbytes = tensor.numel() * tensor.element_size()
            _check(lib().amm_set_workspace(self.h, _ptr(tensor), nbytes), 'amm_set_workspace')
        self._workspace = tensor

    @staticmethod
    def workspace_bytes(chunks_per_group):
        return int(lib().amm_workspace_bytes(chunks_per_group))

    def integrate_batches(self, seed, n_per_graph, n_batches, graph_begin=0, graph_end=None, counter0=0,
                          sampler=0, force_flag=0, blocks_per_cu=0, accumulate=0, accept_tau=None, stream=None):
        rp, _keep = self._run_params(seed, n_per_graph, graph_begin, graph_end, counter0, sampler, force_flag,
                                     blocks_per_cu, accumulate, accept_tau)
        _check(lib().amm_integrate_batches(self.h, C.byref(rp), n_batches, _stream(stream)),
               'amm_integrate_batches')

    def integrate_adaptive(self, seed, n_pilot, budget_per_graph, n_rounds=2, floor_frac=0.25, cost=None,
                           graph_begin=0, graph_end=None, counter0=0, sampler=0, blocks_per_cu=0, accumulate=0,
                           accept_tau=None, stream=None):
        """Adaptive split of the samples over the graphs (amm_integrate_adaptive);
        returns the samples drawn per graph."""
        rp, _keep = self._run_params(seed, n_pilot, graph_begin, graph_end, counter0, sampler, 0,
                                     blocks_per_cu, accumulate, accept_tau)
        ng = rp.graph_end - rp.graph_begin
        done = (C.c_uint64 * ng)()
        cst = None if cost is None else (C.c_double * ng)(*cost)
        _check(lib().amm_integrate_adaptive(self.h, C.byref(rp), budget_per_graph, n_rounds, floor_frac, cst, done,
                                            _stream(stream)), 'amm_integrate_adaptive')
        return list(done)

    def autotune(self, seed, n_per_graph, graph_begin=0, graph_end=None, sampler=0, accept_tau=None, stream=None):
        rp, _keep = self._run_params(seed, n_per_graph, graph_begin, graph_end, 0, sampler, 0, 0, 0, accept_tau)
        b, o, ms = C.c_int(), C.c_int(), C.c_double()
        _check(lib().amm_autotune(self.h, C.byref(rp), C.byref(b), C.byref(o), C.byref(ms), _stream(stream)),
               'amm_autotune')
        return dict(blocks_per_cu=b.value, order_by_cost=o.value, ms=ms.value)

    def set_option(self, option, value):
        _check(lib().amm_set_option(self.h, option, int(value)), 'amm_set_option')

    def set_generated(self, on):
        """Use the build-time generated integrand code (True) or the table
        interpreter (False)."""
        _check(lib().amm_set_option(self.h, 1, int(bool(on))), 'amm_set_option')

    def accept_thresholds(self, n_run, graph_begin=0, graph_end=None):
        graph_end = self.n_se if graph_end is None else graph_end
        tau = (C.c_double * (graph_end - graph_begin))()
        _check(lib().amm_accept_thresholds(self.h, graph_begin, graph_end, n_run, tau), 'amm_accept_thresholds')
        return list(tau)

    def profile(self, enable):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        n, s = C.c_int64(), C.c_int64()
        _check(lib().amm_profile(self.h, int(enable), C.byref(a), C.byref(b), C.byref(c), C.byref(n), C.byref(s)),
               'amm_profile')
        return dict(ms_fp64=a.value, ms_dd=b.value, ms_reduce=c.value, launches=n.value, samples=s.value)

    # ----- learned sector sampler -----
    def pilot(self, seed, n_per_graph, graph_begin=0, graph_end=None, stream=None):
        graph_end = self.n_se if graph_end is None else graph_end
        _check(lib().amm_pilot(self.h, seed, n_per_graph, graph_begin, graph_end, _stream(stream)), 'amm_pilot')

    def pilot_table(self, g):
        """Graph g's pilot table W [2^M, M] (float64 holding exact integers)."""
        import numpy as np
        M = self.M
        W = np.empty((1 << M, M), dtype=np.float64)
        _check(lib().amm_pilot_table(self.h, g, W.ctypes.data_as(C.c_void_p), W.size), 'amm_pilot_table')
        return W

    def mlp_train(self, epochs, lr=1e-2, init_seed=0, stream=None):
        _check(lib().amm_mlp_train(self.h, epochs, lr, init_seed, _stream(stream)), 'amm_mlp_train')

    def mlp_params(self):
        import numpy as np
        cnt = C.c_size_t()
        _check(lib().amm_mlp_params(self.h, None, 0, C.byref(cnt)), 'amm_mlp_params')
        buf = np.empty(cnt.value, dtype=np.float32)
        _check(lib().amm_mlp_params(self.h, buf.ctypes.data_as(C.c_void_p), cnt.value, C.byref(cnt)),
               'amm_mlp_params')
        return buf

    def mlp_get_params(self):
        import numpy as np
        buf = np.empty(5313, dtype=np.float32)
        _check(lib().amm_mlp_get_params(self.h, buf.ctypes.data_as(C.c_void_p), buf.size), 'amm_mlp_get_params')
        return buf

    def mlp_adam(self, grad, t, lr, reset_moments=False, stream=None):
        """One Adam step of the context's parameters with a device FP32 gradient."""
        _check(lib().amm_mlp_adam(self.h, _ptr(grad), int(t), float(lr), int(bool(reset_moments)),
                                  _stream(stream)), 'amm_mlp_adam')

    def mlp_set_params(self, p):
        import numpy as np
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().amm_mlp_set_params(self.h, p.ctypes.data_as(C.c_void_p), p.size), 'amm_mlp_set_params')

    def mlp_features(self, g):
        import numpy as np
        n = C.c_size_t()
        _check(lib().amm_mlp_features(self.h, g, None, None, None, 0, C.byref(n)), 'amm_mlp_features')
        rows = np.empty((n.value, 16), dtype=np.float32)
        s = np.empty(n.value, dtype=np.int32)
        j = np.empty(n.value, dtype=np.int32)
        _check(lib().amm_mlp_features(self.h, g, rows.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p),
                                      j.ctypes.data_as(C.c_void_p), n.value, C.byref(n)), 'amm_mlp_features')
        return rows, s, j

    def mlp_loss_grad(self, rows, w, goff, stream=None):
        import torch
        n = rows.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=rows.device)
        grad = torch.empty(len(self.mlp_params()), dtype=torch.float32, device=rows.device)
        _check(lib().amm_mlp_loss_grad(self.h, _ptr(rows.contiguous()), _ptr(w.contiguous()), _ptr(goff.contiguous()),
                                       n, goff.shape[0] - 1, _ptr(loss), _ptr(grad), _stream(stream)),
               'amm_mlp_loss_grad')
        return loss, grad

    def set_sector_table(self, g, table):
        import numpy as np
        if table is None:
            _check(lib().amm_set_sector_table(self.h, g, None), 'amm_set_sector_table')
            return
        t = np.ascontiguousarray(table, dtype=np.float32)
        _check(lib().amm_set_sector_table(self.h, g, t.ctypes.data_as(C.c_void_p)), 'amm_set_sector_table')

    def read(self, g=-1, e=-1, cls=None):
        est = Estimate()
        k, m, mp = cls if cls is not None else (-1, -1, -1)
        _check(lib().amm_read(self.h, g, e, k, m, mp, C.byref(est)), 'amm_read')
        return est.as_dict()
