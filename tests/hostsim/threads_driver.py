"""Concurrent calls into the host orchestration (CPU double of the kernels), for
the ThreadSanitizer run of tests/test_hostsim_threads.py.  Several threads call
negf_rgf_lesser_greater on their own problems, outputs and workspaces while
another creates, executes and destroys plans; every result must equal the same
call made alone.  Exit status 0 when all agree (a race report ends the process
earlier with the sanitizer's exit code)."""
import ctypes as C
import dataclasses
import os
import sys
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as w  # noqa: E402
from paper_2602_03438_amd import binding as nb  # noqa: E402

P = C.POINTER
vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
L = C.CDLL(sys.argv[1])
L.negf_workspace_bytes.argtypes = [i32, P(nb.negf_problem), i32, i32, P(nb.negf_options)]
L.negf_workspace_bytes.restype = sz
L.negf_rgf_lesser_greater.argtypes = [P(nb.negf_problem), i32, i32, P(nb.negf_options), vp, vp, vp, vp, vp, vp, vp,
                                      vp, vp, sz, vp]
L.negf_plan_create.argtypes = [P(nb.negf_problem), i32, i32, P(nb.negf_options), vp, i32, i32, P(vp)]
L.negf_plan_workspace_bytes.argtypes = [vp]
L.negf_plan_workspace_bytes.restype = sz
L.negf_plan_execute.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
L.negf_plan_destroy.argtypes = [vp]

KEYS = ("GRd", "GRu", "GRl", "GLd", "GLu", "GGd", "GGu")


class Job:
    def __init__(self, dev, E, sc_stride=0, batch=0):
        self.keep = [None if a is None else np.ascontiguousarray(a)
                     for a in (dev.H_diag, dev.H_upper, dev.S_diag, dev.S_upper, dev.sig_r, dev.sig_l, dev.sig_g)]
        self.E = np.ascontiguousarray(E, dtype=np.float64)
        ptr = lambda a: None if a is None else a.ctypes.data
        d = nb.negf_device(dev.nb, dev.b, *[ptr(a) for a in self.keep])
        self.arr = (nb.negf_problem * 1)(nb.negf_problem(d, self.E.size, self.E.ctypes.data, 1e-6, 0.1, -0.1, 0.025,
                                                          sc_stride))
        self.opts = nb.make_options(batch=batch)
        n = self.E.size
        self.nd, self.nu = n * dev.nb * dev.b * dev.b, n * (dev.nb - 1) * dev.b * dev.b
        self.ws = np.zeros(L.negf_workspace_bytes(nb.OP_LESSER_GREATER, self.arr, 1, 0, C.byref(self.opts)) + 256,
                           dtype=np.uint8)

    def outputs(self):
        return {k: np.zeros(self.nd if k.endswith("d") else self.nu, dtype=np.complex128) for k in KEYS}

    def run(self):
        out = self.outputs()
        info = np.zeros(self.E.size, dtype=np.int32)
        ws = np.zeros_like(self.ws)
        code = L.negf_rgf_lesser_greater(self.arr, 1, 0, C.byref(self.opts), *[out[k].ctypes.data for k in KEYS],
                                         info.ctypes.data, ws.ctypes.data, ws.size, None)
        assert code == 0, code
        return out, info

    def run_plan(self):
        h = vp()
        assert L.negf_plan_create(self.arr, 1, 0, C.byref(self.opts), None, 0, 2, C.byref(h)) == 0
        out = self.outputs()
        info = np.zeros(self.E.size, dtype=np.int32)
        ws = np.zeros(L.negf_plan_workspace_bytes(h) + 256, dtype=np.uint8)
        code = L.negf_plan_execute(h, 1, *[out[k].ctypes.data for k in KEYS], info.ctypes.data, None, ws.ctypes.data,
                                   ws.size, None)
        L.negf_plan_destroy(h)
        assert code == 0, code
        return out, info


def main():
    base = w.random_device(5, 16, 3, overlap=0.05)
    scat = w.scattering_self_energies(w.random_device(5, 16, 4), 5, norm=0.05)
    E = np.linspace(-1.0, 1.0, 5)
    per_e = [w.scattering_self_energies(dataclasses.replace(base), 40 + e, norm=0.05) for e in range(E.size)]
    dyn = dataclasses.replace(base, sig_r=np.stack([d.sig_r for d in per_e]), sig_l=np.stack([d.sig_l for d in per_e]),
                              sig_g=np.stack([d.sig_g for d in per_e]))
    jobs = [Job(base, E), Job(scat, E[:3], batch=2), Job(dyn, E, sc_stride=5 * 16 * 16, batch=2),
            Job(w.folded_chain_device(6, 16), np.linspace(-1.5, 1.5, 4))]
    ref = [j.run() for j in jobs]
    ref_plan = jobs[2].run_plan()
    errors = []
    reps = 3
    # every repetition starts in all threads at once, so that the calls overlap in time (a race
    # is reported only between accesses that no lock, GIL hand-over included, orders)
    start = threading.Barrier(len(jobs) + 1)

    def worker(k, reps):
        for _ in range(reps):
            start.wait()
            out, info = jobs[k].run()
            if not all(np.array_equal(out[x], ref[k][0][x]) for x in KEYS) or not np.array_equal(info, ref[k][1]):
                errors.append(k)

    def planner(reps):
        for _ in range(reps):
            start.wait()
            out, info = jobs[2].run_plan()
            if not all(np.array_equal(out[x], ref_plan[0][x]) for x in KEYS):
                errors.append("plan")

    threads = [threading.Thread(target=worker, args=(k, reps)) for k in range(len(jobs))]
    threads.append(threading.Thread(target=planner, args=(reps,)))
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        print("results differ from the calls made alone:", errors)
        return 1
    print(f"{len(threads)} threads: every result equals the call made alone")
    return 0


if __name__ == "__main__":
    sys.exit(main())
