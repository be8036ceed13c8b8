"""Drive the host code from several threads at once, built against the CPU
stand-in of the HIP runtime (fake_hip.cpp) with ThreadSanitizer, the way
serving uses it (one context, batch and thread per size class: admit, step,
poll, retire, then the fidelity and energy of each finished solve) beside
whole batched rounds of the T_s search on a third thread.  Some Hamiltonians,
and in one thread the batch with its context, are left in reference cycles,
so their finalizers run on whatever thread the collector happens to run on
and in no fixed order.  Prints "threads done" and exits 0 when every thread
finished without a library error.

Usage: python drive_threads.py <path of the instrumented libaqc.so>"""
import ctypes as C
import gc
import os
import sys
import threading
import types

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import torch

from paper_1311_3938_amd import _lib as L

L.LIB_PATH = sys.argv[1]
from paper_1311_3938_amd import engine, instances as I, tsearch  # noqa: E402
from paper_1311_3938_amd._lib import check, lib  # noqa: E402


class CpuCtx(engine.Context):
    """A context whose "device" tensors are host tensors."""

    def __init__(self):
        self.device = torch.device("cpu")
        self.stream = types.SimpleNamespace(cuda_stream=0)
        h = C.c_void_p()
        check(lib().aqc_create(0, C.c_void_p(0), C.byref(h)))
        self._h = h


errors = []


def serve_like(tag, n_lo, n_hi, rounds, resident, leave_to_collector):
    try:
        ctx = CpuCtx()
        b = engine.Batch(ctx, torch.complex64, capacity=4, graph=True, resident_max_n=resident)
        live = {}
        k = 0
        for r in range(rounds):
            while len(live) < 4:
                inst = I.workload_serving_request(1000 * tag + k, n_lo=n_lo, n_hi=n_hi)
                k += 1
                ham = engine.Hamiltonian(ctx, inst)
                ham.spectral_bounds(0.0, inst.path["T"])
                psi = torch.zeros(1 << inst.n, dtype=torch.complex64)
                psi[0] = 1
                live[b.admit(ham, psi, 0.0, 1.0, 3 + (k % 7), 0.5)] = ham
            b.step(4)
            for s in b.poll():
                psi, _ = b.retire(s)
                ham = live.pop(s)
                engine.ground_mass(ctx, ham, 1.0, psi)
                engine.energy(ctx, ham, 1.0, psi)
                if k % 3 == 0:
                    cyc = [ham]
                    cyc.append(cyc)      # freed by its finalizer, on any thread
                else:
                    ham.free()
            if r % 5 == 0:
                gc.collect()
        if leave_to_collector:
            cyc = [b, ctx]
            cyc.append(cyc)              # the batch and its context, in no fixed order
        else:
            b.close()
            ctx.close()
    except Exception as e:  # noqa: BLE001
        errors.append((tag, repr(e)))


def ts_rounds():
    try:
        ctx = CpuCtx()
        for _ in range(3):
            insts = [I.workload_usa(8, k, "xy") for k in range(3)]
            tsearch.search_rounds(ctx, insts, [I.plus_state(8)] * 3, tsearch.energies, T_max=16.0,
                                  plan=lambda ham, T: (int(6 + T), 0.5))
            gc.collect()
        ctx.close()
    except Exception as e:  # noqa: BLE001
        errors.append(("ts", repr(e)))


def main():
    ths = [threading.Thread(target=serve_like, args=(1, 8, 11, 40, 0, True)),
           threading.Thread(target=serve_like, args=(2, 12, 14, 30, 12, False)),
           threading.Thread(target=ts_rounds)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    gc.collect()
    assert not errors, errors
    print("threads done", flush=True)


if __name__ == "__main__":
    main()
