"""Runs the micro-benchmarks of libmcrt_micro.so and prints one JSON object:
random-gather rates per working-set size (global memory and LDS), FP64
atomic-add rates (device and workgroup scope; spread and hot-spot) and a
streaming-copy bandwidth.

    python -m paper_1512_02110_amd.micro [--quick]
"""
from __future__ import annotations

import ctypes as C
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(PKG, "libmcrt_micro.so")


def _lib():
    import torch  # noqa: F401  (torch's HIP runtime first, as in mcrt.load_library)
    L = C.CDLL(LIB)
    L.mc_micro_gather.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, C.c_void_p,
                                  C.c_void_p]
    L.mc_micro_atomic.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int, C.c_void_p]
    L.mc_micro_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint32, C.c_void_p]
    L.mc_micro_valu.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_int, C.c_void_p]
    L.mc_micro_gather_write.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                                        C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    L.mc_micro_gather_replay.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_uint32, C.c_uint32,
                                         C.c_uint32, C.c_void_p, C.c_void_p]
    for f in (L.mc_micro_gather, L.mc_micro_atomic, L.mc_micro_copy, L.mc_micro_valu, L.mc_micro_gather_write,
              L.mc_micro_gather_replay):
        f.restype = C.c_int
    return L


def gather_ceiling(s, n_photons, first_step=2000, n_steps=48, reps=20, seed=1000):
    """The render's connection-walk gathers against a replay of the same
    addresses: a capture render (FP32) stores what every lane of every
    wavefront loads on n_steps walk steps from first_step on; the replay
    kernel issues exactly those loads, with the same wavefronts per CU and no
    walk arithmetic, `reps` times over (the rate the vector-memory pipeline
    sustains on this address stream and working set).  The render's own rate
    comes from a plain render of the same photons: loads issued by its walks
    (64 per wavefront step, counting the lanes that read zero without an
    access: rays that have ended, empty runs) plus its free-flight loads, per
    second of kernel time."""
    import torch
    from paper_1512_02110_amd import mcrt as M
    L = _lib()
    dev = torch.device("cuda:0")
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    st_ = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    sc = s.replace(n_photons=n_photons)
    beta = M.beta_tensor(sc, "fp32")
    max_waves = n_cu * 4 * 4  # four 256-thread blocks per CU, as the render runs
    idx, steps, nw, cst = M.mc_capture_gathers(sc, beta, first_step, n_steps, max_waves, seed=seed)
    full = torch.nonzero(steps[:nw] >= first_step + n_steps).flatten()
    nf = (full.numel() // 4) * 4
    if nf < 4:
        raise RuntimeError("no wavefront took enough walk steps for the capture window")
    sel = idx[full[:nf]].contiguous()
    # the library's copy of beta: the voxels, then zeros (the zero word and the padding), then one per layer
    data = torch.cat([beta, torch.zeros(64 + sc.nz, dtype=torch.float32, device=dev)])
    sink = torch.zeros(nf * 64, dtype=torch.float32, device=dev)

    def run():
        rc = L.mc_micro_gather_replay(C.c_void_p(data.data_ptr()), data.numel(), beta.numel(),
                                      C.c_void_p(sel.data_ptr()), nf,
                                      n_steps, reps, C.c_void_p(sink.data_ptr()), st_)
        assert rc == 0, rc
    ms = _time(torch, run)
    replay = nf * 64 * n_steps * reps / (ms * 1e-3)
    M.mc_render(sc, beta, seed=seed + 1, n_photons=max(1, n_photons // 10), stats=False)
    _, rst = M.mc_render(sc, beta, seed=seed)
    t = rst.timing["transport_ms"] * 1e-3
    wave_steps = int(steps[:nw].sum().item())
    issued = (64.0 * wave_steps + rst["vox_free"]) / t
    useful = (rst["vox_conn"] + rst["vox_free"]) / t
    return {"working_set_bytes": 4 * sc.n_vox, "photons": n_photons, "waves_replayed": nf,
            "window_steps": [first_step, first_step + n_steps], "replay_reps": reps, "replay_ms": ms,
            "replay_gloads_per_s": replay / 1e9,
            "render_kernel_ms": rst.timing["transport_ms"],
            "render_issued_gloads_per_s": issued / 1e9, "frac_issued_of_replay": issued / replay,
            "render_algorithmic_gloads_per_s": useful / 1e9, "frac_algorithmic_of_replay": useful / replay,
            "lane_occupancy_of_walk_steps": cst["vox_conn"] / max(64.0 * wave_steps, 1.0)}


def _time(torch, fn, reps=3):
    fn()  # warm-up
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    return best


def main(quick=False):
    import torch
    L = _lib()
    dev = torch.device("cuda:0")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks = n_cu * 8
    out = {"n_cu": n_cu, "blocks": blocks, "gather": [], "atomic": []}
    sink = torch.zeros(blocks * 256, dtype=torch.float32, device=dev)
    loads = 128 if quick else 512
    for nbytes, lds in [(16 << 10, 1), (16 << 10, 0), (1 << 20, 0), (8 << 20, 0), (32 << 20, 0),
                        (256 << 20, 0)]:
        n = nbytes // 4
        data = torch.rand(n, dtype=torch.float32, device=dev)

        def run():
            rc = L.mc_micro_gather(C.c_void_p(data.data_ptr()), n, blocks, loads, lds,
                                   C.c_void_p(sink.data_ptr()), st)
            assert rc == 0, rc
        ms = _time(torch, run)
        total = blocks * 256 * loads
        out["gather"].append({"working_set_bytes": nbytes, "lds": bool(lds), "ms": ms,
                              "gloads_per_s": total / (ms / 1e3) / 1e9,
                              "useful_GBps": total * 4 / (ms / 1e3) / 1e9})
        print(f"[micro] gather {nbytes >> 10} KiB lds={lds}: {out['gather'][-1]['gloads_per_s']:.1f} G/s",
              flush=True)
    ops = 32 if quick else 128
    kinds = {0: "f64 device", 1: "f64 workgroup", 2: "f32 device", 3: "f32 device returning",
             4: "u64 device", 5: "f64 LDS", 6: "f32 LDS", 7: "f64 device, 8 lanes per 64-B line",
             8: "f64 device, 16 lanes per 128-B line"}
    for nbytes in (64, 1 << 20, 16 << 20, 64 << 20):
        n = nbytes // 8
        data = torch.zeros(n, dtype=torch.float64, device=dev)
        for kind, name in kinds.items():
            if kind >= 5 and nbytes != 64 and nbytes != (1 << 20):
                continue
            if kind == 8 and n < 16:
                continue
            nn = n if kind in (0, 1, 4, 7, 8) else (2 * n if kind in (2, 3) else min(n, 8192 if kind == 5 else 16384))

            def run():
                rc = L.mc_micro_atomic(C.c_void_p(data.data_ptr()), nn, blocks, ops, kind, st)
                assert rc == 0, rc
            ms = _time(torch, run)
            total = blocks * 256 * ops
            out["atomic"].append({"addresses": nn, "kind": name, "ms": ms,
                                  "gatomics_per_s": total / (ms / 1e3) / 1e9})
            print(f"[micro] atomic {name} n={nn}: {out['atomic'][-1]['gatomics_per_s']:.2f} G/s", flush=True)
    # dependent gathers (1 MiB working set) with a write every `period` loads
    data = torch.rand((1 << 20) // 4, dtype=torch.float32, device=dev)
    iters = 256 if quick else 1024
    out["gather_write"] = []
    for n_out_bytes in (1 << 20, 1 << 30):
        n_out = n_out_bytes // 32
        dst = torch.zeros(n_out_bytes // 4, dtype=torch.float32, device=dev)
        for kind, name in ((0, "none"), (1, "store 4 B"), (2, "f64 atomic"), (3, "store 32 B")):
            for period in ((1,) if kind == 0 else (32, 8, 2)):
                def run_gw():
                    rc = L.mc_micro_gather_write(C.c_void_p(data.data_ptr()), data.numel(), blocks, iters, period,
                                                 kind, C.c_void_p(dst.data_ptr()), n_out,
                                                 C.c_void_p(sink.data_ptr()), st)
                    assert rc == 0, rc
                ms = _time(torch, run_gw)
                loads = blocks * 256 * iters
                rec = {"write": name, "period": period, "out_bytes": n_out_bytes, "ms": ms,
                       "ns_per_load_per_lane": ms * 1e6 / iters, "gloads_per_s": loads / (ms / 1e3) / 1e9}
                out["gather_write"].append(rec)
                print(f"[micro] gather+write {name} every {period} (out {n_out_bytes >> 20} MiB): "
                      f"{rec['gloads_per_s']:.1f} G loads/s", flush=True)
        del dst
    # VALU issue: wave64 FMA instructions per CU and per ns (x 1e9 / clock for per cycle)
    out["valu"] = []
    vsink = torch.zeros(blocks * 256, dtype=torch.float64, device=dev)
    v_iters = 256 if quick else 2048
    for fp64 in (0, 1):
        def run_v():
            rc = L.mc_micro_valu(C.c_void_p(vsink.data_ptr()), blocks, v_iters, fp64, st)
            assert rc == 0, rc
        ms = _time(torch, run_v)
        instr = blocks * 4 * v_iters * 64  # wave instructions (4 wavefronts per block)
        rec = {"fp64": bool(fp64), "ms": ms, "wave_instr_per_cu_per_ns": instr / n_cu / (ms * 1e6),
               "lane_flops_per_s": 2 * instr * 64 / (ms / 1e3)}
        out["valu"].append(rec)
        print(f"[micro] VALU {'f64' if fp64 else 'f32'} FMA: {rec['wave_instr_per_cu_per_ns']:.3f} wave instr per CU "
              f"per ns, {rec['lane_flops_per_s'] / 1e12:.1f} TFLOP/s", flush=True)
    del vsink
    nb = 1 << 30
    src = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)

    def run_copy():
        rc = L.mc_micro_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb // 16, n_cu * 16, st)
        assert rc == 0, rc
    ms = _time(torch, run_copy)
    out["copy"] = {"bytes_each_way": nb, "ms": ms, "GBps": 2 * nb / (ms / 1e3) / 1e9}
    print(f"[micro] copy: {out['copy']['GBps']:.0f} GB/s", flush=True)
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main(quick="--quick" in sys.argv)
