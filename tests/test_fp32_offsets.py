"""Why the device stores every state as an FP32 offset from the resting state.

Near rest a Hodgkin-Huxley node changes by less per step than half an ulp of
its FP32 value (the gate h near 0.6 has an ulp of 6e-8), so an FP32 state stored
as is drops those increments, and the slow return to rest stalls; stored as
an offset from rest the same increments land on values near zero and
survive.  The test takes the FP64 oracle's per-step increments of a node
relaxing from a 0.05 mV depolarization (3000 Heun steps of 1e-3 ms) and
accumulates them in FP32 both ways: absolute storage ends 100x and more
further from the FP64 trajectory than offsets in every state (about 4e-3 mV
against 7e-8 mV for V_m after 3 ms).
"""
import numpy as np

from oracle import oracle as O


def test_fp32_offsets_keep_the_increments_that_absolute_storage_drops():
    rest = O.rest_state()
    y = rest.copy()[:, None]
    y[0] += 0.05
    cfg = O.Config(dt_0D=1e-3)
    ys = [y[:, 0].copy()]
    for _ in range(3000):
        y = O.reaction(cfg, y, 1e-3)
        ys.append(y[:, 0].copy())
    ys = np.array(ys)
    inc = np.diff(ys, axis=0)
    # h (near 0.6) and n (near 0.32) change by less than half an ulp of
    # their FP32 values in most of the last thousand steps
    half_ulp = 0.5 * np.abs(np.spacing(rest[2:].astype(np.float32))).astype(np.float64)
    assert np.all(np.mean(np.abs(inc[-1000:, 2:]) < half_ulp, axis=0) > 0.5)
    absolute = ys[0].astype(np.float32)
    offset = (ys[0] - rest).astype(np.float32)
    for d in inc:
        d32 = d.astype(np.float32)
        absolute = np.float32(absolute + d32)
        offset = np.float32(offset + d32)
    final = ys[-1]
    err_abs = np.abs(absolute.astype(np.float64) - final)
    err_off = np.abs(offset.astype(np.float64) + rest - final)
    assert np.all(err_abs > 100.0 * err_off)
    assert err_abs[0] > 1e-3 and err_off[0] < 1e-6
