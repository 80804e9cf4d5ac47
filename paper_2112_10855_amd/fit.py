"""Time to a target fit: single-tensor CP-ALS-QR sweeps with the direct
relative error ||X - [[lambda; A]]|| / ||X|| after every sweep (the efficient
form cannot resolve errors near 1e-6 from FP32 data)."""

import torch

from . import cpqr as C


def time_to_fit(X, init, prec=C.PREC_F32, target=1e-6, max_sweeps=200, chunk=5):
    """Sweeps of the single-tensor CP-ALS-QR (direct error after every sweep)
    until relerr <= target.  Returns (sweeps or None, GPU seconds, final
    relerr); the time counts the sweeps run, error included."""
    st = C.AlsState(X, init, prec=prec, error_mode=C.ERROR_DIRECT)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st.init()
    done, hit, last = 0, None, float("nan")
    rel = torch.empty(chunk, dtype=torch.float64, device=X.device)
    while done < max_sweeps and hit is None:
        st.sweep(chunk, rel)
        r = rel.cpu().numpy()
        for i, v in enumerate(r):
            if v <= target:
                hit = done + i + 1
                break
        done += chunk
        last = float(r[-1])
    e1.record()
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    if hit is not None:  # drop the sweeps past the hit from the time
        secs *= hit / done
    return hit, secs, last
