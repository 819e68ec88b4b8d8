"""Helpers of the GPU parity tests: render through the C ABI, compare with
the FP64 oracle.

Bar: RGB and alpha within 2/255 max abs on pixels the oracle does not flag
as fragile, and within 1e-3 mean abs over all pixels.  The same per-pixel
bound holds for the fp16 / bf16 deferred-MLP and fp16-feature paths, which
must also reach 45 dB PSNR over all pixels.
"""
import numpy as np

MAX_ABS = 2.0 / 255.0
MEAN_ABS = 1e-3
MIN_PSNR_DB = 45.0


def say(msg):
    print(msg, flush=True)


def gpu_render(torch, merf, scene, cams, stats=False, **kw):
    r = merf.Renderer(scene)
    try:
        st = torch.zeros(8, dtype=torch.int64, device="cuda") if stats else None
        out = r.render(cams, stats=st, **kw)
        torch.cuda.synchronize()
        res = out.cpu().numpy().astype(np.float64)
        return (res, st.cpu().numpy()) if stats else res
    finally:
        r.close()


def psnr(a, b):
    mse = float(np.mean((a[:, :3] - b[:, :3]) ** 2))
    return 10.0 * np.log10(1.0 / max(mse, 1e-30))


def check(gpu, ref, fragile, label, max_fragile=0.005, min_psnr=None):
    ok = fragile == 0
    err = np.abs(gpu - ref)
    mx = float(err[ok].max()) if ok.any() else 0.0
    mean = float(err.mean())
    p = psnr(gpu, ref)
    say(f"{label}: max|err| non-fragile {mx:.3e}  mean|err| {mean:.3e}  PSNR {p:.2f} dB  "
        f"fragile {float((~ok).mean()):.4%}  pixels {len(ref)}")
    assert np.all(np.isfinite(gpu))
    assert mx <= MAX_ABS, label
    assert mean <= MEAN_ABS, label
    if min_psnr is not None:
        assert p >= min_psnr, label
    if max_fragile is not None:
        assert float((~ok).mean()) < max_fragile, label
    return mx, mean


def rows_of(cams, rows_stride, row_offset):
    """Flat pixel indices of the rows the oracle renders with rows_stride /
    row_offset, camera after camera."""
    sel, off = [], 0
    for c in range(len(cams)):
        w, h = int(cams.size[c, 0]), int(cams.size[c, 1])
        rows = np.arange(row_offset, h, rows_stride)
        sel.append(off + (rows[:, None] * w + np.arange(w)[None, :]).reshape(-1))
        off += w * h
    return np.concatenate(sel)
