"""The whole two-stage standard eigensolver on the CPU (Sec. 2 of the paper):

    A --stage1--> B --stage2--> (d, e, hh, tau) --tridiag--> (lambda, Z^)
      Z_band = BT1(hh, tau, Z^)         (tridiagonal -> band, the hot path)
      Z      = BT2(panels, Z_band)      (band -> full)
"""
from . import bt, stage1, stage2, tridiag


def solve_two_stage(A, nbw, nev=None, seed=12345, blocked=True, nthreads=0):
    n = A.shape[0]
    nev = n if nev is None else nev
    B, panels = stage1.full_to_band(A, nbw, blocked=blocked)
    d, e, hh, tau = stage2.band_to_tridiag(B, nbw)
    lam, Zt = tridiag.eigh_tridiag(d, e, nev, seed=seed, nthreads=nthreads)
    Zb = bt.bt_tridiag_to_band(hh, tau, Zt.astype(hh.dtype), n, nbw, nthreads)
    Z = bt.bt_band_to_full(panels, Zb, nbw)
    return dict(B=B, panels=panels, d=d, e=e, hh=hh, tau=tau, lam=lam, Zt=Zt,
                Zb=Zb, Z=Z)
