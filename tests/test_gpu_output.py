"""Writing phase on the GPU (Section 3.2, writing): the SED reduced on the
device equals the sum of the pixels (and of the oracle's pixels in FP64
validation mode); the FITS cube and text SED written from a result hold the
result's own images and SED."""
import numpy as np
import pytest

import fitsread
import oracle
from paper_1705_04702_amd import mcrt, scenes

pytestmark = pytest.mark.gpu


def test_sed_and_files_fp64(tmp_path):
    sc = scenes.disk(n=(16, 16, 8), n_lambda=3, npix=16)
    # a non-square frame, so x and y cannot be swapped unnoticed
    sc.instruments = [scenes.Instrument(30.0, 20.0, 1.0e4, (40.0, 30.0), (24, 16)), sc.instruments[0]]
    N = 400
    o = oracle.run(sc, N, seed=4)
    ctx = mcrt.Context(0)
    sim = mcrt.Sim(ctx, sc, mcrt.FP64_VALIDATE)
    res = sim.run(N, seed=4)
    for j, img in enumerate(res.images()):
        sed = res.sed(j)
        assert np.allclose(sed, img.sum(axis=(1, 2)), rtol=1e-12, atol=0)
        osed = o["images"][j].sum(axis=(1, 2))
        assert np.allclose(sed, osed, rtol=1e-9, atol=0)
        fp, sp = tmp_path / f"i{j}.fits", tmp_path / f"i{j}.sed"
        res.write(j, fits_path=fp, sed_path=sp)
        hdus = fitsread.read(fp)
        assert np.array_equal(hdus[0][2], img)
        assert np.array_equal(hdus[1][2], np.asarray(sc.lambdas, dtype=np.float64))
        back = np.loadtxt(sp)
        assert np.array_equal(back[:, 1], sed) and np.array_equal(back[:, 0], np.asarray(sc.lambdas))
    res.close()
    sim.close()
    ctx.close()


def test_sed_fp32_matches_pixels():
    sc = scenes.disk(n=(32, 32, 16), n_lambda=4, npix=64)
    ctx = mcrt.Context(0)
    sim = mcrt.Sim(ctx, sc, mcrt.FP32)
    res = sim.run(2000, seed=1)
    for j, img in enumerate(res.images()):
        assert np.allclose(res.sed(j), img.sum(axis=(1, 2)), rtol=1e-12, atol=0)
    with pytest.raises(mcrt.MCRTError):
        res.sed(len(sc.instruments))
    res.close()
    sim.close()
    ctx.close()
