"""The device code generators reproduce the host generators bit for bit."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,bits", [("uniform", 64), ("uniform", 256), ("clustered", 128),
                                       ("clustered", 256)])
def test_device_generator_matches_host(kind, bits):
    n, first = 5000, 123_457
    seed = 4 if kind == "clustered" else 9
    dev = datagen.codes_device(kind, n, bits, seed, first_row=first, chunk=1777)
    host = (datagen.clustered_codes if kind == "clustered" else datagen.uniform_codes)(
        n, bits, seed, first_row=first)
    assert np.array_equal(dev.cpu().numpy().view(np.uint64), host)
