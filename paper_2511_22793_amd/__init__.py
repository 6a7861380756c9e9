"""MI355X-native hemispherical RF Gaussian-splatting renderer (GSpaRC's hot
path): projection onto a receiver-centred equirectangular grid, tile binning
with a (tile, depth) radix sort, and front-to-back compositing, as hand-written
HIP kernels for gfx950 behind the C ABI of include/gsparc.h."""
from .render import (Grid, Params, Workspace, backward, backward_l2, blend, blend_loss, forward, layout,  # noqa: F401
                     live, loss_l1_ssim, loss_spectrum, loss_stats, prepare, spatial_mean, train_geometry,
                     train_pass, TrainScratch)
from .autograd import GSRender, render  # noqa: F401
from .confidence import confidence_loss  # noqa: F401
from .emission import emission_backward, emission_forward  # noqa: F401
