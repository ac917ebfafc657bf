"""MI355X (gfx950) implementation of the JDE tracker's hot path.

The HIP library (csrc/, built into libjde.so) runs the joint detection and
embedding forward, decode, NMS, embedding normalisation and the gated cost
matrix; `jde` is its Python binding (argument marshalling only).
"""

from .jde import (JDE, jde_create, jde_destroy, jde_layer_info, jde_cost_matrix,  # noqa: F401
                  jde_track_emb_update, jde_nms_noalloc, jde_kf_initiate, jde_kf_initiate_n, jde_kf_predict,
                  jde_kf_update, jde_kf_update_n, jde_assign, jde_box_to_z,
                  jde_kf_predict_dev, jde_kf_update_dev, jde_assign_dev, jde_ingest,
                  jde_cost_matrix_batch_fused, jde_iou_cost_batch)
